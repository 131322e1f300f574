"""Seeded synthetic inputs for the space-time Schroedinger solve.

This module is shared by the tests, the benchmark and the smoke check.  It
holds only input generation -- workload sizes, temporal meshes, seeded random
right-hand sides, targets and directions, and the load vectors of separable
manufactured solutions -- and none of the solver's arithmetic.  It imports
neither the oracle nor the GPU package.

Workloads (all on the unit square with the right-diagonal triangulation of
n x n cells, P1 in space, n_x = (n-1)^2 interior dofs):

  c0  n=16,  T=1, 16 uniform time elements, P1 in time  (manufactured, omega = pi)
  c1  n=128, T=1, 128 elements P1, manufactured + 4 random complex rhs
  c2  n=256, T=2, 256 elements P1, manufactured with omega = 4 pi
  c3  n=128, T=1, 128 elements P1, tracking functional with 8 random targets
  c4  n=512, T=1, 256 elements P2 in time (512 time dofs)

The manufactured solution is psi = sin(pi x) sin(pi y) (1 + t^2) e^{i omega t}
with psi_0 = sin(pi x) sin(pi y).  Subtracting psi_0 (constant in time) gives
psi_hat = psi - psi_0 with zero initial value, which solves the same equation
with f_hat = f - 2 pi^2 sin(pi x) sin(pi y).  Both f and f_hat are separable
in space and time, so their load vectors are outer products of a temporal and
a spatial integral.
"""
from dataclasses import dataclass

import numpy as np

PI = np.pi


@dataclass(frozen=True)
class Workload:
    name: str
    n: int            # cells per side
    T: float
    N_t: int          # time elements
    p_t: int          # temporal degree
    omega: float
    n_random: int = 0

    @property
    def n_x(self):
        return (self.n - 1) ** 2

    @property
    def n_t(self):
        return self.p_t * self.N_t

    @property
    def dofs(self):
        return self.n_x * self.n_t


WORKLOADS = {
    "c0": Workload("c0", 16, 1.0, 16, 1, PI),
    "c1": Workload("c1", 128, 1.0, 128, 1, PI, n_random=4),
    "c2": Workload("c2", 256, 2.0, 256, 1, 4 * PI),
    "c3": Workload("c3", 128, 1.0, 128, 1, PI),
    "c4": Workload("c4", 512, 1.0, 256, 2, PI),
}


def uniform_nodes(T, N):
    return T * np.arange(N + 1, dtype=np.float64) / N


def graded_nodes(T, N0, q, levels=0):
    t = T * (np.arange(N0 + 1, dtype=np.float64) / N0) ** q
    for _ in range(levels):
        out = np.empty(2 * len(t) - 1)
        out[0::2] = t
        out[1::2] = 0.5 * (t[:-1] + t[1:])
        t = out
    return t


def random_rhs(seed, n_t, n_x, nrhs=None):
    """Entries i.i.d. N(0,1) + i N(0,1) from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = (n_t, n_x) if nrhs is None else (nrhs, n_t, n_x)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- load vectors
def _gl(m):
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1), 0.5 * w


def _time_basis(p, xi):
    if p == 1:
        return np.stack([1 - xi, xi])
    return np.stack([2 * (xi - 0.5) * (xi - 1), -4 * xi * (xi - 1), 2 * xi * (xi - 0.5)])


def temporal_moments(g, nodes, p, m=8):
    """a[l] = int_0^T g(t) varphi_l(t) dt for every temporal dof l except t_0
    (dofs in position order), by Gauss-Legendre on each element."""
    nodes = np.asarray(nodes, dtype=np.float64)
    N = nodes.size - 1
    xi, w = _gl(m)
    ph = _time_basis(p, xi)
    a = np.zeros(p * N + 1, dtype=np.complex128)
    for e in range(N):
        h = nodes[e + 1] - nodes[e]
        gv = g(nodes[e] + h * xi)
        a[p * e: p * e + p + 1] += h * (ph * (w * gv)).sum(axis=1)
    return a[1:]


def spatial_moments(s, n, m=6):
    """b[k] = int_Omega s(x, y) phi_k(x, y) for the interior P1 hat functions on
    the right-diagonal mesh, by a collapsed Gauss rule on every triangle."""
    h = 1.0 / n
    u, wu = _gl(m)
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    rx = U.ravel()
    ry = (V * (1 - U)).ravel()
    rw = (WU * WV * (1 - U)).ravel() * h * h      # |det J| = h^2 for both triangle kinds
    b = np.zeros((n + 1, n + 1), dtype=np.complex128)   # indexed [j, i]
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    # lower triangle: (i,j), (i+1,j), (i+1,j+1): x = x_i + h (rx + ry), y = y_j + h ry
    # upper triangle: (i,j), (i+1,j+1), (i,j+1): x = x_i + h rx,        y = y_j + h (rx + ry)
    for kind in (0, 1):
        if kind == 0:
            X = (ci[:, None] + rx[None] + ry[None]) * h
            Y = (cj[:, None] + ry[None]) * h
            verts = [(0, 0), (1, 0), (1, 1)]
        else:
            X = (ci[:, None] + rx[None]) * h
            Y = (cj[:, None] + rx[None] + ry[None]) * h
            verts = [(0, 0), (1, 1), (0, 1)]
        sv = s(X, Y) * rw[None]
        lam = [1 - rx - ry, rx, ry]
        for (di, dj), la in zip(verts, lam):
            np.add.at(b, (cj + dj, ci + di), sv @ la)
    return b[1:n, 1:n].ravel()


def manufactured_rhs(wl: Workload, nodes=None, homogenised=True):
    """Load vector (n_t x n_x, complex128) of the manufactured solution of the
    workload.  homogenised=True gives the zero-initial-value problem for
    psi_hat = psi - psi_0 (f_hat = f - 2 pi^2 s); otherwise the load of f."""
    if nodes is None:
        nodes = uniform_nodes(wl.T, wl.N_t)
    w = wl.omega
    shift = 2 * PI ** 2 if homogenised else 0.0

    def g(t):
        return np.exp(1j * w * t) * (2 * PI ** 2 * (1 + t ** 2) - w * (1 + t ** 2) + 2j * t)

    a = temporal_moments(g, nodes, wl.p_t)
    b = spatial_moments(lambda x, y: np.sin(PI * x) * np.sin(PI * y), wl.n)
    F = np.outer(a, b)
    if shift:
        a0 = temporal_moments(lambda t: np.ones_like(t) + 0j, nodes, wl.p_t)
        F -= shift * np.outer(a0, b)
    return F


def manufactured_psi_hat(wl: Workload, nodes=None):
    """Nodal values of psi_hat = psi - psi_0 at the temporal dofs t_1.. and the
    interior vertices (n_t x n_x)."""
    if nodes is None:
        nodes = uniform_nodes(wl.T, wl.N_t)
    nodes = np.asarray(nodes)
    if wl.p_t == 1:
        tp = nodes[1:]
    else:
        tp = np.empty(2 * (nodes.size - 1))
        tp[0::2] = 0.5 * (nodes[:-1] + nodes[1:])
        tp[1::2] = nodes[1:]
    h = 1.0 / wl.n
    xs = np.arange(1, wl.n) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    s = (np.sin(PI * X) * np.sin(PI * Y)).ravel()
    tt = ((1 + tp ** 2) * np.exp(1j * wl.omega * tp) - 1.0)
    return np.outer(tt, s)


def psi0_nodal(n):
    """Nodal values of psi_0 = sin(pi x) sin(pi y) at the interior vertices."""
    xs = np.arange(1, n) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    return (np.sin(PI * X) * np.sin(PI * Y)).ravel().astype(np.complex128)


# ---------------------------------------------------------- tracking targets
def smooth_targets(n, nodes_full, seeds, n_modes=6, kmax=8, omega_max=10.0):
    """Targets psi_target(x, y, t) = sum of n_modes random modes
    a sin(k pi x) sin(l pi y) e^{i omega t}, k, l ~ U{1..kmax},
    omega ~ U[0, omega_max], a ~ N(0,1) + i N(0,1); interpolated at every
    temporal node (t_0 included) and interior vertex.  One target per seed:
    returns (len(seeds), len(nodes_full), n_x)."""
    xs = np.arange(1, n) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    X = X.ravel()
    Y = Y.ravel()
    t = np.asarray(nodes_full, dtype=np.float64)
    out = np.zeros((len(seeds), t.size, X.size), dtype=np.complex128)
    for i, sd in enumerate(seeds):
        rng = np.random.default_rng(sd)
        for _ in range(n_modes):
            k, l = rng.integers(1, kmax + 1, size=2)
            om = rng.uniform(0.0, omega_max)
            a = rng.standard_normal() + 1j * rng.standard_normal()
            out[i] += a * np.outer(np.exp(1j * om * t), np.sin(k * PI * X) * np.sin(l * PI * Y))
    return out


def unit_directions(seeds, shape):
    """Complex normal directions with unit 2-norm, one per seed."""
    out = []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        d = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        out.append(d / np.linalg.norm(d))
    return out


def shifts_upper_half_plane(seed, count, re_max, im_min, im_max):
    """Seeded complex shifts with Re in [-re_max, re_max] and Im in
    [im_min, im_max] (log-uniform), for batched shifted spatial solves."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-re_max, re_max, count)
    im = np.exp(rng.uniform(np.log(im_min), np.log(im_max), count))
    return re + 1j * im
