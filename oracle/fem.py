"""Meshes, element loops and global matrices of the space-time Galerkin method
(test infrastructure only; see the package docstring).

Everything is assembled from element contributions computed by quadrature,
never from closed-form stencils, so that the closed forms can serve as
independent checks in the tests.

Spatial discretisation (Sec. 3, eq. (matrix_x)): continuous P1 on the unit
square, triangulated by n x n squares each cut by the diagonal from its
lower-left to its upper-right corner.  Vertex (i, j) sits at (i/n, j/n);
interior vertices are the unknowns, numbered lexicographically with x fastest:
k = (j-1)(n-1) + (i-1).

Temporal discretisation (Sec. 3, eq. (matrix_t)): continuous Lagrange Pp,
p in {1, 2}, on arbitrary nodes 0 = t_0 < ... < t_N = T.  Degrees of freedom
are ordered by position (t_0, [t_1/2,] t_1, ...); the dof at t_0 is removed
(zero initial value of the homogenised unknown, Sec. 3), leaving n_t = p*N.
Matrix rows are test functions, columns trial functions:
M_t[k, j] = int phi_j phi_k,  B_t[k, j] = int phi_j' phi_k.
"""
import numpy as np
import scipy.sparse as sp

from .quadrature import gauss_legendre, triangle_rule


# --------------------------------------------------------------------------
# time
# --------------------------------------------------------------------------
def time_nodes_uniform(T, N):
    """Uniform temporal mesh t_l = T l / N (Sec. 4, eq. (Mesh_t))."""
    return T * np.arange(N + 1, dtype=np.float64) / N


def time_nodes_graded(T, N0, q, levels=0):
    """Graded temporal mesh t_l = T (l/N0)^q, then `levels` uniform bisections
    of every element (Sec. 4, graded mesh of Table 3)."""
    t = T * (np.arange(N0 + 1, dtype=np.float64) / N0) ** q
    for _ in range(levels):
        mid = 0.5 * (t[:-1] + t[1:])
        out = np.empty(2 * len(t) - 1)
        out[0::2] = t
        out[1::2] = mid
        t = out
    return t


def lagrange_1d(p, xi):
    """Values and derivatives of the degree-p Lagrange basis on [0,1] with
    equispaced nodes a/p, at points xi.  Returns (phi, dphi), each (p+1, len(xi))."""
    xi = np.asarray(xi, dtype=np.float64)
    nodes = np.arange(p + 1) / p
    phi = np.ones((p + 1, xi.size))
    dphi = np.zeros((p + 1, xi.size))
    for a in range(p + 1):
        others = [b for b in range(p + 1) if b != a]
        for b in others:
            phi[a] *= (xi - nodes[b]) / (nodes[a] - nodes[b])
        for c in others:  # product rule
            term = np.full(xi.size, 1.0 / (nodes[a] - nodes[c]))
            for b in others:
                if b != c:
                    term = term * (xi - nodes[b]) / (nodes[a] - nodes[b])
            dphi[a] += term
    return phi, dphi


def assemble_time_full(nodes, p):
    """Full temporal mass and derivative matrices including the t_0 dof.

    Returns (M_full, B_full) of size (pN+1)^2 with B_full[k, j] = int phi_j' phi_k."""
    nodes = np.asarray(nodes, dtype=np.float64)
    N = nodes.size - 1
    nd = p * N + 1
    xq, wq = gauss_legendre(p + 2)
    phi, dphi = lagrange_1d(p, xq)
    Mf = np.zeros((nd, nd))
    Bf = np.zeros((nd, nd))
    for e in range(N):
        h = nodes[e + 1] - nodes[e]
        idx = p * e + np.arange(p + 1)
        # mass: h * int_0^1 phi_a phi_b ; derivative: int_0^1 phi_b' phi_a (h cancels)
        Me = h * (phi * wq) @ phi.T
        Be = (phi * wq) @ dphi.T          # Be[a, b] = sum_q w phi_a dphi_b
        Mf[np.ix_(idx, idx)] += Me
        Bf[np.ix_(idx, idx)] += Be
    return Mf, Bf


def assemble_time(nodes, p):
    """Temporal matrices with the t_0 dof removed, plus the couplings of the
    remaining test functions to the removed dof (needed to lift psi_0).

    Returns M_t, B_t (n_t x n_t), m_col0, b_col0 (n_t)."""
    Mf, Bf = assemble_time_full(nodes, p)
    return Mf[1:, 1:].copy(), Bf[1:, 1:].copy(), Mf[1:, 0].copy(), Bf[1:, 0].copy()


def time_dof_points(nodes, p):
    """Positions of the temporal dofs (t_0 included) in position order."""
    nodes = np.asarray(nodes, dtype=np.float64)
    if p == 1:
        return nodes.copy()
    pts = np.empty(2 * nodes.size - 1)
    pts[0::2] = nodes
    pts[1::2] = 0.5 * (nodes[:-1] + nodes[1:])
    return pts


# --------------------------------------------------------------------------
# space
# --------------------------------------------------------------------------
def square_mesh(n):
    """Right-diagonal triangulation of (0,1)^2 with n cells per side.

    Returns (vertices (V,2), triangles (E,3) vertex ids, interior vertex ids
    in dof order)."""
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    verts = np.stack([i.ravel() * h, j.ravel() * h], axis=1)

    def vid(ii, jj):
        return jj * (n + 1) + ii

    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    t_low = np.stack([vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1)], axis=1)
    t_up = np.stack([vid(ci, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)], axis=1)
    tris = np.concatenate([t_low, t_up], axis=0)
    ii, jj = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="xy")
    interior = vid(ii.ravel(), jj.ravel())
    return verts, tris, interior


def _p1_reference(pts):
    """Reference P1 basis (1-x-y, x, y) and its constant gradients."""
    x, y = pts[:, 0], pts[:, 1]
    lam = np.stack([1.0 - x - y, x, y], axis=0)              # (3, q)
    grad = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # (3, 2)
    return lam, grad


def _affine(verts, tris):
    P0 = verts[tris[:, 0]]
    J = np.stack([verts[tris[:, 1]] - P0, verts[tris[:, 2]] - P0], axis=2)  # (E,2,2): cols = edges
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    return P0, J, det


def assemble_space_full(n):
    """Full P1 mass and stiffness over all (n+1)^2 vertices (boundary included),
    by element loops with quadrature.  Returns (M, A) as CSR matrices."""
    verts, tris, _ = square_mesh(n)
    pts, wts = triangle_rule(3)
    lam, gref = _p1_reference(pts)
    P0, J, det = _affine(verts, tris)
    absdet = np.abs(det)
    # mass: |det| * sum_q w lam_a lam_b
    Mref = (lam * wts) @ lam.T                                   # (3,3)
    Me = absdet[:, None, None] * Mref[None]
    # stiffness: grad_x lam_a = J^{-T} gref_a
    Jinv = np.linalg.inv(J)                                      # (E,2,2)
    G = np.einsum("eji,aj->eai", Jinv, gref)                     # (E,3,2): J^{-T} g
    Ae = absdet[:, None, None] * wts.sum() * np.einsum("eai,ebi->eab", G, G)
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    V = verts.shape[0]
    M = sp.coo_matrix((Me.ravel(), (rows, cols)), shape=(V, V)).tocsr()
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(V, V)).tocsr()
    return M, A


def assemble_space(n):
    """Interior-dof spatial matrices M_x, A_x (Sec. 3, eq. (matrix_x)), CSR."""
    M, A = assemble_space_full(n)
    _, _, interior = square_mesh(n)
    return (M[interior][:, interior].tocsr(), A[interior][:, interior].tocsr())


# --------------------------------------------------------------------------
# space-time load vector, interpolation and evaluation
# --------------------------------------------------------------------------
def load_vector(f, n, nodes, p, m_space=5, m_time=None):
    """F[l, k] = int_Q f(x, t) phi_k(x) varphi_l(t) for all temporal dofs l
    (t_0 included, row 0) and interior spatial dofs k (Sec. 3, right-hand side
    of eq. (LGS)), by a collapsed Gauss rule per triangle and Gauss-Legendre
    per time element.  f(x, y, t) must broadcast over arrays.

    Returns the (p N + 1) x n_x complex array."""
    nodes = np.asarray(nodes, dtype=np.float64)
    if m_time is None:
        m_time = p + 3
    verts, tris, interior = square_mesh(n)
    V = verts.shape[0]
    pts, wts = triangle_rule(m_space)
    lam, _ = _p1_reference(pts)
    P0, J, det = _affine(verts, tris)
    X = P0[:, None, 0] + J[:, 0, 0][:, None] * pts[None, :, 0] + J[:, 0, 1][:, None] * pts[None, :, 1]
    Y = P0[:, None, 1] + J[:, 1, 0][:, None] * pts[None, :, 0] + J[:, 1, 1][:, None] * pts[None, :, 1]
    wsp = np.abs(det)[:, None] * wts[None, :]                   # (E, q)
    tq, tw = gauss_legendre(m_time)
    phit, _ = lagrange_1d(p, tq)
    N = nodes.size - 1
    Ffull = np.zeros((p * N + 1, V), dtype=np.complex128)
    for e in range(N):
        h = nodes[e + 1] - nodes[e]
        for q in range(m_time):
            t = nodes[e] + h * tq[q]
            fv = f(X, Y, t) * wsp                                # (E, q)
            loc = fv @ lam.T                                     # (E, 3): int f lam_b
            contrib = np.zeros(V, dtype=np.complex128)
            np.add.at(contrib, tris.ravel(), loc.ravel())
            for a in range(p + 1):
                Ffull[p * e + a] += h * tw[q] * phit[a, q] * contrib
    return Ffull[:, interior]


def interpolate(u, n, nodes, p):
    """Nodal interpolant of u(x, y, t) in the space-time FE space: values at
    every temporal dof (t_0 included) and interior spatial vertex."""
    verts, _, interior = square_mesh(n)
    tp = time_dof_points(nodes, p)
    x = verts[interior, 0]
    y = verts[interior, 1]
    return np.stack([u(x, y, t) for t in tp], axis=0)


def full_vertex_field(U, n):
    """Embed interior values (rows x n_x) into all vertices with zero boundary."""
    _, _, interior = square_mesh(n)
    out = np.zeros((U.shape[0], (n + 1) ** 2), dtype=U.dtype)
    out[:, interior] = U
    return out
