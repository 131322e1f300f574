"""Pins of the CPU oracle against what the paper and the mathematics fix:
values printed in the paper, closed forms, invariants, special cases, library
routines and brute force on tiny inputs.  None of these re-derive the oracle's
own formula."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, norms, problems, quadrature, solvers

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


# ------------------------------------------------------------------ quadrature
@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_gauss_legendre_exactness(m):
    x, w = quadrature.gauss_legendre(m)
    for k in range(2 * m):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    # degree 2m is not integrated exactly
    assert abs(np.sum(w * x ** (2 * m)) - 1.0 / (2 * m + 1)) > 1e-8


@pytest.mark.parametrize("m", [2, 3, 5])
def test_triangle_rule_exactness(m):
    pts, w = quadrature.triangle_rule(m)
    for a in range(2 * m - 1):
        for b in range(2 * m - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b) - exact) < 1e-14


# ------------------------------------------------------------ temporal matrices
@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("graded", [False, True])
def test_time_matrix_invariants(p, graded):
    T = 2.5
    nodes = fem.time_nodes_graded(T, 7, 1.5, 1) if graded else fem.time_nodes_uniform(T, 9)
    Mf, Bf = fem.assemble_time_full(nodes, p)
    nd = Mf.shape[0]
    one = np.ones(nd)
    # sum of all basis functions is 1: 1^T M 1 = T, and (M 1)_k = int phi_k > 0
    assert abs(one @ Mf @ one - T) < 1e-13
    # int phi_j' dt = phi_j(T) - phi_j(0)  (column sums of B)
    e0 = np.zeros(nd)
    e0[0] = 1
    eN = np.zeros(nd)
    eN[-1] = 1
    assert np.abs(one @ Bf - (eN - e0)).max() < 1e-13
    # integration by parts: B + B^T = e_N e_N^T - e_0 e_0^T
    assert np.abs(Bf + Bf.T - (np.outer(eN, eN) - np.outer(e0, e0))).max() < 1e-13
    # mass integrates t exactly: (t^T M 1) = T^2/2 (t nodal interpolant is exact)
    tp = fem.time_dof_points(nodes, p)
    assert abs(tp @ Mf @ one - T ** 2 / 2) < 1e-12
    # M symmetric positive definite
    assert np.abs(Mf - Mf.T).max() < 1e-15
    assert np.linalg.eigvalsh(Mf).min() > 0


def test_time_matrix_closed_forms_p1():
    N, T = 6, 3.0
    h = T / N
    Mt, Bt, mc, bc = fem.assemble_time(fem.time_nodes_uniform(T, N), 1)
    Mc = np.diag(np.r_[np.full(N - 1, 2 * h / 3), h / 3]) + np.diag(np.full(N - 1, h / 6), 1) + np.diag(np.full(N - 1, h / 6), -1)
    Bc = np.diag(np.full(N - 1, 0.5), 1) - np.diag(np.full(N - 1, 0.5), -1)
    Bc[-1, -1] = 0.5
    assert np.abs(Mt - Mc).max() < 1e-15
    assert np.abs(Bt - Bc).max() < 1e-15
    assert np.allclose(mc, np.r_[h / 6, np.zeros(N - 1)], atol=1e-15)
    assert np.allclose(bc, np.r_[-0.5, np.zeros(N - 1)], atol=1e-15)


def test_time_matrix_closed_forms_p2():
    # one element of length h: textbook quadratic Lagrange element matrices
    h = 0.7
    Mf, Bf = fem.assemble_time_full(np.array([0.0, h]), 2)
    Me = h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]])
    Be = np.array([[-3, 4, -1], [-4, 0, 4], [1, -4, 3]]) / 6.0
    assert np.abs(Mf - Me).max() < 1e-15
    assert np.abs(Bf - Be).max() < 1e-14


# ------------------------------------------------------------- spatial matrices
@pytest.mark.parametrize("n", [2, 5, 8])
def test_space_matrix_closed_forms(n):
    Mx, Ax = fem.assemble_space(n)
    h = 1.0 / n
    m = n - 1
    Md = Mx.toarray()
    Ad = Ax.toarray()
    for j in range(m):
        for i in range(m):
            k = j * m + i
            row_a = {k: 4.0}
            row_m = {k: h * h / 2}
            for di, dj, mv in [(1, 0, 1), (-1, 0, 1), (0, 1, 1), (0, -1, 1), (1, 1, 0), (-1, -1, 0)]:
                ii, jj = i + di, j + dj
                if 0 <= ii < m and 0 <= jj < m:
                    kk = jj * m + ii
                    row_m[kk] = h * h / 12
                    if mv:
                        row_a[kk] = -1.0
            ref_a = np.zeros(m * m)
            ref_m = np.zeros(m * m)
            for kk, v in row_a.items():
                ref_a[kk] = v
            for kk, v in row_m.items():
                ref_m[kk] = v
            assert np.abs(Ad[k] - ref_a).max() < 1e-13
            assert np.abs(Md[k] - ref_m).max() < 1e-16


def test_space_matrix_invariants():
    n = 7
    M, A = fem.assemble_space_full(n)
    verts, _, interior = fem.square_mesh(n)
    V = verts.shape[0]
    one = np.ones(V)
    assert abs(one @ (M @ one) - 1.0) < 1e-14           # area of the unit square
    lin = 0.3 + 1.7 * verts[:, 0] - 2.1 * verts[:, 1]
    assert np.abs((A @ lin)[interior]).max() < 1e-13    # P1 reproduces linears exactly
    assert np.abs(A @ one).max() < 1e-13
    assert abs(lin @ (M @ one) - (0.3 + 1.7 / 2 - 2.1 / 2)) < 1e-14


# ------------------------------------------------------------ temporal decomposition
@pytest.mark.parametrize("Nt", [64, 128, 256])
def test_kappa_uniform_matches_table2(Nt):
    Mt, Bt, _, _ = fem.assemble_time(fem.time_nodes_uniform(5.0, Nt), 1)
    k = solvers.kappa2_Xt(Mt, Bt)
    printed = GOLDEN["kappa2_uniform"][str(Nt)]
    assert abs(k - printed) <= 0.05 * 10 ** math.floor(math.log10(printed)), (k, printed)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_kappa_graded_matches_table3(level):
    nodes = fem.time_nodes_graded(5.0, 64, 1.5, level)
    Mt, Bt, _, _ = fem.assemble_time(nodes, 1)
    k = solvers.kappa2_Xt(Mt, Bt)
    printed = GOLDEN["kappa2_graded"][str(64 * 2 ** level)]
    assert abs(k - printed) <= 0.05 * 10 ** math.floor(math.log10(printed)), (k, printed)
    h = np.diff(nodes)
    assert abs(h.max() / h.min() - GOLDEN["graded_ht_ratio"]["ratio"]) < 0.5


@pytest.mark.slow
def test_kappa_uniform_512_matches_table2():
    Mt, Bt, _, _ = fem.assemble_time(fem.time_nodes_uniform(5.0, 512), 1)
    k = solvers.kappa2_Xt(Mt, Bt)
    assert abs(k - 7.1e3) <= 50, k


def test_kappa_independent_of_T():
    a = solvers.kappa2_Xt(*fem.assemble_time(fem.time_nodes_uniform(1.0, 96), 1)[:2])
    b = solvers.kappa2_Xt(*fem.assemble_time(fem.time_nodes_uniform(5.0, 96), 1)[:2])
    assert abs(a - b) < 1e-8 * a


@pytest.mark.parametrize("p,Nt", [(1, 40), (2, 20)])
def test_eigen_invariants(p, Nt):
    T = 1.3
    Mt, Bt, _, _ = fem.assemble_time(fem.time_nodes_uniform(T, Nt), p)
    mu, X = solvers.temporal_eigvecs(Mt, Bt)
    lam = 1.0 / mu                            # eigenvalues of M_t^{-1} (i B_t)
    # Im lam = |x_N|^2 / (2 x^H M x) > 0 because B + B^T = e_N e_N^T
    assert lam.imag.min() > 0
    # real matrices: spectrum symmetric under lam -> -conj(lam)
    for l in lam:
        assert np.min(np.abs(lam + np.conj(l))) < 1e-9 * abs(l)


def test_eigen_single_element():
    h = 0.37
    Mt, Bt, _, _ = fem.assemble_time(np.array([0.0, h]), 1)
    mu, _ = solvers.temporal_eigvecs(Mt, Bt)
    assert abs(1.0 / mu[0] - 1.5j / h) < 1e-13


def test_eigen_max_real_part_p1():
    # max |Re lam| h_t -> sqrt(3) for P1 on uniform meshes
    Nt, T = 400, 1.0
    Mt, Bt, _, _ = fem.assemble_time(fem.time_nodes_uniform(T, Nt), 1)
    mu, _ = solvers.temporal_eigvecs(Mt, Bt)
    assert abs(np.abs((1.0 / mu).real).max() * T / Nt - math.sqrt(3)) < 2e-3


# ------------------------------------------------------------------ global solves
def _c0_system(p=1, Nt=16, n=16, T=1.0):
    nodes = fem.time_nodes_uniform(T, Nt)
    Mt, Bt, mc, bc = fem.assemble_time(nodes, p)
    Mx, Ax = fem.assemble_space(n)
    return nodes, Mt, Bt, mc, bc, Mx, Ax


def test_dense_matches_sparse_library_solve():
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(Nt=6, n=7)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((6, 36)) + 1j * rng.standard_normal((6, 36))
    a = solvers.solve_dense(Mt, Bt, Mx, Ax, F)
    b = solvers.solve_sparse(Mt, Bt, Mx, Ax, F)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def test_kron_layout_brute_force():
    # (A kron B) vec(U) = vec(A U B^T) with the time-major layout, entry by entry
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(Nt=3, n=3)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    KU = solvers.apply_global(Mt, Bt, Mx, Ax, U)
    Mxd, Axd = Mx.toarray(), Ax.toarray()
    ref = np.zeros_like(U)
    for l in range(3):
        for k in range(4):
            s = 0
            for m in range(3):
                for j in range(4):
                    s += (1j * Bt[l, m] * Mxd[k, j] + Mt[l, m] * Axd[k, j]) * U[m, j]
            ref[l, k] = s
    assert np.abs(KU - ref).max() < 1e-14


@pytest.mark.parametrize("p", [1, 2])
def test_fdm_and_bs_match_dense(p):
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(p=p, Nt=16 // p)
    rng = np.random.default_rng(11)
    F = rng.standard_normal((16, 225)) + 1j * rng.standard_normal((16, 225))
    ref = solvers.solve_dense(Mt, Bt, Mx, Ax, F)
    fdm = solvers.fdm_paper(Mt, Bt, Mx, Ax, F)
    bs = solvers.bartels_stewart_paper(Mt, Bt, Mx, Ax, F)
    assert np.linalg.norm(fdm - ref) / np.linalg.norm(ref) < 1e-12
    assert np.linalg.norm(bs - ref) / np.linalg.norm(ref) < 1e-12
    assert solvers.relres(Mt, Bt, Mx, Ax, fdm, F) < 1e-13


def test_dense_adjoint_dot_test():
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(Nt=8, n=8)
    rng = np.random.default_rng(3)
    a = rng.standard_normal((8, 49)) + 1j * rng.standard_normal((8, 49))
    b = rng.standard_normal((8, 49)) + 1j * rng.standard_normal((8, 49))
    x = solvers.solve_dense(Mt, Bt, Mx, Ax, a)
    y = solvers.solve_dense_adjoint(Mt, Bt, Mx, Ax, b)
    lhs = np.vdot(b, x)             # <K^{-1} a, b> = b^H K^{-1} a
    rhs = np.vdot(y, a)             # <a, K^{-H} b> = (K^{-H} b)^H a
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_block_solve_matches_dense():
    Mx, Ax = fem.assemble_space(6)
    lam = np.array([-30 + 0.5j, 12 + 3j, -200 + 1e-3j])
    rng = np.random.default_rng(0)
    G = rng.standard_normal((3, 25)) + 1j * rng.standard_normal((3, 25))
    U = solvers.block_solve(Mx, Ax, lam, G)
    for l in range(3):
        ref = np.linalg.solve(lam[l] * Mx.toarray() + Ax.toarray(), G[l])
        assert np.linalg.norm(U[l] - ref) < 1e-10 * np.linalg.norm(ref)


# -------------------------------------------------- manufactured solutions, rates
@pytest.mark.parametrize("prob", [problems.PaperSolution(), problems.OmegaSolution(4 * np.pi)])
def test_rhs_matches_finite_differences(prob):
    rng = np.random.default_rng(2)
    x, y, t = rng.uniform(0.1, 0.9, 3)
    e = 1e-4
    dt = (prob.psi(x, y, t + e) - prob.psi(x, y, t - e)) / (2 * e)
    lap = (prob.psi(x + e, y, t) + prob.psi(x - e, y, t) + prob.psi(x, y + e, t)
           + prob.psi(x, y - e, t) - 4 * prob.psi(x, y, t)) / e ** 2
    assert abs(1j * dt - lap - prob.f(x, y, t)) < 1e-5 * max(1, abs(prob.f(x, y, t)))
    assert abs(prob.dt(x, y, t) - dt) < 1e-6 * max(1, abs(dt))
    gx = (prob.psi(x + e, y, t) - prob.psi(x - e, y, t)) / (2 * e)
    gy = (prob.psi(x, y + e, t) - prob.psi(x, y - e, t)) / (2 * e)
    ax, ay = prob.grad(x, y, t)
    assert abs(ax - gx) < 1e-6 * max(1, abs(gx)) and abs(ay - gy) < 1e-6 * max(1, abs(gy))
    assert abs(prob.psi(x, y, 0.0) - prob.psi0(np.array(x), np.array(y))) < 1e-15


def _paper_errors(n, Nt, nodes=None, T=5.0):
    prob = problems.PaperSolution()
    if nodes is None:
        nodes = fem.time_nodes_uniform(T, Nt)
    Mt, Bt, _, _ = fem.assemble_time(nodes, 1)
    Mx, Ax = fem.assemble_space(n)
    F = fem.load_vector(prob.f, n, nodes, 1)
    U = solvers.fdm_paper(Mt, Bt, Mx, Ax, F[1:])
    Uf = np.concatenate([np.zeros((1, U.shape[1])), U])
    return norms.errors(prob, Uf, n, nodes, 1)


def _printed_ok(value, printed):
    return abs(value - printed) <= 0.05 * 10 ** math.floor(math.log10(printed))


def test_paper_J0_errors_uniform():
    l2, h1 = _paper_errors(32, 64)
    g = GOLDEN["errors_J0_uniform"]
    assert _printed_ok(l2, g["L2"]), l2
    assert _printed_ok(h1, g["H1"]), h1


def test_paper_J0_errors_graded():
    nodes = fem.time_nodes_graded(5.0, 64, 1.5, 0)
    l2, h1 = _paper_errors(32, 64, nodes=nodes)
    g = GOLDEN["errors_J0_graded"]
    assert _printed_ok(l2, g["L2"]), l2
    assert _printed_ok(h1, g["H1"]), h1


@pytest.mark.slow
def test_paper_J1_errors_uniform():
    l2, h1 = _paper_errors(64, 128)
    g = GOLDEN["errors_J1_uniform"]
    assert _printed_ok(l2, g["L2"]), l2
    assert _printed_ok(h1, g["H1"]), h1


def test_paper_dof_bookkeeping():
    for J in range(5):
        nx = (2 ** (5 + J) - 1) ** 2
        assert nx * 64 * 2 ** J == GOLDEN["dofs"][str(J)]


def test_convergence_rates_omega_with_lift():
    # psi_0 != 0: lift with psi_0 constant in time; eoc -> 2 (L2) and 1 (H1)
    prob = problems.OmegaSolution(np.pi)
    errs = []
    for n in (4, 8, 16):
        nodes = fem.time_nodes_uniform(1.0, n)
        Mf, Bf = fem.assemble_time_full(nodes, 1)
        Mx, Ax = fem.assemble_space(n)
        F = fem.load_vector(prob.f, n, nodes, 1)
        psi0 = fem.interpolate(lambda x, y, t: prob.psi0(x, y), n, nodes, 1)[0]
        Fh = solvers.lift_constant(F, psi0, Mf, Ax)
        U = solvers.solve_sparse(Mf[1:, 1:], Bf[1:, 1:], Mx, Ax, Fh)
        Uf = np.concatenate([np.zeros((1, U.shape[1])), U]) + psi0[None, :]
        errs.append(norms.errors(prob, Uf, n, nodes, 1))
    errs = np.array(errs)
    r2 = norms.eoc(errs[:, 0])
    r1 = norms.eoc(errs[:, 1])
    assert 1.8 < r2[-1] < 2.2, r2
    assert 0.9 < r1[-1] < 1.1, r1


def test_convergence_rates_p2_in_time():
    # P2 in time with P1 in space: still eoc 2 in L2 (limited by space)
    prob = problems.OmegaSolution(np.pi)
    errs = []
    for n in (4, 8, 16):
        nodes = fem.time_nodes_uniform(1.0, max(n // 2, 1))
        Mf, Bf = fem.assemble_time_full(nodes, 2)
        Mx, Ax = fem.assemble_space(n)
        F = fem.load_vector(prob.f, n, nodes, 2)
        psi0 = fem.interpolate(lambda x, y, t: prob.psi0(x, y), n, nodes, 2)[0]
        Fh = solvers.lift_constant(F, psi0, Mf, Ax)
        U = solvers.solve_sparse(Mf[1:, 1:], Bf[1:, 1:], Mx, Ax, Fh)
        Uf = np.concatenate([np.zeros((1, U.shape[1])), U]) + psi0[None, :]
        errs.append(norms.errors(prob, Uf, n, nodes, 2))
    r2 = norms.eoc(np.array(errs)[:, 0])
    assert 1.8 < r2[-1] < 2.3, r2


def test_lift_by_t0_hat_equals_constant_lift():
    # psi_h is unique: lifting with the t_0 hat function (only the first
    # temporal row changes) and with psi_0 constant in time give the same psi_h.
    prob = problems.OmegaSolution(np.pi)
    n, Nt = 6, 5
    nodes = fem.time_nodes_uniform(1.0, Nt)
    Mf, Bf = fem.assemble_time_full(nodes, 1)
    Mt, Bt, mc, bc = fem.assemble_time(nodes, 1)
    Mx, Ax = fem.assemble_space(n)
    F = fem.load_vector(prob.f, n, nodes, 1)
    psi0 = fem.interpolate(lambda x, y, t: prob.psi0(x, y), n, nodes, 1)[0]
    Uc = solvers.solve_dense(Mt, Bt, Mx, Ax, solvers.lift_constant(F, psi0, Mf, Ax)) + psi0[None]
    Fh = F[1:] - (1j * np.outer(bc, Mx @ psi0) + np.outer(mc, Ax @ psi0))
    Uh = solvers.solve_dense(Mt, Bt, Mx, Ax, Fh)
    assert np.abs(Uc - Uh).max() < 1e-12 * np.abs(Uc).max()


def test_structured_matvec_matches_kron():
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(p=2, Nt=4, n=6)
    rng = np.random.default_rng(8)
    U = rng.standard_normal((2, 8, 25)) + 1j * rng.standard_normal((2, 8, 25))
    a = solvers.apply_global_structured(Mt, Bt, Mx, Ax, U)
    for k in range(2):
        assert np.abs(a[k] - solvers.apply_global(Mt, Bt, Mx, Ax, U[k])).max() < 1e-14


def test_fdm_paper_multiple_rhs():
    _, Mt, Bt, _, _, Mx, Ax = _c0_system(Nt=5, n=6)
    rng = np.random.default_rng(9)
    F = rng.standard_normal((3, 5, 25)) + 1j * rng.standard_normal((3, 5, 25))
    a = solvers.fdm_paper(Mt, Bt, Mx, Ax, F)
    for k in range(3):
        assert np.abs(a[k] - solvers.solve_dense(Mt, Bt, Mx, Ax, F[k])).max() < 1e-12 * np.abs(a[k]).max()
