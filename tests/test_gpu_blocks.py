"""Parity of the batched shifted spatial solver (band fill + LDL^T + sweeps,
HIP) with the oracle's sparse LU solves of (lambda_l M_x + A_x) u_l = g_l.

Tolerance: without pivoting, L D L^T is backward stable up to the growth of
|L||D||L^T|; the forward error of block l is bounded by
    c * u * cond_2(S_l) * growth_l,  u = 2^-53 (FP64) or 2^-24 (FP32),
with c a modest multiple of the half-bandwidth.  The tests compute cond_2 and
the growth ||(|L||D||L^T|)||_F / ||S||_F from the returned factor (dense, on
the CPU, small sizes) and require err_l <= 4 sqrt(kd) u cond_l growth_l."""
import numpy as np
import pytest
import torch

import paper_2504_07269_amd as st
import synth
from oracle import fem, solvers
from gpu_util import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _dense_band(Bd, n_x, kd):
    """L (unit lower) and D from band rows [d, j] = L[j+d][j], row 0 = D."""
    L = np.eye(n_x, dtype=np.complex128)
    D = Bd[0, :n_x].copy()
    for d in range(1, kd + 1):
        j = np.arange(n_x - d)
        L[j + d, j] = Bd[d, j]
    return L, D


def _case(n, count, seed, im_min):
    Ms, As, n_x, kd = st.assemble_2d_space(n)
    Mx, Ax = fem.assemble_space(n)
    lam = synth.shifts_upper_half_plane(seed, count, 3.0 * n * n, im_min, 50.0)
    return Ms, As, n_x, kd, Mx, Ax, lam


@pytest.mark.parametrize("precision", [64, 32])
# n = 40 (kd = 40) puts the panel width below kd with a partial last tile row
# of the trailing window (FP32: 32 + 8 rows, FP64: 16 + 16 + 8 rows)
@pytest.mark.parametrize("n,count,nrhs", [(2, 3, 1), (3, 5, 2), (7, 6, 3), (16, 16, 5), (21, 4, 1), (40, 2, 2)])
def test_factor_and_solve_match_oracle(precision, n, count, nrhs):
    Ms, As, n_x, kd, Mx, Ax, lam = _case(n, count, 100 + n, 1e-2)
    G = synth.random_rhs(7 + n, count, n_x, nrhs)
    ref = np.stack([solvers.block_solve(Mx, Ax, lam, G[r]) for r in range(nrhs)])
    blocks = st.shifted_factor(n, Ms, As, lam, precision)
    U = to_host(blocks.solve(to_dev(G)))
    u = U64 if precision == 64 else U32
    for l in range(count):
        S = lam[l] * Mx.toarray() + Ax.toarray()
        Lf, D = _dense_band(blocks.factor_band(l), n_x, kd)
        LDL = Lf @ np.diag(D) @ Lf.T
        growth = np.linalg.norm(np.abs(Lf) @ np.diag(np.abs(D)) @ np.abs(Lf.T)) / np.linalg.norm(S)
        # the factorisation reproduces S (complex symmetric, no pivoting)
        assert np.linalg.norm(LDL - S) <= 8 * kd * u * growth * np.linalg.norm(S)
        tol = 4 * np.sqrt(kd) * u * np.linalg.cond(S) * max(growth, 1.0) + 4 * u
        for r in range(nrhs):
            assert relerr(U[r, l], ref[r, l]) <= tol, (l, r, relerr(U[r, l], ref[r, l]), tol)


@pytest.mark.parametrize("precision", [64, 32])
def test_conjugate_solve_and_in_place(precision):
    n, count = 12, 7
    Ms, As, n_x, kd, Mx, Ax, lam = _case(n, count, 5, 1e-1)
    G = synth.random_rhs(3, count, n_x, 2)
    ref = np.stack([solvers.block_solve(Mx, Ax, lam.conj(), G[r]) for r in range(2)])
    blocks = st.shifted_factor(n, Ms, As, lam, precision)
    Gd = to_dev(G)
    out = blocks.solve(Gd, conj=True, out=Gd)          # in place
    U = to_host(out)
    tol = 1e-9 if precision == 64 else 2e-3
    assert relerr(U, ref) < tol


def test_fp32_and_fp64_factors_agree_to_fp32_accuracy():
    n, count = 24, 9
    Ms, As, n_x, kd, Mx, Ax, lam = _case(n, count, 9, 1.0)
    G = to_dev(synth.random_rhs(1, count, n_x))
    a = to_host(st.shifted_factor(n, Ms, As, lam, 64).solve(G))
    b = to_host(st.shifted_factor(n, Ms, As, lam, 32).solve(G))
    assert relerr(b, a) < 1e-3
    ref = solvers.block_solve(Mx, Ax, lam, to_host(G))
    assert relerr(a, ref) < 1e-10


def test_factor_is_deterministic():
    n, count = 17, 5
    Ms, As, n_x, kd, Mx, Ax, lam = _case(n, count, 2, 1e-1)
    G = to_dev(synth.random_rhs(2, count, n_x, 2))
    a = to_host(st.shifted_factor(n, Ms, As, lam, 32).solve(G))
    b = to_host(st.shifted_factor(n, Ms, As, lam, 32).solve(G))
    assert np.array_equal(a, b)


def test_rejects_shift_without_positive_imaginary_part():
    Ms, As, _, _ = st.assemble_2d_space(5)
    with pytest.raises(st.StfemError) as e:
        st.shifted_factor(5, Ms, As, np.array([1.0 + 0.0j]), 64)
    assert e.value.status == -1


@pytest.mark.parametrize("precision", [64, 32])
def test_full_size_c2_blocks_sampled(precision):
    """The launch configuration of the n=256, N_t=256 workload (256 blocks of
    n_x = 65025, kd = 256), checked on 3 sampled blocks against the oracle."""
    n = 256
    wl = synth.WORKLOADS["c2"]
    Mt, Bt, _, _ = fem.assemble_time(synth.uniform_nodes(wl.T, wl.N_t), 1)
    mu, _ = solvers.temporal_eigvecs(Mt, Bt)
    lam = np.sort_complex(1.0 / mu)
    Ms, As, n_x, kd = st.assemble_2d_space(n)
    Mx, Ax = fem.assemble_space(n)
    G = synth.random_rhs(11, lam.size, n_x)
    blocks = st.shifted_factor(n, Ms, As, lam, precision)
    U = to_host(blocks.solve(to_dev(G)))
    del blocks
    torch.cuda.empty_cache()
    for l in (0, 101, 255):
        ref = solvers.block_solve(Mx, Ax, lam[l:l + 1], G[l:l + 1])[0]
        # block residual relative to ||S|| ||u||, the backward error of the solve
        S = lam[l] * Mx + Ax
        res = np.linalg.norm(S @ U[l] - G[l]) / (abs(lam[l]) * np.abs(Mx).sum(axis=1).max() * np.linalg.norm(U[l])
                                                 + np.abs(Ax).sum(axis=1).max() * np.linalg.norm(U[l]))
        bound = 1e-12 if precision == 64 else 1e-4
        assert res < bound, (l, res)
        if precision == 64:
            assert relerr(U[l], ref) < 1e-6, (l, relerr(U[l], ref))
