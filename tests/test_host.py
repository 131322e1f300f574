"""CPU tests of the library's host side: the C ABI loads and exports every
declared entry point, host assembly equals the oracle's element loops, the
host temporal eigen-step matches the oracle's LAPACK decomposition and the
paper's kappa_2 values, and argument errors are reported."""
import json
import math
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2504_07269_amd as st
from paper_2504_07269_amd import _lib
from oracle import fem, solvers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))


def header_functions():
    text = open(os.path.join(ROOT, "include", "stfem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = header_functions()
    assert "fdm_factor" in names and "fdm_solve_adjoint" in names and "assemble_1d_time" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_lib.exported_symbols())


def test_strerror_names_every_status():
    L = _lib.lib()
    for code in range(-6, 1):
        assert L.stfem_strerror(code).decode() != "unknown status"


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("graded", [False, True])
def test_assemble_1d_time_matches_oracle(p, graded):
    nodes = fem.time_nodes_graded(2.0, 9, 1.5, 1) if graded else fem.time_nodes_uniform(3.0, 11)
    M, B, m0, b0 = st.assemble_1d_time(nodes, p)
    Mo, Bo, m0o, b0o = fem.assemble_time(nodes, p)
    assert np.abs(M - Mo).max() < 1e-15 * max(1, np.abs(Mo).max()) + 1e-16
    assert np.abs(B - Bo).max() < 1e-14
    assert np.abs(m0 - m0o).max() < 1e-15
    assert np.abs(b0 - b0o).max() < 1e-14


def stencil_matrix(n, stc):
    """Sparse matrix of a 7-point stencil in the library's order (C,E,W,N,S,NE,SW)."""
    m = n - 1
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]
    rows, cols, vals = [], [], []
    for j in range(m):
        for i in range(m):
            for (di, dj), v in zip(offs, stc):
                ii, jj = i + di, j + dj
                if 0 <= ii < m and 0 <= jj < m and v != 0:
                    rows.append(j * m + i)
                    cols.append(jj * m + ii)
                    vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m * m, m * m))


@pytest.mark.parametrize("n", [2, 3, 9, 32])
def test_assemble_2d_space_matches_oracle(n):
    Ms, As, nx, kd = st.assemble_2d_space(n)
    assert nx == (n - 1) ** 2 and kd == n
    Mo, Ao = fem.assemble_space(n)
    assert abs(stencil_matrix(n, Ms) - Mo).max() < 1e-14 * abs(Mo).max()
    assert abs(stencil_matrix(n, As) - Ao).max() < 1e-13


def _temporal(Nt, T, p=1, graded=False):
    nodes = fem.time_nodes_graded(T, Nt, 1.5, 0) if graded else fem.time_nodes_uniform(T, Nt)
    return st.assemble_1d_time(nodes, p)[:2]


@pytest.mark.parametrize("Nt,T,p,graded", [(1, 0.3, 1, False), (16, 1.0, 1, False), (64, 5.0, 1, True),
                                           (128, 1.0, 1, False), (24, 1.0, 2, False)])
def test_fdm_temporal_matches_oracle(Nt, T, p, graded):
    M, B = _temporal(Nt, T, p, graded)
    lam, X, W, kap, its = st.fdm_temporal(M, B)
    mu, Xo = solvers.temporal_eigvecs(M, B)
    lam_o = 1.0 / mu
    # every oracle eigenvalue is matched (relative error at the eigenvalue-conditioning level)
    for l in lam_o:
        assert np.min(np.abs(lam - l)) <= 1e-10 * abs(l)
    # ascending real parts
    assert np.all(np.diff(lam.real) >= 0)
    # unit columns, M^{-1} i B X = X Lambda, W M X = I
    assert np.abs(np.linalg.norm(X, axis=0) - 1).max() < 1e-13
    A = np.linalg.solve(M, 1j * B)
    assert np.abs(A @ X - X * lam).max() < 1e-11 * np.abs(lam).max()
    assert np.abs(W @ M @ X - np.eye(M.shape[0])).max() < 1e-10
    kref = np.linalg.cond(Xo)
    assert abs(kap - kref) < 0.02 * kref


@pytest.mark.parametrize("Nt", [64, 128, 256])
def test_fdm_temporal_kappa_matches_table2(Nt):
    M, B = _temporal(Nt, 5.0)
    kap = st.fdm_temporal(M, B)[3]
    printed = GOLDEN["kappa2_uniform"][str(Nt)]
    assert abs(kap - printed) <= 0.05 * 10 ** math.floor(math.log10(printed)), kap


def test_fdm_temporal_single_element_closed_form():
    h = 0.37
    M, B = st.assemble_1d_time(np.array([0.0, h]), 1)[:2]
    lam = st.fdm_temporal(M, B)[0]
    assert abs(lam[0] - 1.5j / h) < 1e-13 / h


def test_host_decomposition_gives_exact_fdm_on_cpu():
    # Using the library's lambda, X, W with exact (oracle) block solves
    # reproduces the dense global solve: checks the transform convention.
    n, Nt = 9, 12
    M, B = _temporal(Nt, 1.0)
    Mx, Ax = fem.assemble_space(n)
    lam, X, W, _, _ = st.fdm_temporal(M, B)
    rng = np.random.default_rng(4)
    F = rng.standard_normal((Nt, 64)) + 1j * rng.standard_normal((Nt, 64))
    U = solvers.block_solve(Mx, Ax, lam, W @ F)
    ref = solvers.solve_dense(M, B, Mx, Ax, F)
    assert np.linalg.norm(X @ U - ref) / np.linalg.norm(ref) < 1e-12


def test_argument_errors():
    with pytest.raises(_lib.StfemError) as e:
        st.assemble_1d_time(np.array([0.0, 0.5, 0.5, 1.0]), 1)
    assert e.value.status == -1
    with pytest.raises(_lib.StfemError):
        st.assemble_1d_time(np.array([0.1, 0.5]), 1)
    with pytest.raises(_lib.StfemError):
        st.assemble_2d_space(1)
    wide = np.eye(12)
    wide[0, 11] = 1.0
    with pytest.raises(_lib.StfemError) as e:
        st.fdm_temporal(wide, np.eye(12))
    assert e.value.status == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message, before
    any device work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_block_refinement_is_accepted_and_unknown_modes_rejected():
    """refine='block' maps to STFEM_REFINE_BLOCK; other names are refused
    before the library is called."""
    assert st.FDM.REFINE == {"gmres": 0, "plain": 1, "block": 2}
    header = open(os.path.join(ROOT, "include", "stfem.h")).read()
    assert "STFEM_REFINE_BLOCK = 2" in header
    Mt = np.eye(2)
    with pytest.raises(ValueError):
        st.fdm_factor(Mt, Mt, np.zeros(7), np.zeros(7), 4, refine="bogus")
