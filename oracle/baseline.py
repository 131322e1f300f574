"""The oracle's fast diagonalization run time-parallel on the host cores: the
CPU throughput baseline (test infrastructure only).

It is the paper's own parallelisation of the method (Sec. 4, discussion of
Table 2): the n_t spatial problems of eq. (LGS_x) are independent once S_t is
diagonal, so they are distributed over worker processes, one sparse direct
factorisation and solve each; the temporal decomposition and the two
transforms run in numpy on the parent.  Nothing here is tuned.
"""
import os
import time

import numpy as np

_G = {}


def _init(n):
    from .fem import assemble_space
    import scipy.sparse as sp
    Mx, Ax = assemble_space(n)
    _G["Mx"] = sp.csc_matrix(Mx)
    _G["Ax"] = sp.csc_matrix(Ax)


def _solve_block(args):
    import scipy.sparse.linalg as spla
    mu, g = args
    lu = spla.splu((_G["Mx"] + mu * _G["Ax"]).tocsc())
    return lu.solve(g)


def default_workers():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    return max(1, min(16, cores))


def fdm_timed(Mt, Bt, n, F, workers=None, block_stride=1):
    """Time the paper-form FDM on one right-hand side F (n_t x n_x).

    Spatial problems l = 0, block_stride, 2 block_stride, ... are solved (all
    of them for block_stride = 1) and their wall time is scaled by the
    fraction solved.  Returns (psi or None, dict of timings in seconds)."""
    import multiprocessing as mp
    workers = workers or default_workers()
    t0 = time.perf_counter()
    iB = 1j * np.asarray(Bt, dtype=np.complex128)
    A = np.linalg.solve(iB, np.asarray(Mt, dtype=np.float64))
    mu, X = np.linalg.eig(A)
    X = X / np.linalg.norm(X, axis=0)
    Y = np.linalg.solve(X, np.linalg.inv(iB))
    t1 = time.perf_counter()
    G = Y @ F
    t2 = time.perf_counter()
    idx = list(range(0, G.shape[0], block_stride))
    ctx = mp.get_context("spawn")
    # one BLAS thread per worker: several multithreaded BLAS pools on the same
    # cores spin against each other and slow every sparse LU down many times
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with ctx.Pool(workers, initializer=_init, initargs=(n,)) as pool:
            pool.map(_solve_block, [(mu[0], np.ascontiguousarray(G[0]))] * workers)   # start-up, not timed
            t3 = time.perf_counter()
            sols = pool.map(_solve_block, [(mu[l], np.ascontiguousarray(G[l])) for l in idx], chunksize=1)
            t4 = time.perf_counter()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    psi = None
    t5 = t6 = 0.0
    if block_stride == 1:
        Wb = np.stack(sols)
        t5 = time.perf_counter()
        psi = X @ Wb
        t6 = time.perf_counter()
        back = t6 - t5
    else:
        back = t2 - t1          # same shape of GEMM as the forward transform
    blocks = (t4 - t3) * G.shape[0] / len(idx)
    timing = dict(eig=t1 - t0, transform=t2 - t1, blocks=blocks, back_transform=back, workers=workers,
                  blocks_solved=len(idx), blocks_total=G.shape[0])
    timing["total"] = timing["eig"] + timing["transform"] + timing["blocks"] + timing["back_transform"]
    return psi, timing
