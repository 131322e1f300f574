"""MI355X space-time Galerkin solver for the linear Schroedinger equation.

Python face of libstfem.so: the functions here have the names of the C entry
points (include/stfem.h) and only marshal arguments.  torch provides device
memory and the current HIP stream; all arithmetic of the solve runs in the
library.

    M_t, B_t, m0, b0 = assemble_1d_time(t_nodes, p)
    Ms, As, n_x, kd  = assemble_2d_space(n)
    h   = fdm_factor(M_t, B_t, Ms, As, n, precision=32, tol=1e-10, max_iter=30)
    Psi = fdm_solve(h, F)            # F: complex128 cuda tensor [(nrhs,) n_t, n_x]
    Lam = fdm_solve_adjoint(h, G)
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import Options, Report, StfemError, check, cptr, dptr, lib

__all__ = ["assemble_1d_time", "assemble_2d_space", "fdm_temporal", "fdm_factor", "fdm_solve", "fdm_solve_adjoint", "fdm_apply",
           "FDM", "ShiftedBlocks", "shifted_factor", "apply_spatial", "StfemError", "lib"]


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous complex128 CUDA tensor" % name)


# ------------------------------------------------------------------ assembly
def assemble_1d_time(t_nodes, p=1):
    """Temporal matrices (Sec. 3, eq. (matrix_t)) without the t_0 dof.
    Returns (M_t, B_t, m_col0, b_col0) as float64 numpy arrays."""
    t = np.ascontiguousarray(t_nodes, dtype=np.float64)
    n_el = t.size - 1
    nt = p * n_el
    M = np.zeros((nt, nt))
    B = np.zeros((nt, nt))
    m0 = np.zeros(nt)
    b0 = np.zeros(nt)
    check(lib().assemble_1d_time(n_el, dptr(t), p, dptr(M), dptr(B), dptr(m0), dptr(b0)))
    return M, B, m0, b0


def assemble_2d_space(n):
    """7-point P1 stencils of M_x and A_x (order C, E, W, N, S, NE, SW) on the
    right-diagonal mesh with n cells per side.  Returns (M_st, A_st, n_x, kd)."""
    Ms = np.zeros(7)
    As = np.zeros(7)
    nx = ctypes.c_int()
    kd = ctypes.c_int()
    check(lib().assemble_2d_space(n, dptr(Ms), dptr(As), ctypes.byref(nx), ctypes.byref(kd)))
    return Ms, As, nx.value, kd.value


# ----------------------------------------------------------------------- FDM
def fdm_temporal(M_t, B_t):
    """Host temporal decomposition M_t^{-1} i B_t = X diag(lambda) X^{-1},
    W = (M_t X)^{-1}.  Returns (lambda, X, W, kappa_estimate, sweeps)."""
    M_t = np.ascontiguousarray(M_t, dtype=np.float64)
    B_t = np.ascontiguousarray(B_t, dtype=np.float64)
    nt = M_t.shape[0]
    lam = np.zeros(nt, np.complex128)
    X = np.zeros((nt, nt), np.complex128)
    W = np.zeros((nt, nt), np.complex128)
    kap = ctypes.c_double()
    its = ctypes.c_int()
    check(lib().fdm_temporal(dptr(M_t), dptr(B_t), nt, cptr(lam), cptr(X), cptr(W), ctypes.byref(kap),
                             ctypes.byref(its)))
    return lam, X, W, kap.value, its.value


class FDM:
    """Owner of a factored Kronecker system (stfem_handle)."""

    REFINE = {"gmres": 0, "plain": 1, "block": 2}

    def __init__(self, M_t, B_t, M_st, A_st, n, precision=64, tol=1e-10, max_iter=30, stream=None, refine="gmres",
                 restart=0, factor_budget=0.0):
        M_t = np.ascontiguousarray(M_t, dtype=np.float64)
        B_t = np.ascontiguousarray(B_t, dtype=np.float64)
        M_st = np.ascontiguousarray(M_st, dtype=np.float64)
        A_st = np.ascontiguousarray(A_st, dtype=np.float64)
        nt = M_t.shape[0]
        if M_t.shape != (nt, nt) or B_t.shape != (nt, nt):
            raise ValueError("temporal matrices must be square and equal in size")
        if refine not in self.REFINE:
            raise ValueError("refine must be one of %s" % sorted(self.REFINE))
        opt = Options(int(precision), int(max_iter), float(tol), self.REFINE[refine], int(restart),
                      float(factor_budget))
        h = ctypes.c_void_p()
        check(lib().fdm_factor(dptr(M_t), dptr(B_t), nt, dptr(M_st), dptr(A_st), int(n), ctypes.byref(opt),
                               _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n_t, self.n_x, self.n, self.precision = nt, (n - 1) ** 2, n, precision
        self.last_report = None

    def _solve(self, fn, F, out, stream):
        import torch
        _check_tensor(F, "right-hand side")
        squeeze = F.dim() == 2
        Fv = F.unsqueeze(0) if squeeze else F
        if tuple(Fv.shape[1:]) != (self.n_t, self.n_x):
            raise ValueError("expected shape [nrhs, %d, %d], got %s" % (self.n_t, self.n_x, tuple(F.shape)))
        if out is None:
            out = torch.empty_like(Fv)
        _check_tensor(out, "output")
        rep = Report()
        st = fn(self._h, ctypes.c_void_p(Fv.data_ptr()), ctypes.c_void_p(out.data_ptr()), Fv.shape[0],
                _stream(stream), ctypes.byref(rep))
        self.last_report = rep.as_dict()
        check(st)
        return out[0] if squeeze else out

    def solve(self, F, out=None, stream=None):
        """Psi = K^{-1} F (Sec. 3, eq. (LGS)), with refinement to the factor-time tolerance."""
        return self._solve(lib().fdm_solve, F, out, stream)

    def solve_adjoint(self, G, out=None, stream=None):
        """Lam = K^{-H} G with the same factors."""
        return self._solve(lib().fdm_solve_adjoint, G, out, stream)

    def apply(self, Psi, adjoint=False, out=None, stream=None):
        """K Psi (or K^H Psi) by the GPU Kronecker matvec."""
        import torch
        _check_tensor(Psi, "Psi")
        squeeze = Psi.dim() == 2
        P = Psi.unsqueeze(0) if squeeze else Psi
        if out is None:
            out = torch.empty_like(P)
        check(lib().fdm_apply(self._h, ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(out.data_ptr()), P.shape[0],
                              int(bool(adjoint)), _stream(stream)))
        return out[0] if squeeze else out

    def decomposition(self):
        """(lambda, X, W, kappa) of the host temporal eigen-step, numpy."""
        nt = self.n_t
        lam = np.zeros(nt, np.complex128)
        X = np.zeros((nt, nt), np.complex128)
        W = np.zeros((nt, nt), np.complex128)
        kap = ctypes.c_double()
        check(lib().fdm_decomposition(self._h, cptr(lam), cptr(X), cptr(W), ctypes.byref(kap)))
        return lam, X, W, kap.value

    def close(self):
        if getattr(self, "_h", None):
            lib().fdm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fdm_factor(M_t, B_t, M_st, A_st, n, precision=64, tol=1e-10, max_iter=30, stream=None, refine="gmres",
               restart=0, factor_budget=0.0):
    return FDM(M_t, B_t, M_st, A_st, n, precision, tol, max_iter, stream, refine, restart, factor_budget)


def fdm_solve(h, F, out=None, stream=None):
    return h.solve(F, out, stream)


def fdm_solve_adjoint(h, G, out=None, stream=None):
    return h.solve_adjoint(G, out, stream)


def fdm_apply(h, Psi, adjoint=False, out=None, stream=None):
    return h.apply(Psi, adjoint, out, stream)


# ---------------------------------------------------- batched shifted blocks
class ShiftedBlocks:
    """Factored blocks lambda_l M_x + A_x (stfem_blocks)."""

    def __init__(self, n, M_st, A_st, lambdas, precision=64, stream=None):
        lam = np.ascontiguousarray(lambdas, dtype=np.complex128)
        M_st = np.ascontiguousarray(M_st, dtype=np.float64)
        A_st = np.ascontiguousarray(A_st, dtype=np.float64)
        h = ctypes.c_void_p()
        check(lib().shifted_factor(int(n), dptr(M_st), dptr(A_st), cptr(lam), lam.size, int(precision),
                                   _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n, self.count, self.n_x, self.kd, self.precision = n, lam.size, (n - 1) ** 2, n, precision

    def solve(self, G, conj=False, out=None, stream=None):
        import torch
        _check_tensor(G, "G")
        squeeze = G.dim() == 2
        Gv = G.unsqueeze(0) if squeeze else G
        if tuple(Gv.shape[1:]) != (self.count, self.n_x):
            raise ValueError("expected shape [nrhs, %d, %d]" % (self.count, self.n_x))
        if out is None:
            out = torch.empty_like(Gv)
        check(lib().shifted_solve(self._h, ctypes.c_void_p(Gv.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  Gv.shape[0], int(bool(conj)), _stream(stream)))
        return out[0] if squeeze else out

    def factor_band(self, l):
        """Block l's factor as (kd+1) x n_x complex128: [d, j] = L[j+d][j], row 0 = D."""
        band = np.zeros(self.n_x * (self.kd + 1), np.complex128)
        check(lib().shifted_factor_band(self._h, int(l), cptr(band)))
        return band.reshape(self.n_x, self.kd + 1).T.copy()

    def close(self):
        if getattr(self, "_h", None):
            lib().shifted_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shifted_factor(n, M_st, A_st, lambdas, precision=64, stream=None):
    return ShiftedBlocks(n, M_st, A_st, lambdas, precision, stream)


def apply_spatial(n, M_st, A_st, alpha, beta, X, out=None, stream=None):
    """Y = (alpha M_x + beta A_x) X for X of shape [..., n_x] (complex128 cuda)."""
    import torch
    _check_tensor(X, "X")
    nx = (n - 1) ** 2
    if X.shape[-1] != nx:
        raise ValueError("last dimension must be n_x = %d" % nx)
    if out is None:
        out = torch.empty_like(X)
    count = X.numel() // nx
    M_st = np.ascontiguousarray(M_st, dtype=np.float64)
    A_st = np.ascontiguousarray(A_st, dtype=np.float64)
    alpha = complex(alpha)
    beta = complex(beta)
    check(lib().apply_spatial(int(n), dptr(M_st), dptr(A_st), alpha.real, alpha.imag, beta.real, beta.imag,
                              ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(out.data_ptr()), count, _stream(stream)))
    return out
