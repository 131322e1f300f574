"""Differentiable space-time solve for gradients of tracking functionals.

The unknowns of the Galerkin system (Sec. 3, eq. (VF_FEM)) are psi_hat_h with
zero initial value; psi_h = psi_hat_h + psi_0 lifts the initial datum.  Here
the lift uses the nodal hat function of t_0 in time: psi_h = psi_tilde +
psi_0 varphi_0 with psi_tilde in the homogeneous space, which changes only the
temporal rows coupled to t_0,

    F_hat[l] = F[l] - (i b_col0[l] M_x + m_col0[l] A_x) psi_0,

and gives the same psi_h as lifting with psi_0 constant in time (both are the
unique discrete solution with psi_h(0) = psi_0).  psi_h at t_0 is psi_0 and at
the remaining temporal dofs it is psi_tilde.

Gradients follow PyTorch's convention for complex inputs: for y = A x the
backward of x receives A^H grad(y).  The backward of the solve is the adjoint
solve K^H lam = grad(psi) with the same factors.
"""
import numpy as np
import torch

from . import FDM, apply_spatial


class FDMSolveFn(torch.autograd.Function):
    """psi = K^{-1} F with backward grad_F = K^{-H} grad_psi."""

    @staticmethod
    def forward(ctx, F, handle):
        ctx.handle = handle
        return handle.solve(F.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.handle.solve_adjoint(g.contiguous()), None


class SpatialApplyFn(torch.autograd.Function):
    """y = (alpha M_x + beta A_x) x on the last dimension; M_x, A_x real
    symmetric, so the backward is (conj(alpha) M_x + conj(beta) A_x) grad_y."""

    @staticmethod
    def forward(ctx, x, n, Ms, As, alpha, beta):
        ctx.args = (n, Ms, As, complex(alpha), complex(beta))
        return apply_spatial(n, Ms, As, alpha, beta, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        n, Ms, As, a, b = ctx.args
        return apply_spatial(n, Ms, As, a.conjugate(), b.conjugate(), g.contiguous()), None, None, None, None, None


def fdm_solve_diff(handle: FDM, F):
    """Differentiable psi_hat = K^{-1} F."""
    return FDMSolveFn.apply(F, handle)


def spatial_apply_diff(n, Ms, As, alpha, beta, x):
    return SpatialApplyFn.apply(x, n, Ms, As, alpha, beta)


def lift_rhs(F, psi0, n, Ms, As, m_col0, b_col0):
    """F_hat = F - (i b_col0 (x) M_x + m_col0 (x) A_x) psi_0 (differentiable in
    F and psi0).  F: [(nrhs,) n_t, n_x]; psi0: [(nrhs,) n_x]."""
    rows = [int(l) for l in np.nonzero((np.asarray(m_col0) != 0) | (np.asarray(b_col0) != 0))[0]]
    corr = []
    for l in range(F.shape[-2]):
        if l in rows:
            corr.append(spatial_apply_diff(n, Ms, As, 1j * float(b_col0[l]), float(m_col0[l]), psi0))
        else:
            corr.append(torch.zeros_like(psi0))
    return F - torch.stack(corr, dim=-2)


def solve_with_initial_value(handle: FDM, F, psi0, n, Ms, As, m_col0, b_col0):
    """psi_h at every temporal dof including t_0: [(nrhs,) n_t + 1, n_x]."""
    psi_hat = fdm_solve_diff(handle, lift_rhs(F, psi0, n, Ms, As, m_col0, b_col0))
    return torch.cat([psi0.unsqueeze(-2), psi_hat], dim=-2)


def l2q_norm_sq(e, n, Ms, As, Mt_full):
    """||e_h||^2_{L2(Q)} = e^H (M_t_full (x) M_x) e for nodal values e at every
    temporal dof including t_0 (shape [(nrhs,) n_t + 1, n_x])."""
    Me = spatial_apply_diff(n, Ms, As, 1.0, 0.0, e)
    Mt = torch.as_tensor(Mt_full, dtype=e.dtype, device=e.device)
    MMe = torch.matmul(Mt, Me)
    return torch.sum((e.conj() * MMe).real, dim=(-2, -1))
