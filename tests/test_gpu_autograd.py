"""Gradients of the tracking functional J = 1/2 ||psi_h - psi_target||^2_{L2(Q)}
with respect to the load vector F and the initial value psi_0, through the
differentiable solve (adjoint solve in the backward pass): central finite
differences on seeded directions and the oracle's dense adjoint."""
import numpy as np
import pytest
import torch

import paper_2504_07269_amd as st
from paper_2504_07269_amd import autograd as ad
import synth
from oracle import fem, problems, solvers
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def setup(n, N_t, T=1.0, precision=64, tol=1e-13):
    nodes = synth.uniform_nodes(T, N_t)
    Mt, Bt, m0, b0 = st.assemble_1d_time(nodes, 1)
    Ms, As, n_x, _ = st.assemble_2d_space(n)
    Mf, _ = fem.assemble_time_full(nodes, 1)
    h = st.fdm_factor(Mt, Bt, Ms, As, n, precision=precision, tol=tol, max_iter=20)
    return nodes, Mt, Bt, m0, b0, Ms, As, Mf, h


def J_of(h, F, psi0, n, Ms, As, m0, b0, Mf, target):
    psi = ad.solve_with_initial_value(h, F, psi0, n, Ms, As, m0, b0)
    return 0.5 * ad.l2q_norm_sq(psi - target, n, Ms, As, Mf)


def test_gradient_matches_dense_adjoint_small():
    n, N_t = 16, 16
    nodes, Mt, Bt, m0, b0, Ms, As, Mf, h = setup(n, N_t)
    Mx, Ax = fem.assemble_space(n)
    prob = problems.OmegaSolution(np.pi)
    F = fem.load_vector(prob.f, n, nodes, 1)[1:]
    psi0 = synth.psi0_nodal(n)
    target = synth.smooth_targets(n, nodes, [100])[0]
    Ft = to_dev(F).requires_grad_(True)
    p0 = to_dev(psi0).requires_grad_(True)
    J = J_of(h, Ft, p0, n, Ms, As, m0, b0, Mf, to_dev(target))
    J.backward()
    gF, gp = to_host(Ft.grad), to_host(p0.grad)
    # oracle: psi_hat = K^{-1}(F - lift psi0); e = [psi0; psi_hat] - target;
    # dJ/dconj(e) = (Mf (x) Mx) e; grad_F = 2 K^{-H} (Mf (x) Mx) e |_{rows 1..}
    Fh = F - (1j * np.outer(b0, Mx @ psi0) + np.outer(m0, Ax @ psi0))
    psi_hat = solvers.solve_dense(Mt, Bt, Mx, Ax, Fh)
    e = np.concatenate([psi0[None], psi_hat]) - target
    Me = Mf @ (Mx @ e.T).T
    lam = solvers.solve_dense_adjoint(Mt, Bt, Mx, Ax, Me[1:])
    ref_gF = lam                                        # PyTorch: grad = 2 dJ/dconj(z) = K^{-H} Me
    ref_gp = Me[0] - (Mx @ (-1j * b0[0] * lam[0]) + Ax @ (m0[0] * lam[0]))
    assert np.linalg.norm(gF - ref_gF) / np.linalg.norm(ref_gF) < 1e-11
    assert np.linalg.norm(gp - ref_gp) / np.linalg.norm(ref_gp) < 1e-11


def test_gradient_central_differences_c3():
    """n=128, N_t=128, batch of 8 targets, 20 seeded directions, step 1e-6."""
    wl = synth.WORKLOADS["c3"]
    n = wl.n
    # J is evaluated with the single-pass FP64 solve (no residual-driven
    # refinement), an exactly fixed linear map, so that central differences
    # of the quadratic J see only rounding.
    nodes, Mt, Bt, m0, b0, Ms, As, Mf, h = setup(n, wl.N_t, wl.T, tol=0.0)
    targets = to_dev(synth.smooth_targets(n, nodes, list(range(100, 108))))
    F0 = synth.manufactured_rhs(wl, homogenised=False)
    psi0 = synth.psi0_nodal(n)
    Fb = to_dev(np.broadcast_to(F0, (8,) + F0.shape)).requires_grad_(True)
    pb = to_dev(np.broadcast_to(psi0, (8, psi0.size))).requires_grad_(True)
    J = J_of(h, Fb, pb, n, Ms, As, m0, b0, Mf, targets)
    J.sum().backward()
    gF, gp = to_host(Fb.grad), to_host(pb.grad)
    dirs_F = synth.unit_directions(range(200, 220), Fb.shape)
    dirs_p = synth.unit_directions(range(300, 320), pb.shape)
    eps = 1e-6
    with torch.no_grad():
        for dF, dp in zip(dirs_F, dirs_p):
            Jp = J_of(h, Fb + eps * to_dev(dF), pb + eps * to_dev(dp), n, Ms, As, m0, b0, Mf, targets).sum().item()
            Jm = J_of(h, Fb - eps * to_dev(dF), pb - eps * to_dev(dp), n, Ms, As, m0, b0, Mf, targets).sum().item()
            fd = (Jp - Jm) / (2 * eps)
            an = np.vdot(gF, dF).real + np.vdot(gp, dp).real
            # J is quadratic: central differences are exact up to rounding ~ u |J| / eps
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-300) + 4e-16 * abs(J.sum().item()) / eps, (fd, an)
