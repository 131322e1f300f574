"""Space-time error norms (Sec. 4, definitions before Table 1); test
infrastructure only.

||e||_{L2(Q)} and |e|_{H1(Q)} = (||d_t e||^2 + ||grad_x e||^2)^{1/2} of
e = psi - psi_h, by quadrature on every prism (triangle x time element).
psi_h is given by its nodal values at every temporal dof (t_0 included) and
every interior vertex; boundary values are zero.
"""
import numpy as np

from .fem import _affine, _p1_reference, full_vertex_field, lagrange_1d, square_mesh
from .quadrature import gauss_legendre, triangle_rule


def errors(problem, Uh_full, n, nodes, p, m_space=4, m_time=None):
    """Returns (L2 error, H1 seminorm error)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    if m_time is None:
        m_time = p + 3
    verts, tris, _ = square_mesh(n)
    Uv = full_vertex_field(Uh_full, n)                       # (pN+1, V)
    pts, wts = triangle_rule(m_space)
    lam, gref = _p1_reference(pts)
    P0, J, det = _affine(verts, tris)
    Jinv = np.linalg.inv(J)
    G = np.einsum("eji,aj->eai", Jinv, gref)                 # (E,3,2) physical gradients
    X = P0[:, None, 0] + J[:, 0, 0][:, None] * pts[None, :, 0] + J[:, 0, 1][:, None] * pts[None, :, 1]
    Y = P0[:, None, 1] + J[:, 1, 0][:, None] * pts[None, :, 0] + J[:, 1, 1][:, None] * pts[None, :, 1]
    wsp = np.abs(det)[:, None] * wts[None, :]
    tq, tw = gauss_legendre(m_time)
    phit, dphit = lagrange_1d(p, tq)
    N = nodes.size - 1
    l2 = 0.0
    h1 = 0.0
    for e in range(N):
        h = nodes[e + 1] - nodes[e]
        loc = Uv[p * e: p * e + p + 1]                       # (p+1, V)
        for q in range(m_time):
            t = nodes[e] + h * tq[q]
            ut = phit[:, q] @ loc                            # psi_h(., t) at vertices
            dut = (dphit[:, q] @ loc) / h                    # d_t psi_h(., t)
            vt = ut[tris]                                    # (E, 3)
            dvt = dut[tris]
            uh = vt @ lam                                    # (E, q)
            duh = dvt @ lam
            gh = np.einsum("ea,eai->ei", vt, G)              # (E, 2), constant per element
            ex = problem.psi(X, Y, t) - uh
            edt = problem.dt(X, Y, t) - duh
            gx, gy = problem.grad(X, Y, t)
            egx = gx - gh[:, 0:1]
            egy = gy - gh[:, 1:2]
            w = h * tw[q] * wsp
            l2 += np.sum(w * np.abs(ex) ** 2)
            h1 += np.sum(w * (np.abs(edt) ** 2 + np.abs(egx) ** 2 + np.abs(egy) ** 2))
    return np.sqrt(l2), np.sqrt(h1)


def eoc(errs):
    """Experimental orders of convergence for a sequence halving h each time."""
    errs = np.asarray(errs, dtype=np.float64)
    return np.log(errs[:-1] / errs[1:]) / np.log(2.0)
