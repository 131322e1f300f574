"""Solvers for the global space-time system (test infrastructure only).

Unknowns are ordered in n_t blocks of n_x spatial values (Sec. 3, step 2 of the
Kronecker solver), so a space-time vector is stored as an n_t x n_x array U
with vec(U) = U.ravel() and (A kron B) vec(U) = vec(A U B^T).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def global_matrix(Mt, Bt, Mx, Ax):
    """K = i B_t kron M_x + M_t kron A_x (Sec. 3, eq. (LGS)), sparse CSR."""
    Mt = sp.csr_matrix(Mt)
    Bt = sp.csr_matrix(Bt)
    return (1j * sp.kron(Bt, Mx) + sp.kron(Mt, Ax)).tocsr()


def apply_global(Mt, Bt, Mx, Ax, U):
    """K vec(U) as an n_t x n_x array, from the sparse Kronecker product."""
    K = global_matrix(Mt, Bt, Mx, Ax)
    return (K @ U.ravel()).reshape(U.shape)


def solve_dense(Mt, Bt, Mx, Ax, F):
    """Dense LU of the assembled global matrix (small problems only)."""
    K = global_matrix(Mt, Bt, Mx, Ax).toarray()
    return np.linalg.solve(K, F.ravel()).reshape(F.shape)


def solve_dense_adjoint(Mt, Bt, Mx, Ax, G):
    """Dense solve with K^H = -i B_t^T kron M_x + M_t^T kron A_x."""
    K = global_matrix(Mt, Bt, Mx, Ax).toarray()
    return np.linalg.solve(K.conj().T, G.ravel()).reshape(G.shape)


def solve_sparse(Mt, Bt, Mx, Ax, F):
    """Sparse direct solve of the global system (SuperLU)."""
    K = global_matrix(Mt, Bt, Mx, Ax).tocsc()
    return spla.spsolve(K, F.ravel()).reshape(F.shape)


def apply_global_structured(Mt, Bt, Mx, Ax, U):
    """K vec(U) = vec(i B_t U M_x^T + M_t U A_x^T) without forming the
    Kronecker product (for large problems).  U: (n_t, n_x) or (k, n_t, n_x)."""
    U = np.asarray(U)
    if U.ndim == 3:
        return np.stack([apply_global_structured(Mt, Bt, Mx, Ax, u) for u in U])
    UM = (sp.csr_matrix(Mx) @ U.T).T
    UA = (sp.csr_matrix(Ax) @ U.T).T
    return 1j * (sp.csr_matrix(Bt) @ UM) + sp.csr_matrix(Mt) @ UA


def fdm_paper(Mt, Bt, Mx, Ax, F, return_parts=False):
    """Fast diagonalisation, exactly in the paper's form (Sec. 3, solver steps
    1-4 with the eigenvalue decomposition as the second choice of X_t, S_t):

      1. (i B_t)^{-1} M_t = X_t S_t X_t^{-1}, S_t diagonal, X_t eigenvectors
         (unit 2-norm columns);
      2. g = (Y_t kron I) f with Y_t = X_t^{-1} (i B_t)^{-1};
      3. (M_x + S_t[l,l] A_x) w_l = g_l for every l, independently;
      4. psi = (X_t kron I) w.
    F may hold several right-hand sides, shape (k, n_t, n_x); each spatial
    matrix is then factored once for all of them.
    """
    F = np.asarray(F)
    multi = F.ndim == 3
    Fs = F if multi else F[None]
    iB = 1j * np.asarray(Bt, dtype=np.complex128)
    Mt = np.asarray(Mt, dtype=np.float64)
    A = np.linalg.solve(iB, Mt)
    mu, X = np.linalg.eig(A)
    X = X / np.linalg.norm(X, axis=0)
    Y = np.linalg.solve(X, np.linalg.inv(iB))
    G = np.einsum("lm,kmx->klx", Y, Fs)
    Wb = np.empty_like(G)
    Mx = sp.csc_matrix(Mx)
    Ax = sp.csc_matrix(Ax)
    for l in range(G.shape[1]):
        lu = spla.splu((Mx + mu[l] * Ax).tocsc())
        for k in range(G.shape[0]):
            Wb[k, l] = lu.solve(np.ascontiguousarray(G[k, l]))
    psi = np.einsum("lm,kmx->klx", X, Wb)
    if not multi:
        psi = psi[0]
    if return_parts:
        return psi, dict(mu=mu, X=X, Y=Y)
    return psi


def bartels_stewart_paper(Mt, Bt, Mx, Ax, F):
    """Bartels-Stewart in the paper's form (Sec. 3, first choice of X_t, S_t):
    complex Schur (i B_t)^{-1} M_t = X_t S_t X_t^H with X_t unitary and S_t
    upper triangular, then the spatial problems of eq. (LGS_x) for
    l = n_t, ..., 1, each with the accumulated right-hand side."""
    iB = 1j * np.asarray(Bt, dtype=np.complex128)
    A = np.linalg.solve(iB, np.asarray(Mt, dtype=np.complex128))
    S, X = sla.schur(A, output="complex")
    Y = X.conj().T @ np.linalg.inv(iB)
    G = Y @ F
    nt = G.shape[0]
    Mx = sp.csc_matrix(Mx)
    Ax = sp.csc_matrix(Ax)
    Wb = np.zeros_like(G)
    AW = np.zeros_like(G)           # A_x w_k, kept for the accumulated sums
    for l in range(nt - 1, -1, -1):
        rhs = G[l] - S[l, l + 1:] @ AW[l + 1:]
        lu = spla.splu((Mx + S[l, l] * Ax).tocsc())
        Wb[l] = lu.solve(rhs)
        AW[l] = Ax @ Wb[l]
    return X @ Wb


def temporal_eigvecs(Mt, Bt):
    """Eigenvalues mu and unit-2-norm eigenvectors X of (i B_t)^{-1} M_t."""
    A = np.linalg.solve(1j * np.asarray(Bt, dtype=np.complex128), np.asarray(Mt, dtype=np.complex128))
    mu, X = np.linalg.eig(A)
    return mu, X / np.linalg.norm(X, axis=0)


def kappa2_Xt(Mt, Bt):
    """Spectral condition number kappa_2(X_t) (Sec. 4, Tables 2-3)."""
    _, X = temporal_eigvecs(Mt, Bt)
    return np.linalg.cond(X)


def block_solve(Mx, Ax, lam, G):
    """Shifted spatial solves (lam_l M_x + A_x) u_l = g_l, one sparse LU each."""
    Mx = sp.csc_matrix(Mx)
    Ax = sp.csc_matrix(Ax)
    U = np.empty(G.shape, dtype=np.complex128)
    for l in range(G.shape[0]):
        U[l] = spla.splu((lam[l] * Mx + Ax).tocsc()).solve(np.ascontiguousarray(G[l]))
    return U


def lift_constant(F_full, psi0_nodal, Mt_full, Ax):
    """Homogenisation with psi_0 constant in time (Sec. 3):
    F_hat = <f, v> - a(psi_0, v).  Since d_t psi_0 = 0 only the stiffness term
    survives: a(psi_0, phi_k varphi_l) = (int varphi_l dt) (A_x psi_0)_k.
    F_full has a row per temporal dof including t_0; the t_0 row is dropped."""
    tint = np.asarray(Mt_full).sum(axis=1)         # int varphi_l dt (partition of unity)
    Apsi = Ax @ psi0_nodal
    return F_full[1:] - np.outer(tint[1:], Apsi)


def relres(Mt, Bt, Mx, Ax, U, F):
    """||F - K vec(U)||_2 / ||F||_2 with the sparse Kronecker matvec."""
    R = F - apply_global(Mt, Bt, Mx, Ax, U)
    return np.linalg.norm(R) / np.linalg.norm(F)
