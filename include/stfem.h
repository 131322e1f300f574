/*
 * stfem.h -- C ABI of the MI355X space-time finite element solver for the
 * linear Schroedinger equation  i d_t psi - Lap_x psi = f  (Zank, "A Space-Time
 * Continuous Galerkin Finite Element Method for Linear Schroedinger
 * Equations").
 *
 * The library solves the global Galerkin system of Sec. 3, eq. (LGS),
 *
 *     K psi = f,    K = i B_t (x) M_x + M_t (x) A_x,
 *
 * by the fast diagonalization method of Sec. 3 (second choice of the temporal
 * decomposition): the temporal pencil is diagonalised on the host in FP64,
 * M_t^{-1} (i B_t) = X diag(lambda) X^{-1}, and then on the GPU
 *
 *     G   = W F,                         W = (M_t X)^{-1}    (rhs transform)
 *     u_l = (lambda_l M_x + A_x)^{-1} g_l  for every l        (spatial solves)
 *     Psi = X U                                               (back-transform)
 *
 * which is the paper's psi = (X_t (x) I)(I (x) M_x + S_t (x) A_x)^{-1}(Y_t (x) I) f
 * with S_t = diag(1/lambda), rescaled block by block.  The spatial solves use a
 * batched banded complex-symmetric LDL^T factorisation, in complex FP32 (with
 * FP64 iterative refinement on the global Kronecker residual) or complex FP64.
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved (re, im) pairs of doubles (complex128).
 *  - A space-time array is time-major: element (l, k) of an n_t x n_x array
 *    sits at offset l*n_x + k (Sec. 3: psi = (g_1, ..., g_{n_t}), g_l in C^{n_x}).
 *    A batch of nrhs such arrays is stored contiguously, [nrhs][n_t][n_x].
 *  - Spatial unknowns are the interior vertices of the unit square cut into
 *    n x n cells, each split by its lower-left to upper-right diagonal; vertex
 *    (i, j), 1 <= i, j <= n-1, is unknown k = (j-1)(n-1) + (i-1); n_x = (n-1)^2.
 *  - Temporal unknowns are the continuous Pp (p = 1, 2) Lagrange dofs on the
 *    nodes 0 = t_0 < ... < t_N = T in position order, without the dof at t_0
 *    (Sec. 3: homogenised unknown with zero initial value); n_t = p N.
 *  - "Device" pointers are HIP device allocations owned by the caller; the
 *    library never frees them.  "Host" pointers are ordinary memory.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.  GPU
 *    work is enqueued on it; entry points that must read a result back (the
 *    refinement loop) synchronise that stream.
 *  - Every int-returning entry point returns STFEM_OK (0) or a negative
 *    status; stfem_last_error() then describes the failure of the calling
 *    thread's last call.  No C++ exception crosses this interface.
 */
#ifndef STFEM_H
#define STFEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum stfem_status {
    STFEM_OK = 0,
    STFEM_EINVAL = -1,      /* invalid argument (size, pointer, option) */
    STFEM_ENOMEM = -2,      /* device or host allocation failed */
    STFEM_EHIP = -3,        /* a HIP runtime call failed */
    STFEM_ENOTDIAG = -4,    /* temporal eigen-decomposition failed or X singular */
    STFEM_ENOCONV = -5,     /* refinement did not reach the requested tolerance */
    STFEM_EBREAKDOWN = -6   /* zero or non-finite pivot in a spatial factorisation */
};

/* Spatial stencil coefficient order used by assemble_2d_space and the solver:
 * centre, east (+x), west (-x), north (+y), south (-y), north-east, south-west. */
enum { STFEM_ST_C = 0, STFEM_ST_E, STFEM_ST_W, STFEM_ST_N, STFEM_ST_S, STFEM_ST_NE, STFEM_ST_SW, STFEM_ST_COUNT };

/* Refinement of fdm_solve / fdm_solve_adjoint.  Both form every residual in
 * FP64 with the Kronecker matvec and precondition with the factored FDM
 * inverse (FP32 or FP64 factors):
 *  - STFEM_REFINE_GMRES: flexible GMRES, restarted after `restart` (at most
 *    23, fewer if the basis would exceed 16 GiB) applications of the inverse,
 *    with classical Gram-Schmidt applied twice; each cycle ends with a
 *    recomputed residual;
 *  - STFEM_REFINE_PLAIN: classical iterative refinement,
 *    Psi <- Psi + FDM^{-1} (F - K Psi);
 *  - STFEM_REFINE_BLOCK: GMRES on every block system S_l u_l = g_l in the
 *    eigen-coordinates g = W F (Sec. 3: K = (M_t X (x) I) blockdiag(S_l)
 *    (X^{-1} (x) I), so the transformed operator is block diagonal), with
 *    FP64 block residuals and one forward and one back transform per round;
 *    each block is driven to tol ||F|| / (||M_t X||_2 sqrt(n_t)) (adjoint:
 *    ||X^{-1}||_2), the global residual is then checked, and at most three
 *    rounds run.  This is how chunked factors are always refined.
 * GMRES contracts much faster when a few spatial blocks are ill conditioned
 * in FP32, because their error lives in a few directions that the Krylov
 * space removes. */
enum { STFEM_REFINE_GMRES = 0, STFEM_REFINE_PLAIN = 1, STFEM_REFINE_BLOCK = 2 };

typedef struct stfem_options {
    int precision;      /* 32: complex FP32 factors and sweeps, FP64 refinement;
                           64: complex FP64 factors and sweeps                     */
    int max_iter;       /* applications of the FDM inverse beyond the first (>= 0) */
    double tol;         /* target ||F - K Psi||_2 / ||F||_2, per right-hand side;
                           <= 0 disables the residual check (single pass)          */
    int refine;         /* STFEM_REFINE_GMRES (0, default), _PLAIN or _BLOCK       */
    int restart;        /* GMRES: applications of the inverse per cycle before a
                           restart; 0 = automatic (1 + max_iter, at most 23)       */
    double factor_budget; /* bytes of device memory for factor storage; 0 = the
                           free memory less the solve workspaces.  When the
                           factors of all n_t blocks exceed it, fdm_factor keeps
                           storage for one chunk of eigen-indices and every
                           solve factors the chunks again, one after the other */
} stfem_options;

typedef struct stfem_report {
    int iterations;         /* applications of the FDM inverse beyond the first   */
    double rel_residual;    /* max over rhs of ||F - K Psi||_2 / ||F||_2 (FP64)   */
    double kappa_x;         /* estimate of kappa_2(X), unit 2-norm columns        */
    double ms_eig;          /* host temporal eigen-step (fdm_factor)              */
    double ms_factor;       /* band fill + LDL^T + uploads, wall (fdm_factor)     */
    double ms_total;        /* wall time of the call                              */
    /* GPU time of single kernels measured with HIP events on the call's
     * stream: of the factorisation in fdm_factor, and summed over this call */
    double ms_band_fill;    /* band fill kernel (fdm_factor)                      */
    double ms_ldlt;         /* LDL^T kernel (fdm_factor)                          */
    double ms_sweeps;       /* all sweep kernels of this call                     */
    double ms_transforms;   /* all temporal-transform GEMM kernels of this call   */
    double ms_residual;     /* all residual kernels of this call                  */
    double history[16];     /* relative residual after each of the first 16
                               applications of the inverse (GMRES: its own
                               estimate; chunked factors: after each round;
                               unused entries are -1)                              */
    int chunks;             /* chunks of eigen-indices the factors were computed in
                               (1: all blocks factored once in fdm_factor)         */
} stfem_report;

typedef struct stfem_handle stfem_handle;   /* FDM solver: X, W, lambda, factors */
typedef struct stfem_blocks stfem_blocks;   /* batch of factored shifted spatial blocks */

/* ---------------------------------------------------------------- assembly */

/* Temporal matrices of Sec. 3, eq. (matrix_t), for continuous Pp Lagrange
 * elements (p = 1 or 2) on the n_el+1 host nodes t_nodes (t_nodes[0] = 0,
 * strictly increasing).  Row = test function, column = trial function:
 *   M_t[k][j] = int phi_j phi_k dt,   B_t[k][j] = int phi_j' phi_k dt,
 * with the dof at t_0 removed; n_t = p*n_el.  Outputs are caller-allocated
 * host arrays: M_t, B_t are n_t x n_t row-major; m_col0, b_col0 (length n_t,
 * may be NULL) are the couplings M_full[k][0], B_full[k][0] of each remaining
 * test function to the removed t_0 trial function, used to lift psi_0. */
int assemble_1d_time(int n_el, const double* t_nodes, int p,
                     double* M_t, double* B_t, double* m_col0, double* b_col0);

/* Spatial P1 matrices of Sec. 3, eq. (matrix_x), on the right-diagonal mesh
 * with n >= 2 cells per side, as 7-point stencils in the STFEM_ST_* order
 * (host arrays of 7 doubles each).  Couplings that would cross the boundary
 * are simply absent.  n_x (may be NULL) receives (n-1)^2 and kd (may be NULL)
 * the half-bandwidth n of the lexicographic ordering. */
int assemble_2d_space(int n, double* M_stencil, double* A_stencil, int* n_x, int* kd);

/* ------------------------------------------------------------------ FDM path */

/* Host-only temporal step of fast diagonalization (Sec. 3, solver step 1):
 * M_t^{-1} (i B_t) = X diag(lambda) X^{-1} with unit 2-norm columns of X and
 * W = (M_t X)^{-1}; eigenvalues in ascending order of real part (then
 * imaginary part).  The paper's decomposition (i B_t)^{-1} M_t = X_t S_t X_t^{-1}
 * has X_t = X and S_t = diag(1/lambda).  M_t, B_t: host n_t x n_t row-major,
 * banded with bandwidth <= 4.  Outputs (host, caller-allocated, any may be
 * NULL): lambda complex128[n_t]; X, W complex128[n_t*n_t] row-major; kappa =
 * estimate of kappa_2(X) (power iterations); iters = simultaneous-iteration
 * sweeps taken.  No GPU is used.  Errors: EINVAL, ENOTDIAG. */
int fdm_temporal(const double* M_t, const double* B_t, int n_t, double* lambda, double* X, double* W,
                 double* kappa, int* iters);

/* Factor the Kronecker system for fast diagonalization (Sec. 3, solver step 1
 * with the eigenvalue decomposition, then the spatial factorisations of step 3).
 *  M_t, B_t : host n_t x n_t row-major temporal matrices (banded; bandwidth
 *             is detected; at most 2).
 *  M_stencil, A_stencil : host 7-point spatial stencils (see assemble_2d_space)
 *             for n cells per side.
 *  opt      : precision 32 or 64, refinement settings used by fdm_solve.
 * Host FP64: eigenvalues of M_t^{-1} i B_t by simultaneous (Aberth) iteration,
 * right and left eigenvectors by inverse iteration, X (unit 2-norm columns),
 * W = (M_t X)^{-1} from the biorthogonality of left and right eigenvectors.
 * GPU: lambda_l M_x + A_x written in band storage and factored as L D L^T
 * (no pivoting; every leading minor is nonzero because Im lambda_l > 0).
 * Synchronises `stream` before returning.  On success *out owns all device
 * memory (release with fdm_destroy).  Errors: EINVAL, ENOMEM, EHIP, ENOTDIAG
 * (eigen-iteration failed), EBREAKDOWN (zero/non-finite pivot). */
int fdm_factor(const double* M_t, const double* B_t, int n_t,
               const double* M_stencil, const double* A_stencil, int n,
               const stfem_options* opt, void* stream, stfem_handle** out);

/* Solve K Psi = F for nrhs right-hand sides.  F_dev, Psi_dev: device
 * complex128 [nrhs][n_t][n_x]; they must not overlap.  One application of the
 * FDM inverse is G = W F, batched sweeps, Psi = X U.  With opt.tol > 0 the
 * solve is refined (opt.refine) until the FP64 relative residual of every rhs
 * is <= opt.tol or 1 + opt.max_iter inverses were applied.  The GMRES
 * refinement allocates its Krylov basis on the first call that needs it (at
 * most 2 KRYLOV_MAX vectors of nrhs n_t n_x complex128, capped at 16 GiB) and
 * keeps it with the handle.  rep (may be NULL) receives statistics.  Returns
 * ENOCONV (Psi still holds the last iterate) if tol was not met. */
int fdm_solve(stfem_handle* h, const void* F_dev, void* Psi_dev, int nrhs,
              void* stream, stfem_report* rep);

/* Adjoint solve K^H Lam = G with the same factors (K^H = -i B_t^T (x) M_x +
 * M_t^T (x) A_x):  Lam = W^H S^{-H} X^H G, where S_l^H = conj(S_l) because
 * every spatial block is complex symmetric, so the sweeps run on conjugated
 * factors.  Same layout, refinement and errors as fdm_solve. */
int fdm_solve_adjoint(stfem_handle* h, const void* G_dev, void* Lam_dev, int nrhs,
                      void* stream, stfem_report* rep);

/* Y = K Psi (adjoint = 0) or Y = K^H Psi (adjoint = 1) in FP64 on the GPU:
 * the Kronecker matvec of Sec. 3, eq. (LGS) used for refinement residuals. */
int fdm_apply(stfem_handle* h, const void* Psi_dev, void* Y_dev, int nrhs, int adjoint, void* stream);

/* Copy the host-side temporal decomposition out of a handle: lambda (n_t
 * complex128), X and W (n_t x n_t complex128 row-major), kappa estimate.
 * Any output pointer may be NULL. */
int fdm_decomposition(const stfem_handle* h, double* lambda, double* X, double* W, double* kappa);

/* Sizes of a handle: n_t, n_x, n, precision (any may be NULL). */
int fdm_sizes(const stfem_handle* h, int* n_t, int* n_x, int* n, int* precision);

void fdm_destroy(stfem_handle* h);

/* ------------------------------------------------- batched shifted blocks */

/* Factor count complex-shifted spatial blocks S_l = lambda_l M_x + A_x (the
 * spatial problems of Sec. 3, eq. (LGS_x), in the scaling lambda = 1/S_t[l,l])
 * as S_l = L_l D_l L_l^T with unit lower-triangular L_l of half-bandwidth
 * kd = n, in complex FP32 (precision 32) or FP64 (precision 64).
 * lambda: host complex128[count]; every Im lambda_l must be > 0 (this is what
 * makes the factorisation without pivoting exist).  Enqueued on `stream` and
 * synchronised (the pivot check reads a flag back).  Errors: EINVAL, ENOMEM,
 * EHIP, EBREAKDOWN. */
int shifted_factor(int n, const double* M_stencil, const double* A_stencil,
                   const double* lambda, int count, int precision, void* stream,
                   stfem_blocks** out);

/* U_l = S_l^{-1} G_l (conj = 0) or U_l = S_l^{-H} G_l = conj(S_l)^{-1} G_l
 * (conj = 1) for every block l and rhs r.  G_dev, U_dev: device complex128
 * [nrhs][count][n_x]; U may alias G.  Computed in the factor precision and
 * returned in FP64.  Enqueued on `stream`, not synchronised. */
int shifted_solve(stfem_blocks* b, const void* G_dev, void* U_dev, int nrhs, int conj, void* stream);

/* Copy block l's factor out to the host in FP64: band[j*(kd+1)+d] = L[j+d][j]
 * for d = 1..kd and band[j*(kd+1)] = D[j]  (complex128, (kd+1)*n_x). */
int shifted_factor_band(const stfem_blocks* b, int l, double* band);

void shifted_destroy(stfem_blocks* b);

/* ------------------------------------------------------------ spatial apply */

/* Y_r = (alpha M_x + beta A_x) X_r for count vectors of n_x complex128 values
 * (device), with 7-point stencils for n cells per side; alpha, beta complex
 * given as (re, im).  Used to lift psi_0 (Sec. 3, homogenisation) and to
 * evaluate space-time L2 functionals.  Enqueued on `stream`. */
int apply_spatial(int n, const double* M_stencil, const double* A_stencil,
                  double alpha_re, double alpha_im, double beta_re, double beta_im,
                  const void* X_dev, void* Y_dev, int count, void* stream);

/* Factor storage (tens of GB) released by fdm_destroy / shifted_destroy is
 * kept by the library, at most two buffers per device, and reused by later
 * factorisations that fit; this returns all of it to the device.  Not to be
 * called while another thread is inside the library. */
void stfem_release_cache(void);

/* ------------------------------------------------------------------ errors */
const char* stfem_strerror(int status);
const char* stfem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STFEM_H */
