// Launch wrappers of the HIP kernels (implemented in kernels.hip).  All
// pointers are device pointers; complex values are interleaved (re, im).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/stfem.h"

namespace stfem {
namespace gpu {

// 7-point stencils of M_x and A_x in STFEM_ST_* order for n cells per side.
struct Stencil {
    double M[7];
    double A[7];
    int n;      // cells per side
    int m;      // grid width n-1; n_x = m*m, kd = n = m+1
};

// Band storage of one block: band[j*(kd+1) + d] = S[j+d][j], d = 0..kd;
// blocks are band_stride() complex values apart.
// S_l = lambda_l M_x + A_x for l in [0, count); lambda: complex128[count].
inline long long band_stride_host(int n) {
    return (((long long)(n - 1) * (n - 1) * (n + 1)) + 63) / 64 * 64;
}
hipError_t band_fill(int precision, void* band, const double* lambda, int count, const Stencil& st,
                     hipStream_t s);

// In-place L D L^T of `count` bands; info[l] = 1 + first bad column (0 = ok).
hipError_t ldlt_factor(int precision, void* band, int count, const Stencil& st, int* info, hipStream_t s);

// U[r][l] = S_l^{-1} G[r][l] (conj: conj(S_l)^{-1}); G, U complex128
// [nrhs][count][n_x]; may alias.
hipError_t sweep_solve(int precision, const void* band, int count, const Stencil& st, const double* G,
                       double* U, int nrhs, int conj, hipStream_t s);

// C[b] = op(A) B[b] (+ C[b] if accumulate); A complex128 n x n row-major,
// op = A (trans = 0) or A^H (trans = 1); B[b], C[b] complex128 n x ncols
// row-major with batch strides strideB, strideC (in complex elements).
hipError_t zgemm_small_left(int n, int ncols, int batch, const double* A, int trans, const double* B,
                            long long strideB, double* C, long long strideC, int accumulate, hipStream_t s);

// R = F - K Psi (adjoint = 0) or F - K^H Psi (adjoint = 1), with
// K = i B_t (x) M_x + M_t (x) A_x; temporal matrices in band storage
// tM[l*(2w+1) + (m-l+w)], tB[...] (doubles).  Per-rhs squared norms of R and
// F are accumulated into norms[2*r], norms[2*r+1] (overwritten).
// Uses `partial` (>= residual_partial_size doubles) as scratch.
hipError_t kron_residual(const double* Psi, const double* F, double* R, int nrhs, int n_t, int w,
                         const double* tM, const double* tB, const Stencil& st, int adjoint,
                         double* partial, double* norms, hipStream_t s);
size_t residual_partial_size(int nrhs, int n_t, int n_x);

// Y = K Psi or K^H Psi (no F, no norms).
hipError_t kron_apply(const double* Psi, double* Y, int nrhs, int n_t, int w, const double* tM,
                      const double* tB, const Stencil& st, int adjoint, hipStream_t s);

// Y_v = (alpha M + beta A) X_v for `count` vectors of n_x.
hipError_t spatial_apply(const Stencil& st, double ar, double ai, double br, double bi, const double* X,
                         double* Y, int count, hipStream_t s);

// Krylov vectors of the refinement: complex128, nrhs slices of N elements;
// a basis of nv vectors vstride complex elements apart (nv <= KRYLOV_MAX).
// `partial` holds >= krylov_partial_size(nrhs) doubles of scratch.
constexpr int KRYLOV_MAX = 24;
constexpr int VEC_BLOCKS = 1024;
size_t krylov_partial_size(int nrhs);
// out[r][i] = <V_i[r], w[r]> = sum_e conj(V_i[r][e]) w[r][e]   (complex, device)
hipError_t vec_mdot(const double* V, long long vstride, int nv, const double* w, long long N, int nrhs,
                    double* partial, double* out, hipStream_t s);
// w[r] = (accumulate ? w[r] : 0) + sign sum_i coef[r][i] V_i[r]; coef complex
// [nrhs][nv] on the device; norms[r] = ||w[r]||^2 afterwards if norms != null.
hipError_t vec_mcomb(double* w, long long N, int nrhs, const double* V, long long vstride, int nv, const double* coef,
                     double sign, int accumulate, double* partial, double* norms, hipStream_t s);
// norms[r] = ||x[r]||^2
hipError_t vec_norm2(const double* x, long long N, int nrhs, double* partial, double* norms, hipStream_t s);
// y[r] = sc[r] x[r], sc real [nrhs] on the device; y may equal x
hipError_t vec_scale(double* y, const double* x, long long N, int nrhs, const double* sc, hipStream_t s);

// Shifted spatial blocks of a chunk, FP64: for systems s < nsys (each n_x
// complex128), l = l0 + s % cnt, S_l = lambda_l M + A (conj: conj(lambda_l));
// Y_s = S_l X_s, or Y_s = B_s - S_l X_s when B != null.  lambda: device
// complex128 of all eigen-indices.
hipError_t shifted_apply(const Stencil& st, const double* lambda, int l0, int cnt, int conj, const double* X,
                         double* Y, const double* B, int nsys, hipStream_t s);

// p[0..count) = value (a kernel, so that it may be recorded in a graph).
hipError_t fill_int(int* p, int count, int value, hipStream_t s);

}  // namespace gpu
}  // namespace stfem
