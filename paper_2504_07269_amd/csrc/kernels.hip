// HIP kernels (gfx950) of the fast-diagonalization space-time solver.
//
//  band_fill     S_l = lambda_l M_x + A_x in lower band storage        (Sec. 3, eq. (LGS_x))
//  ldlt          blocked right-looking L D L^T of every band, no pivoting
//  sweep         L y = g, z = D^{-1} y, L^T x = z for every block and rhs
//  zgemm         the temporal transforms G = W F and Psi = X U          (Sec. 3, steps 2 and 4)
//  kron_residual R = F - (i B_t (x) M_x + M_t (x) A_x) Psi                (Sec. 3, eq. (LGS))
//
// Band storage of a block: band[j*(kd+1) + d] = S[j+d][j], 0 <= d <= kd, for
// column j of the lower triangle; after factorisation d = 0 holds D_j and
// d >= 1 holds L[j+d][j].  Column-contiguous storage makes every access of the
// factorisation and of both sweeps coalesced along d.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace stfem {
namespace gpu {
namespace {

template <class R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <class R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a*b + c
template <class R>
__device__ __forceinline__ cpx<R> cfma(cpx<R> a, cpx<R> b, cpx<R> c) {
    c.x = fma(a.x, b.x, c.x);
    c.x = fma(-a.y, b.y, c.x);
    c.y = fma(a.x, b.y, c.y);
    c.y = fma(a.y, b.x, c.y);
    return c;
}
template <class R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) {
    return {a.x - b.x, a.y - b.y};
}
template <class R>
__device__ __forceinline__ cpx<R> cinv_or_zero(cpx<R> d, bool& ok) {
    const R dn = d.x * d.x + d.y * d.y;
    ok = (dn > R(0)) && isfinite(dn);
    if (!ok) return {R(0), R(0)};
    return {d.x / dn, -d.y / dn};
}
template <class R>
__device__ __forceinline__ cpx<R> shfl(cpx<R> v, int src) {
    return {__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}
template <class R>
__device__ __forceinline__ cpx<R> shfl_xor(cpx<R> v, int mask) {
    return {__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64)};
}

__device__ __forceinline__ long long band_elems(const Stencil& st) {
    return (long long)st.m * st.m * (st.n + 1);
}

// ------------------------------------------------------------------ band fill
template <class R>
__global__ __launch_bounds__(256) void k_band_fill(cpx<R>* __restrict__ band, const double* __restrict__ lam,
                                                   Stencil st) {
    const int l = blockIdx.y;
    const double lr = lam[2 * l], li = lam[2 * l + 1];
    const int m = st.m, ld = st.n + 1;
    const long long per = band_elems(st);
    cpx<R>* B = band + (size_t)l * per;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < per;
         e += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(e / ld), d = (int)(e - (long long)j * ld);
        const int jx = j % m, jy = j / m;
        int q = -1;
        if (d == 0)
            q = STFEM_ST_C;
        else if (d == 1 && jx < m - 1)
            q = STFEM_ST_E;
        else if (d == m && jy < m - 1)
            q = STFEM_ST_N;
        else if (d == m + 1 && jx < m - 1 && jy < m - 1)
            q = STFEM_ST_NE;
        cpx<R> v = {R(0), R(0)};
        if (q >= 0) v = {(R)(lr * st.M[q] + st.A[q]), (R)(li * st.M[q])};
        B[e] = v;
    }
}

// ---------------------------------------------------------------------- LDL^T
// One workgroup factors one band.  Panel of NB columns and its kd+NB rows in
// LDS (column-major P[c*LP + r], r relative to the panel start k); the panel
// is factored column by column, written back, and the trailing kd x kd lower
// triangle is updated in place in global memory:
//   A[i][j] -= sum_c L[i][c] D_c L[j][c].
template <class R, int NB>
__global__ __launch_bounds__(256) void k_ldlt(cpx<R>* __restrict__ band, Stencil st, int* __restrict__ info) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* P = reinterpret_cast<cpx<R>*>(smem_raw);
    const int m = st.m, kd = st.n, n_x = m * m, ld = kd + 1, LP = NB + kd;
    const int l = blockIdx.x;
    cpx<R>* A = band + (size_t)l * band_elems(st);
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
    int bad = 0;
    for (int k = 0; k < n_x; k += NB) {
        const int nb = min(NB, n_x - k);
        const int mrows = min(nb + kd, n_x - k);
        for (int e = tid; e < nb * mrows; e += nth) {
            const int c = e / mrows, r = e - c * mrows;
            cpx<R> v = {R(0), R(0)};
            if (r >= c && r - c <= kd) v = A[(size_t)(k + c) * ld + (r - c)];
            P[c * LP + r] = v;
        }
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            bool ok;
            const cpx<R> inv = cinv_or_zero(P[c * LP + c], ok);
            if (!ok && bad == 0) bad = k + c + 1;
            const int nr = mrows - (c + 1), ncol = nb - c - 1;
            for (int e = tid; e < ncol * nr; e += nth) {
                const int c2 = c + 1 + e / nr, r = c + 1 + e % nr;
                if (r < c2) continue;
                const cpx<R> lc2 = cmul(P[c * LP + c2], inv);
                P[c2 * LP + r] = csub(P[c2 * LP + r], cmul(P[c * LP + r], lc2));
            }
            __syncthreads();
            for (int r = c + 1 + tid; r < mrows; r += nth) P[c * LP + r] = cmul(P[c * LP + r], inv);
            __syncthreads();
        }
        for (int e = tid; e < nb * ld; e += nth) {
            const int c = e / ld, d = e - c * ld;
            if (c + d < mrows) A[(size_t)(k + c) * ld + d] = P[c * LP + c + d];
        }
        // trailing update: columns jl in [nb, mrows), rows il in [jl, mrows)
        // (relative to k), in items of 4 columns x 64 rows, round-robin over waves
        const int ncols = mrows - nb;
        const int ngroups = (ncols + 3) >> 2;
        int item = 0;
        for (int g = 0; g < ngroups; ++g) {
            const int jl0 = nb + 4 * g;
            const int nchunk = (mrows - jl0 + 63) >> 6;
            for (int q = 0; q < nchunk; ++q, ++item) {
                if (item % nwave != wave) continue;
                const int il = jl0 + 64 * q + lane;
                if (il >= mrows) continue;
                cpx<R> a[4];
                size_t idx[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jl = jl0 + u;
                    idx[u] = (size_t)(k + jl) * ld + (il - jl);
                    a[u] = (jl < mrows && il >= jl) ? A[idx[u]] : cpx<R>{R(0), R(0)};
                }
                cpx<R> acc[4] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
                const int j1 = min(jl0 + 1, mrows - 1), j2 = min(jl0 + 2, mrows - 1), j3 = min(jl0 + 3, mrows - 1);
                for (int c = 0; c < nb; ++c) {
                    const cpx<R>* Pc = P + c * LP;
                    const cpx<R> t = cmul(Pc[c], Pc[il]);     // D_c L[i][c]
                    acc[0] = cfma(t, Pc[jl0], acc[0]);
                    acc[1] = cfma(t, Pc[j1], acc[1]);
                    acc[2] = cfma(t, Pc[j2], acc[2]);
                    acc[3] = cfma(t, Pc[j3], acc[3]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jl = jl0 + u;
                    if (jl < mrows && il >= jl) A[idx[u]] = csub(a[u], acc[u]);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) info[l] = bad;
}

// ---------------------------------------------------------------------- sweeps
// One workgroup solves S_l x = g for up to 4 right-hand sides.  The rows that
// a panel of NB columns touches (kd+NB of them) live in an LDS ring of
// Sz = kd + 2 NB slots per rhs.  Forward, per panel: wave 0 solves the unit
// triangle of the diagonal NB x NB block with lane shuffles, then all threads
// apply the panel to the kd rows below (threads over rows, coalesced reads of
// L's columns).  Backward (L^T x = z), per panel from the bottom: all waves
// form the dot products of the panel columns with the finished x below
// (lanes over rows, wave reductions), then wave 0 solves the transposed
// diagonal triangle.  KS = ceil(kd / 256).
template <class R, int NB, int KS, bool CONJ>
__global__ __launch_bounds__(256) void k_sweep(const cpx<R>* __restrict__ band, Stencil st, const double* G,
                                               double* U, int nr, long long rstride) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = st.m, kd = st.n, n_x = m * m, ld = kd + 1;
    const int Sz = kd + 2 * NB;
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(smem_raw);   // Y[rh*Sz + slot]
    cpx<R>* S = Y + 4 * Sz;                           // S[rh*NB + c]
    const int l = blockIdx.x;
    const cpx<R>* L = band + (size_t)l * band_elems(st);
    const double2* g = reinterpret_cast<const double2*>(G) + (size_t)l * n_x;
    double2* u = reinterpret_cast<double2*>(U) + (size_t)l * n_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    auto ldL = [&](int row, int col) -> cpx<R> {   // L[row][col] (or D at row == col), 0 <= row-col <= kd
        cpx<R> v = L[(size_t)col * ld + (row - col)];
        if (CONJ) v.y = -v.y;
        return v;
    };

    // initial window: rows [0, min(NB + kd, n_x))
    {
        const int rows0 = min(NB + kd, n_x);
        for (int e = tid; e < nr * rows0; e += blockDim.x) {
            const int rh = e / rows0, i = e - rh * rows0;
            const double2 v = g[(size_t)rh * rstride + i];
            Y[rh * Sz + i % Sz] = {(R)v.x, (R)v.y};
        }
    }
    __syncthreads();

    // ------------------------------------------------------------- forward
    for (int k = 0; k < n_x; k += NB) {
        const int nb = min(NB, n_x - k);
        // prefetch this thread's panel rows for the update below
        cpx<R> Lr[KS][NB];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int i = k + nb + tid + 256 * s;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool in = (c < nb) && (i < n_x) && (i - (k + c) <= kd) && (tid + 256 * s < kd);
                Lr[s][c] = in ? ldL(i, k + c) : cpx<R>{R(0), R(0)};
            }
        }
        if (wave == 0) {
            const int r = lane;
            cpx<R> y[4];
            cpx<R> Lrow[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c)
                Lrow[c] = (r < nb && c < r && r - c <= kd) ? ldL(k + r, k + c) : cpx<R>{R(0), R(0)};
            const int slot = (k + min(r, nb - 1)) % Sz;
#pragma unroll
            for (int rh = 0; rh < 4; ++rh) y[rh] = (rh < nr) ? Y[rh * Sz + slot] : cpx<R>{R(0), R(0)};
#pragma unroll
            for (int c = 0; c < NB - 1; ++c) {
#pragma unroll
                for (int rh = 0; rh < 4; ++rh) {
                    const cpx<R> yc = shfl(y[rh], c);
                    if (r > c) y[rh] = csub(y[rh], cmul(Lrow[c], yc));   // Lrow[c] = 0 beyond nb
                }
            }
            if (r < nb) {
                bool ok;
                const cpx<R> dinv = cinv_or_zero(ldL(k + r, k + r), ok);
#pragma unroll
                for (int rh = 0; rh < 4; ++rh) {
                    if (rh < nr) {
                        Y[rh * Sz + slot] = y[rh];
                        const cpx<R> z = cmul(y[rh], dinv);
                        u[(size_t)rh * rstride + k + r] = make_double2((double)z.x, (double)z.y);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int t = tid + 256 * s, i = k + nb + t;
            if (t < kd && i < n_x) {
#pragma unroll
                for (int rh = 0; rh < 4; ++rh) {
                    if (rh < nr) {
                        cpx<R> acc = {R(0), R(0)};
#pragma unroll
                        for (int c = 0; c < NB; ++c)   // Lr[s][c] = 0 for c >= nb
                            acc = cfma(Lr[s][c], Y[rh * Sz + (k + c) % Sz], acc);
                        cpx<R>& yi = Y[rh * Sz + i % Sz];
                        yi = csub(yi, acc);
                    }
                }
            }
        }
        // rows entering the window for the next panel
        if (tid < NB * nr) {
            const int rh = tid / NB, a = tid - rh * NB;
            const int i = k + NB + kd + a;
            if (i < n_x) {
                const double2 v = g[(size_t)rh * rstride + i];
                Y[rh * Sz + i % Sz] = {(R)v.x, (R)v.y};
            }
        }
        __syncthreads();
    }

    // ------------------------------------------------------------ backward
    const int kb = ((n_x - 1) / NB) * NB;
    for (int k = kb; k >= 0; k -= NB) {
        const int nb = min(NB, n_x - k);
        // dot products of panel columns with the finished x below the panel
        for (int c = wave; c < nb; c += 4) {
            cpx<R> part[4] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
            const int col = k + c;
            const int ilast = min(col + kd, n_x - 1);
#pragma unroll
            for (int p = 0; p < 4 * KS; ++p) {
                const int i = k + nb + lane + 64 * p;
                if (i <= ilast) {
                    const cpx<R> lv = ldL(i, col);
#pragma unroll
                    for (int rh = 0; rh < 4; ++rh)
                        if (rh < nr) part[rh] = cfma(lv, Y[rh * Sz + i % Sz], part[rh]);
                }
            }
#pragma unroll
            for (int rh = 0; rh < 4; ++rh) {
                cpx<R> v = part[rh];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const cpx<R> o = shfl_xor(v, off);
                    v.x += o.x;
                    v.y += o.y;
                }
                if (lane == 0 && rh < nr) S[rh * NB + c] = v;
            }
        }
        __syncthreads();
        if (wave == 0) {
            const int r = lane;
            cpx<R> v[4];
            cpx<R> Lt[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c)
                Lt[c] = (r < nb && c > r && c < nb && c - r <= kd) ? ldL(k + c, k + r) : cpx<R>{R(0), R(0)};
#pragma unroll
            for (int rh = 0; rh < 4; ++rh) {
                v[rh] = {R(0), R(0)};
                if (rh < nr && r < nb) {
                    const double2 z = u[(size_t)rh * rstride + k + r];
                    v[rh] = csub(cpx<R>{(R)z.x, (R)z.y}, S[rh * NB + r]);
                }
            }
#pragma unroll
            for (int c = NB - 1; c >= 1; --c) {
#pragma unroll
                for (int rh = 0; rh < 4; ++rh) {
                    const cpx<R> xc = shfl(v[rh], c);
                    if (r < c) v[rh] = csub(v[rh], cmul(Lt[c], xc));   // Lt[c] = 0 for c >= nb
                }
            }
            if (r < nb) {
#pragma unroll
                for (int rh = 0; rh < 4; ++rh) {
                    if (rh < nr) {
                        Y[rh * Sz + (k + r) % Sz] = v[rh];
                        u[(size_t)rh * rstride + k + r] = make_double2((double)v[rh].x, (double)v[rh].y);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------- zgemm
// C = op(A) B with A n x n (small), B n x ncols, complex FP64.  64 x 64 output
// tile per workgroup, K step 16, 4 x 4 complex outputs per thread.
__global__ __launch_bounds__(256) void k_zgemm(int n, int ncols, const double2* __restrict__ A, int trans,
                                               const double2* __restrict__ B, long long sB, double2* C, long long sC,
                                               int accumulate) {
    __shared__ double2 As[16][64 + 1];
    __shared__ double2 Bs[16][64];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int c0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const double2* Bb = B + (size_t)blockIdx.z * sB;
    double2* Cb = C + (size_t)blockIdx.z * sC;
    double accr[4][4] = {}, acci[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += 16) {
        for (int e = tid; e < 1024; e += 256) {
            int kk, mm;
            double2 v = make_double2(0.0, 0.0);
            if (!trans) {
                mm = e >> 4;
                kk = e & 15;
                if (m0 + mm < n && k0 + kk < n) v = A[(size_t)(m0 + mm) * n + k0 + kk];
            } else {
                kk = e >> 6;
                mm = e & 63;
                if (m0 + mm < n && k0 + kk < n) {
                    v = A[(size_t)(k0 + kk) * n + m0 + mm];
                    v.y = -v.y;
                }
            }
            As[kk][mm] = v;
            const int bk = e >> 6, bc = e & 63;
            double2 bv = make_double2(0.0, 0.0);
            if (k0 + bk < n && c0 + bc < ncols) bv = Bb[(size_t)(k0 + bk) * ncols + c0 + bc];
            Bs[bk][bc] = bv;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            double2 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    accr[i][j] = fma(a[i].x, b[j].x, accr[i][j]);
                    accr[i][j] = fma(-a[i].y, b[j].y, accr[i][j]);
                    acci[i][j] = fma(a[i].x, b[j].y, acci[i][j]);
                    acci[i][j] = fma(a[i].y, b[j].x, acci[i][j]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = m0 + ty * 4 + i;
        if (row >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = c0 + tx + 16 * j;
            if (col >= ncols) continue;
            double2* p = Cb + (size_t)row * ncols + col;
            double2 v = make_double2(accr[i][j], acci[i][j]);
            if (accumulate) {
                const double2 o = *p;
                v.x += o.x;
                v.y += o.y;
            }
            *p = v;
        }
    }
}

// ------------------------------------------------------------ kron residual
__device__ __forceinline__ void stencil_apply(const double2* __restrict__ v, int x, int m, const Stencil& st,
                                              double2& Mv, double2& Av) {
    const int ix = x % m, iy = x / m;
    double2 c = v[x];
    Mv = make_double2(st.M[STFEM_ST_C] * c.x, st.M[STFEM_ST_C] * c.y);
    Av = make_double2(st.A[STFEM_ST_C] * c.x, st.A[STFEM_ST_C] * c.y);
    auto add = [&](int q, int idx) {
        const double2 w = v[idx];
        Mv.x += st.M[q] * w.x;
        Mv.y += st.M[q] * w.y;
        Av.x += st.A[q] * w.x;
        Av.y += st.A[q] * w.y;
    };
    if (ix + 1 < m) add(STFEM_ST_E, x + 1);
    if (ix > 0) add(STFEM_ST_W, x - 1);
    if (iy + 1 < m) add(STFEM_ST_N, x + m);
    if (iy > 0) add(STFEM_ST_S, x - m);
    if (ix + 1 < m && iy + 1 < m) add(STFEM_ST_NE, x + m + 1);
    if (ix > 0 && iy > 0) add(STFEM_ST_SW, x - m - 1);
}

// grid (ceil(n_x/256), n_t, nrhs).  Psi/F/R: [nrhs][n_t][n_x].
__global__ __launch_bounds__(256) void k_kron(const double2* __restrict__ Psi, const double2* __restrict__ F,
                                              double2* __restrict__ R, int n_t, int w,
                                              const double* __restrict__ tM, const double* __restrict__ tB,
                                              Stencil st, int adjoint, double* __restrict__ partial) {
    const int m = st.m, n_x = m * m;
    const int l = blockIdx.y, rh = blockIdx.z;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const size_t base = (size_t)rh * n_t * n_x;
    const int bw = 2 * w + 1;
    double2 acc = make_double2(0.0, 0.0), f = make_double2(0.0, 0.0);
    if (x < n_x) {
        for (int dm = -w; dm <= w; ++dm) {
            const int mm = l + dm;
            if (mm < 0 || mm >= n_t) continue;
            double cm, cb;
            if (!adjoint) {
                cm = tM[l * bw + dm + w];
                cb = tB[l * bw + dm + w];
            } else {   // K^H = -i B^T (x) M + M^T (x) A
                cm = tM[mm * bw + (l - mm) + w];
                cb = -tB[mm * bw + (l - mm) + w];
            }
            if (cm == 0.0 && cb == 0.0) continue;
            double2 Mv, Av;
            stencil_apply(Psi + base + (size_t)mm * n_x, x, m, st, Mv, Av);
            acc.x += -cb * Mv.y + cm * Av.x;
            acc.y += cb * Mv.x + cm * Av.y;
        }
        if (F) {
            f = F[base + (size_t)l * n_x + x];
            acc = make_double2(f.x - acc.x, f.y - acc.y);
        }
        R[base + (size_t)l * n_x + x] = acc;
    }
    if (!partial) return;
    double rr = acc.x * acc.x + acc.y * acc.y, ff = f.x * f.x + f.y * f.y;
    for (int off = 32; off >= 1; off >>= 1) {
        rr += __shfl_xor(rr, off, 64);
        ff += __shfl_xor(ff, off, 64);
    }
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = rr;
        red[1][wave] = ff;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t pidx = ((size_t)rh * gridDim.y + l) * gridDim.x + blockIdx.x;
        partial[2 * pidx] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partial[2 * pidx + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// one workgroup per rhs: sum `per` (rr, ff) pairs in a fixed order
__global__ __launch_bounds__(256) void k_norm_reduce(const double* __restrict__ partial, long long per,
                                                     double* __restrict__ norms) {
    const int rh = blockIdx.x;
    const double* p = partial + 2 * (size_t)rh * per;
    double rr = 0, ff = 0;
    for (long long e = threadIdx.x; e < per; e += 256) {
        rr += p[2 * e];
        ff += p[2 * e + 1];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        rr += __shfl_xor(rr, off, 64);
        ff += __shfl_xor(ff, off, 64);
    }
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = rr;
        red[1][wave] = ff;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        norms[2 * rh] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        norms[2 * rh + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

__global__ __launch_bounds__(256) void k_spatial(const double2* __restrict__ X, double2* __restrict__ Y, Stencil st,
                                                 double ar, double ai, double br, double bi) {
    const int n_x = st.m * st.m;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= n_x) return;
    const size_t base = (size_t)blockIdx.y * n_x;
    double2 Mv, Av;
    stencil_apply(X + base, x, st.m, st, Mv, Av);
    Y[base + x] = make_double2(ar * Mv.x - ai * Mv.y + br * Av.x - bi * Av.y,
                               ar * Mv.y + ai * Mv.x + br * Av.y + bi * Av.x);
}

__global__ void k_fill_int(int* p, int count, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// LDS panel width for the factorisation: the largest of 32, 16, 8 whose panel
// ((NB + kd) x NB complex values) stays within 150 KiB.
int ldlt_nb(int kd, size_t elem) {
    for (int nb : {32, 16, 8})
        if ((size_t)(nb + kd) * nb * elem <= 150u * 1024u) return nb;
    return 0;
}

template <class R, int NB>
hipError_t launch_ldlt(void* band, int count, const Stencil& st, int* info, hipStream_t s) {
    const size_t lds = (size_t)(NB + st.n) * NB * sizeof(cpx<R>);
    auto kern = k_ldlt<R, NB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(count), dim3(256), lds, s, (cpx<R>*)band, st, info);
    return hipGetLastError();
}

template <class R, int NB, int KS>
hipError_t launch_sweep_ks(const void* band, int count, const Stencil& st, const double* G, double* U, int nrhs,
                           int conj, hipStream_t s) {
    const int Sz = st.n + 2 * NB;
    const size_t lds = (size_t)(4 * Sz + 4 * NB) * sizeof(cpx<R>);
    const long long rstride = (long long)count * st.m * st.m * 2;   // doubles between rhs
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nr = std::min(4, nrhs - r0);
        const double* Gr = G + (size_t)r0 * rstride;
        double* Ur = U + (size_t)r0 * rstride;
        if (conj) {
            auto kern = k_sweep<R, NB, KS, true>;
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(count), dim3(256), lds, s, (const cpx<R>*)band, st, Gr, Ur, nr, rstride / 2);
        } else {
            auto kern = k_sweep<R, NB, KS, false>;
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(count), dim3(256), lds, s, (const cpx<R>*)band, st, Gr, Ur, nr, rstride / 2);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class R>
hipError_t launch_sweep(const void* band, int count, const Stencil& st, const double* G, double* U, int nrhs, int conj,
                        hipStream_t s) {
    constexpr int NB = 16;
    if (st.n <= 256) return launch_sweep_ks<R, NB, 1>(band, count, st, G, U, nrhs, conj, s);
    if (st.n <= 512) return launch_sweep_ks<R, NB, 2>(band, count, st, G, U, nrhs, conj, s);
    if (st.n <= 1024) return launch_sweep_ks<R, NB, 4>(band, count, st, G, U, nrhs, conj, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t band_fill(int precision, void* band, const double* lambda, int count, const Stencil& st, hipStream_t s) {
    const long long per = (long long)st.m * st.m * (st.n + 1);
    const int bx = (int)std::min<long long>((per + 255) / 256, 2048);
    if (precision == 32)
        hipLaunchKernelGGL(k_band_fill<float>, dim3(bx, count), dim3(256), 0, s, (cpx<float>*)band, lambda, st);
    else
        hipLaunchKernelGGL(k_band_fill<double>, dim3(bx, count), dim3(256), 0, s, (cpx<double>*)band, lambda, st);
    return hipGetLastError();
}

hipError_t ldlt_factor(int precision, void* band, int count, const Stencil& st, int* info, hipStream_t s) {
    if (precision == 32) {
        switch (ldlt_nb(st.n, sizeof(cpx<float>))) {
            case 32: return launch_ldlt<float, 32>(band, count, st, info, s);
            case 16: return launch_ldlt<float, 16>(band, count, st, info, s);
            case 8: return launch_ldlt<float, 8>(band, count, st, info, s);
        }
    } else {
        switch (ldlt_nb(st.n, sizeof(cpx<double>))) {
            case 32: return launch_ldlt<double, 32>(band, count, st, info, s);
            case 16: return launch_ldlt<double, 16>(band, count, st, info, s);
            case 8: return launch_ldlt<double, 8>(band, count, st, info, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t sweep_solve(int precision, const void* band, int count, const Stencil& st, const double* G, double* U,
                       int nrhs, int conj, hipStream_t s) {
    if (precision == 32) return launch_sweep<float>(band, count, st, G, U, nrhs, conj, s);
    return launch_sweep<double>(band, count, st, G, U, nrhs, conj, s);
}

hipError_t zgemm_small_left(int n, int ncols, int batch, const double* A, int trans, const double* B, long long strideB,
                            double* C, long long strideC, int accumulate, hipStream_t s) {
    dim3 grid((ncols + 63) / 64, (n + 63) / 64, batch);
    hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, s, n, ncols, (const double2*)A, trans, (const double2*)B, strideB,
                       (double2*)C, strideC, accumulate);
    return hipGetLastError();
}

size_t residual_partial_size(int nrhs, int n_t, int n_x) {
    return 2 * (size_t)nrhs * n_t * ((n_x + 255) / 256);
}

hipError_t kron_residual(const double* Psi, const double* F, double* R, int nrhs, int n_t, int w, const double* tM,
                         const double* tB, const Stencil& st, int adjoint, double* partial, double* norms,
                         hipStream_t s) {
    const int n_x = st.m * st.m;
    dim3 grid((n_x + 255) / 256, n_t, nrhs);
    hipLaunchKernelGGL(k_kron, grid, dim3(256), 0, s, (const double2*)Psi, (const double2*)F, (double2*)R, n_t, w, tM,
                       tB, st, adjoint, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long per = (long long)n_t * grid.x;
    hipLaunchKernelGGL(k_norm_reduce, dim3(nrhs), dim3(256), 0, s, partial, per, norms);
    return hipGetLastError();
}

hipError_t kron_apply(const double* Psi, double* Y, int nrhs, int n_t, int w, const double* tM, const double* tB,
                      const Stencil& st, int adjoint, hipStream_t s) {
    const int n_x = st.m * st.m;
    dim3 grid((n_x + 255) / 256, n_t, nrhs);
    hipLaunchKernelGGL(k_kron, grid, dim3(256), 0, s, (const double2*)Psi, (const double2*)nullptr, (double2*)Y, n_t, w,
                       tM, tB, st, adjoint, (double*)nullptr);
    return hipGetLastError();
}

hipError_t spatial_apply(const Stencil& st, double ar, double ai, double br, double bi, const double* X, double* Y,
                         int count, hipStream_t s) {
    const int n_x = st.m * st.m;
    hipLaunchKernelGGL(k_spatial, dim3((n_x + 255) / 256, count), dim3(256), 0, s, (const double2*)X, (double2*)Y, st,
                       ar, ai, br, bi);
    return hipGetLastError();
}

hipError_t fill_int(int* p, int count, int value, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

}  // namespace gpu
}  // namespace stfem
