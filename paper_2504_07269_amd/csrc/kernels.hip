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
// y - a*b in four fused multiply-adds
template <class R>
__device__ __forceinline__ cpx<R> cfms(cpx<R> y, cpx<R> a, cpx<R> b) {
    y.x = fma(-a.x, b.x, y.x);
    y.x = fma(a.y, b.y, y.x);
    y.y = fma(-a.x, b.y, y.y);
    y.y = fma(-a.y, b.x, y.y);
    return y;
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

// Lane permutations by DPP (a VALU operand modifier, no LDS round trip):
// quad_perm [1,0,3,2] and [2,3,0,1] (partner lane ^1, ^2), half-row mirror
// (lane i <-> 7-i within 8) and row mirror (i <-> 15-i within 16).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, class R>
__device__ __forceinline__ void add_dpp(cpx<R>& a) {
    a.x += dpp<CTRL>(a.x);
    a.y += dpp<CTRL>(a.y);
}
// Sum over aligned groups of G consecutive lanes; every lane of a group
// receives the group's total.
template <int G, class R>
__device__ __forceinline__ void group_sum(cpx<R>& a) {
    if (G >= 2) add_dpp<0xB1>(a);
    if (G >= 4) add_dpp<0x4E>(a);
    if (G >= 8) add_dpp<0x141>(a);
    if (G >= 16) add_dpp<0x140>(a);
    if (G >= 32) {
        const cpx<R> o = shfl_xor(a, 16);
        a.x += o.x;
        a.y += o.y;
    }
    if (G >= 64) {
        const cpx<R> o = shfl_xor(a, 32);
        a.x += o.x;
        a.y += o.y;
    }
}

// Complex values between consecutive blocks of band storage: n_x (kd + 1)
// rounded up to a multiple of 64, so that every block starts 512-byte aligned.
__host__ __device__ __forceinline__ long long band_stride(const Stencil& st) {
    return (((long long)st.m * st.m * (st.n + 1)) + 63) / 64 * 64;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the thread, which would drain
// the prefetches issued ahead of their use; this one leaves them in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
template <class R>
__device__ __forceinline__ cpx<R> rdlane(cpx<R> v, int l) {
    return {rdlane(v.x, l), rdlane(v.y, l)};
}

// 16-byte unit of the factor stream: two FP32 complex values or one FP64.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <class R>
struct Unit;
template <>
struct Unit<float> {
    typedef f32x4 T;
    static constexpr int CPU = 2;   // complex values per unit
};
template <>
struct Unit<double> {
    typedef f64x2 T;
    static constexpr int CPU = 1;
};
// ------------------------------------------------------------------ band fill
// Entries of S_l = lambda_l M + A in the lower band: C on the diagonal, E
// (d = 1, not at the right end of a grid row), N (d = m, not in the top grid
// row) and NE (d = m + 1, neither); everything else, including rows beyond
// the matrix, is zero.  A thread writes the 16-byte units t, t + 256, ... of
// its block's chunk and follows (column j, offset d) incrementally instead of
// dividing per entry.
constexpr int FILL_UPT = 8;   // 16-byte units per thread and chunk
template <class R>
__global__ __launch_bounds__(256) void k_band_fill(cpx<R>* __restrict__ band, const double* __restrict__ lam,
                                                   Stencil st) {
    typedef typename Unit<R>::T UT;
    constexpr int CPU = Unit<R>::CPU;
    const int l = blockIdx.y;
    const double lr = lam[2 * l], li = lam[2 * l + 1];
    const int m = st.m, ld = st.n + 1;
    const cpx<R> vC = {(R)(lr * st.M[STFEM_ST_C] + st.A[STFEM_ST_C]), (R)(li * st.M[STFEM_ST_C])};
    const cpx<R> vE = {(R)(lr * st.M[STFEM_ST_E] + st.A[STFEM_ST_E]), (R)(li * st.M[STFEM_ST_E])};
    const cpx<R> vN = {(R)(lr * st.M[STFEM_ST_N] + st.A[STFEM_ST_N]), (R)(li * st.M[STFEM_ST_N])};
    const cpx<R> vNE = {(R)(lr * st.M[STFEM_ST_NE] + st.A[STFEM_ST_NE]), (R)(li * st.M[STFEM_ST_NE])};
    auto val = [=](int d, int jx, int jy) -> cpx<R> {
        const bool e = d == 1 && jx < m - 1, n = d == m && jy < m - 1;
        const bool ne = d == m + 1 && jx < m - 1 && jy < m - 1;
        R x = d == 0 ? vC.x : R(0), y = d == 0 ? vC.y : R(0);
        x = e ? vE.x : x;
        y = e ? vE.y : y;
        x = n ? vN.x : x;
        y = n ? vN.y : y;
        x = ne ? vNE.x : x;
        y = ne ? vNE.y : y;
        return cpx<R>{x, y};
    };
    const long long per = (long long)m * m * ld;                 // entries of one block
    const long long units = (per + CPU - 1) / CPU;               // the last may run into the padding
    UT* B = reinterpret_cast<UT*>(band + (size_t)l * band_stride(st));
    const long long chunk = 256LL * FILL_UPT;
    for (long long base = (long long)blockIdx.x * chunk; base < units; base += (long long)gridDim.x * chunk) {
        const long long e0 = (base + threadIdx.x) * CPU;         // first entry of the thread's first unit
        int j = (int)(e0 / ld), d = (int)(e0 - (long long)j * ld);
        int jx = j % m, jy = j / m;
#pragma unroll
        for (int i = 0; i < FILL_UPT; ++i) {
            const long long u = base + threadIdx.x + 256LL * i;
            if (u < units) {
                const cpx<R> v0 = val(d, jx, jy);
                if constexpr (CPU == 2) {
                    // the unit's second entry, possibly the next column's first
                    const bool wrap = d + 1 == ld;
                    const int jx1 = wrap ? (jx + 1 == m ? 0 : jx + 1) : jx;
                    const int jy1 = wrap ? (jx + 1 == m ? jy + 1 : jy) : jy;
                    const cpx<R> v1 = val(wrap ? 0 : d + 1, jx1, jy1);
                    B[u] = UT{v0.x, v0.y, v1.x, v1.y};
                } else {
                    B[u] = UT{v0.x, v0.y};
                }
            }
            // advance by 256 units
            d += 256 * CPU;
            while (d >= ld) {
                d -= ld;
                if (++jx == m) { jx = 0; ++jy; }
            }
        }
    }
}

// ---------------------------------------------------------------------- LDL^T
// Matrix-core shapes.  A complex product C += P Q is computed as the real
// product C' += A' B': every complex row of C is a real row pair (Re, Im) of
// C', every complex k a real pair of A' columns / B' rows, A' holds the blocks
// [[Pr, -Pi], [Pi, Pr]] and B' the pairs [Qr; Qi]:
//   C'(Re row) = sum_k Pr Qr - Pi Qi,   C'(Im row) = sum_k Pi Qr + Pr Qi.
// FP32: v_mfma_f32_32x32x2f32 = 16 complex rows x 32 complex cols x 1 complex k.
// FP64: v_mfma_f64_16x16x4f64 =  8 complex rows x 16 complex cols x 2 complex k.
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class R>
struct Mma;
template <>
struct Mma<float> {
    // C' rows alternate: row 2i = Re(row i), row 2i+1 = Im(row i).
    // Operand and result lane layout of v_mfma_f32_32x32x2f32 (wave64):
    // A'[i'][k'] from lane i' + 32 k', B'[k'][j] from lane j + 32 k',
    // result register r of lane l = C'[8 (r/4) + 4 (l/32) + r%4][l%32].
    static constexpr int ROWS = 16, COLS = 32, KC = 1, NACC = 16, NENT = 8;
    typedef f32x16 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    // A' element held by `lane`: complex row, real/imag row, complex k, real/imag column
    static __device__ __forceinline__ int a_row(int lane) { return (lane & 31) >> 1; }
    static __device__ __forceinline__ int a_im(int lane) { return lane & 1; }
    static __device__ __forceinline__ int a_k(int) { return 0; }
    static __device__ __forceinline__ int a_b(int lane) { return lane >> 5; }
    // B' element: complex column, complex k, real/imag
    static __device__ __forceinline__ int b_col(int lane) { return lane & 31; }
    static __device__ __forceinline__ int b_k(int) { return 0; }
    static __device__ __forceinline__ int b_b(int lane) { return lane >> 5; }
    // complex result entry e (0..NENT-1) of `lane`: row, and the registers of its parts
    static __device__ __forceinline__ int e_row(int lane, int e) { return 4 * (e >> 1) + 2 * (lane >> 5) + (e & 1); }
    static __device__ __forceinline__ int e_re(int e) { return 2 * e; }
    static __device__ __forceinline__ int e_im(int e) { return 2 * e + 1; }
    static __device__ __forceinline__ int c_col(int lane) { return lane & 31; }
};
template <>
struct Mma<double> {
    // C' rows 0-7 = Re(rows 0-7), rows 8-15 = Im(rows 0-7).
    // v_mfma_f64_16x16x4f64 (wave64): A'[i'][k'] from lane i' + 16 k',
    // B'[k'][j] from lane j + 16 k', result register r of lane l =
    // C'[4 r + l/16][l%16].
    static constexpr int ROWS = 8, COLS = 16, KC = 2, NACC = 4, NENT = 2;
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int a_row(int lane) { return lane & 7; }
    static __device__ __forceinline__ int a_im(int lane) { return (lane >> 3) & 1; }
    static __device__ __forceinline__ int a_k(int lane) { return lane >> 5; }
    static __device__ __forceinline__ int a_b(int lane) { return (lane >> 4) & 1; }
    static __device__ __forceinline__ int b_col(int lane) { return lane & 15; }
    static __device__ __forceinline__ int b_k(int lane) { return lane >> 5; }
    static __device__ __forceinline__ int b_b(int lane) { return (lane >> 4) & 1; }
    // registers e and e+2 hold Re and Im of complex row 4 e + l/16 (l/16 in 0..3)
    static __device__ __forceinline__ int e_row(int lane, int e) { return 4 * e + (lane >> 4); }
    static __device__ __forceinline__ int e_re(int e) { return e; }
    static __device__ __forceinline__ int e_im(int e) { return e + 2; }
    static __device__ __forceinline__ int c_col(int lane) { return lane & 15; }
};

// Wave-level ordering of LDS accesses (a wave's LDS operations complete in
// issue order once the compiler keeps that order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
}

// One workgroup (4 waves) factors one band as L D L^T, right-looking, NB
// columns per step, NB <= the tile size Mma::COLS.  The NB columns of a step
// are one contiguous chunk of band storage held in LDS in that layout
// (Pb[c*ld + d] = entry (k+c+d, k+c)); its diagonal block was factored one
// step earlier.  Per step:
//  1. the W table W[c][c2] = D_c2 L[c][c2] of the diagonal block; the block
//     itself goes to global memory (final);
//  2. every thread solves one row below the diagonal block, left-looking in
//     registers: L[r][c] D_c = A[r][c] - sum_{c'<c} L[r][c'] D_c' L[c][c'],
//     and stores L to global memory (final) and N = -L D to LDS as the
//     matrix-core A' operands;
//  3. the first tile column of the trailing kd x kd lower triangle gets
//     A -= (L D) L^T on the matrix cores; its first NB columns are the next
//     step's chunk and go straight into the LDS panel, with the entries of
//     the next chunk below the window;
//  4. wave 0 factors the next chunk's NB x NB diagonal block in registers
//     (lane r holds row r, column multipliers are broadcast between lanes),
//     while the other waves, and wave 0 once it is done,
//     update the rest of the trailing triangle in global memory, one tile row
//     at a time taken from a shared counter, longest rows first.
// The update runs in square tiles of Mma::COLS complex rows and columns (two
// matrix-core row blocks per tile); a wave keeps one tile row's B' operands,
// L = -N D^{-1}, in registers and sweeps that row's tiles.  Each tile's
// product is formed from zero and added to the tile just before its store;
// two tile buffers take turns, the next tile's loads in flight during the
// current tile's MFMAs.
// One row of the panel below its diagonal block: x[C] = (x[C] - sum_{c2<C}
// x[c2] W[C][c2]) D^{-1}_C for C = 0..NB-1, unrolled at compile time so that
// the row stays in registers; the sum is formed on its own and subtracted
// once (fewer roundings at the entry's magnitude).  The value before the
// scaling, L[r][C] D_C, goes negated to Nrow[C * ROWS].
template <int C, int NB, int ROWS, class R>
__device__ __forceinline__ void row_solve(cpx<R> (&x)[NB], const cpx<R>* W, const cpx<R>* Dinv, cpx<R>* Nrow) {
    if constexpr (C < NB) {
        if constexpr (C > 0) {
            cpx<R> sum = {R(0), R(0)};
#pragma unroll
            for (int c2 = 0; c2 < C; ++c2) sum = cfma(x[c2], W[C * NB + c2], sum);
            x[C] = csub(x[C], sum);
        }
        Nrow[C * ROWS] = cpx<R>{-x[C].x, -x[C].y};
        x[C] = cmul(x[C], Dinv[C]);
        // finish this column before the next column's table reads, or all
        // NB^2/2 of them would be in registers at once
        __asm__ volatile("" : "+v"(x[C].x), "+v"(x[C].y) : : "memory");
        row_solve<C + 1, NB, ROWS>(x, W, Dinv, Nrow);
    }
}

template <class R, int NB>
__global__ __launch_bounds__(256, 1) void k_ldlt(cpx<R>* __restrict__ band, Stencil st, int* __restrict__ info) {
    typedef Mma<R> MM;
    typedef typename MM::acc_t AT;
    typedef typename Unit<R>::T UT;
    constexpr int CPU = Unit<R>::CPU;
    constexpr int TS = MM::COLS;          // tile size (complex rows = cols)
    constexpr int RB = TS / MM::ROWS;     // matrix-core row blocks per tile (2)
    constexpr int KS = NB / MM::KC;       // matrix-core k steps per tile
    constexpr int QB = 16;                // 16-byte transfers in flight per thread
    constexpr int NW = 4;                 // waves
    static_assert(NB <= TS, "the next chunk must lie in the first tile column");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = st.m, kd = st.n, n_x = m * m, ld = kd + 1;
    cpx<R>* Pb = reinterpret_cast<cpx<R>*>(smem_raw);                 // NB*ld, rounded to units
    cpx<R>* Dinv = Pb + (NB * ld + CPU - 1) / CPU * CPU;             // 2 * NB (two steps)
    cpx<R>* W = Dinv + 2 * NB;                                        // NB * NB
    cpx<R>* Xb = W + NB * NB;                                         // 2 * NB
    cpx<R>* Nsw = Xb + 2 * NB;                                        // ceil(kd/TS) * TS * NB
    int* ctr = reinterpret_cast<int*>(Nsw + (kd + TS - 1) / TS * TS * NB);
    const int l = blockIdx.x;
    cpx<R>* A = band + (size_t)l * band_stride(st);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const cpx<R> zero = {R(0), R(0)};
    int bad = 0;
    // entry (row r, column c) of the panel, relative to the step start
    auto PV = [&](int c, int r) -> cpx<R> {
        const int d = r - c;
        return (d >= 0 && d <= kd) ? Pb[c * ld + d] : zero;
    };
    // diagonal block of the chunk in Pb (columns k0.., nbk of them), wave 0:
    // column by column, the pivot by a lane broadcast, L[.][c] published
    // through LDS (Xb, double-buffered) and read back as broadcasts
    auto diag = [&](int k0, int nbk, cpx<R>* Dout) {
        const int r = lane;
        cpx<R> y[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) y[c] = (r < nbk && c <= r && c < nbk) ? PV(c, r) : zero;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c < nbk) {
                bool ok;
                const cpx<R> d = rdlane(y[c], c);
                const cpx<R> inv = cinv_or_zero(d, ok);
                if (!ok && bad == 0) bad = k0 + c + 1;
                const cpx<R> lr = cmul(y[c], inv);          // L[r][c] for r > c
                cpx<R>* xb = Xb + (c & 1) * NB;
                if (r < NB) xb[r] = lr;
                wave_sync();
#pragma unroll
                for (int c2 = c + 1; c2 < NB; ++c2)          // Y[r][c2] -= Y[r][c] L[c2][c]
                    y[c2] = cfms(y[c2], y[c], xb[c2]);
                if (r > c) y[c] = lr;
                if (r == c) Dout[c] = inv;
            }
        }
        if (r < nbk) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c <= r && r - c <= kd) Pb[c * ld + (r - c)] = y[c];
        }
    };
    // ---- first chunk to LDS, its diagonal block
    {
        const int units = (min(NB, n_x) * ld + CPU - 1) / CPU;
        const UT* src = reinterpret_cast<const UT*>(A);
        UT* dst = reinterpret_cast<UT*>(Pb);
        for (int base = 0; base < units; base += QB * 256) {
            UT q[QB];
#pragma unroll
            for (int j = 0; j < QB; ++j) {
                const int e = base + tid + 256 * j;
                if (e < units) q[j] = src[e];
            }
#pragma unroll
            for (int j = 0; j < QB; ++j) {
                const int e = base + tid + 256 * j;
                if (e < units) dst[e] = q[j];
            }
        }
    }
    lds_barrier();
    if (wave == 0) diag(0, min(NB, n_x), Dinv);
    lds_barrier();
    // matrix-core operands: the 2x2 real block of a complex N entry is
    // [[x, -y], [y, x]]; a lane's A' element is component a_im ^ a_b of N,
    // negated for (a_im, a_b) = (0, 1)
    const R* Nf = reinterpret_cast<const R*>(Nsw);
    const int a_off = 2 * (MM::a_k(lane) * MM::ROWS + MM::a_row(lane)) + (MM::a_im(lane) ^ MM::a_b(lane));
    const R a_sgn = (MM::a_b(lane) && !MM::a_im(lane)) ? R(-1) : R(1);
    int par = 0;                                  // Dinv half of the current step
    for (int k = 0; k < n_x; k += NB) {
        const int nb = min(NB, n_x - k);
        const int mrows = min(nb + kd, n_x - k);
        const int ntr = mrows - nb;               // trailing rows/cols
        const int TT = (ntr + TS - 1) / TS;       // tile rows
        const int nbn = min(NB, n_x - k - nb);    // width of the next chunk (0 at the end)
        const cpx<R>* Dk = Dinv + par * NB;
        cpx<R>* Dn = Dinv + (par ^ 1) * NB;
        // The trailing update, tile (I, J), J <= I, of the lower triangle
        // computed transposed, C^T += N_J L_I^T: a lane owns one row of the
        // tile (window row TS I + c_col), and its loads and stores of the tile
        // run down the band columns (contiguous).
        // tiles J0..J1 of tile row I; head: the first tile column, whose
        // columns below nbn go to the LDS panel of the next step
        auto tile_row = [&](int I, int J0, int J1, bool head) {
            // B' operands of tile row I: L = -N D^{-1}, real/imaginary parts
            R bv[KS];
            {
                const int rr = TS * I + MM::b_col(lane);
                const int jb = rr / MM::ROWS, i = rr % MM::ROWS;
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int c = s * MM::KC + MM::b_k(lane);
                    cpx<R> lv = zero;
                    if (c < nb) lv = cmul(Nsw[(jb * NB + c) * MM::ROWS + i], Dk[c]);
                    bv[s] = MM::b_b(lane) ? -lv.y : -lv.x;
                }
            }
            const bool rows_full = TS * (I + 1) <= ntr;
            const int brow = TS * I + MM::c_col(lane);   // window row held by this lane
            // window column of accumulator entry e of row block rb, relative to tile column J
            auto tcol = [&](int rb, int e) { return MM::ROWS * rb + MM::e_row(lane, e); };
            // band address of window entry (brow, col): column-major lower band
            auto addr = [&](int col) { return A + (size_t)(k + nb + col) * ld + (brow - col); };
            auto load_c = [&](int J, typename MM::acc_t (&acc)[RB]) {
                if (J < I && rows_full) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int e = 0; e < MM::NENT; ++e) {
                            const cpx<R> cv = *addr(TS * J + tcol(rb, e));
                            acc[rb][MM::e_re(e)] = cv.x;
                            acc[rb][MM::e_im(e)] = cv.y;
                        }
                } else {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int e = 0; e < MM::NENT; ++e) {
                            const int cc = TS * J + tcol(rb, e);
                            // unconditional load from a valid address (window
                            // entry (0, 0) stands in), zero selected after
                            const bool in = J <= J1 && brow < ntr && cc < ntr && brow >= cc;
                            const cpx<R> lv = *(in ? addr(cc) : A + (size_t)(k + nb) * ld);
                            const cpx<R> cv = in ? lv : zero;
                            acc[rb][MM::e_re(e)] = cv.x;
                            acc[rb][MM::e_im(e)] = cv.y;
                        }
                }
            };
            auto store_c = [&](int J, const typename MM::acc_t (&acc)[RB]) {
                if (head) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int e = 0; e < MM::NENT; ++e) {
                            const int cc = TS * J + tcol(rb, e);
                            const cpx<R> v = {acc[rb][MM::e_re(e)], acc[rb][MM::e_im(e)]};
                            if (brow < ntr && cc < ntr && brow >= cc) {
                                if (cc < nbn) Pb[cc * ld + (brow - cc)] = v;
                                else *addr(cc) = v;
                            }
                        }
                } else if (J < I && rows_full) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int e = 0; e < MM::NENT; ++e)
                            *addr(TS * J + tcol(rb, e)) = cpx<R>{acc[rb][MM::e_re(e)], acc[rb][MM::e_im(e)]};
                } else {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int e = 0; e < MM::NENT; ++e) {
                            const int cc = TS * J + tcol(rb, e);
                            if (brow < ntr && cc < ntr && brow >= cc)
                                *addr(cc) = cpx<R>{acc[rb][MM::e_re(e)], acc[rb][MM::e_im(e)]};
                        }
                }
            };
            // The product of a tile is formed from zero and added to the tile
            // just before its store, so that the tile's loads only have to
            // land by then; two tile buffers take turns, the next tile's loads
            // in flight during the current tile's MFMAs.
            auto update = [&](int J, const typename MM::acc_t (&c)[RB]) {
                typename MM::acc_t acc[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[rb] = typename MM::acc_t{};
#pragma unroll
                for (int s = 0; s < KS; ++s)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const R av = a_sgn * Nf[((J * RB + rb) * NB + s * MM::KC) * MM::ROWS * 2 + a_off];
                        acc[rb] = MM::mma(av, bv[s], acc[rb]);
                    }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[rb] += c[rb];
                store_c(J, acc);
            };
            typename MM::acc_t ta[RB], tb[RB];
            load_c(J0, ta);
            for (int J = J0; J <= J1; J += 2) {
                if (J < J1) load_c(J + 1, tb);
                update(J, ta);
                if (J == J1) break;
                if (J + 1 < J1) load_c(J + 2, ta);
                update(J + 1, tb);
            }
        };
        // ---- 1. W table, the diagonal block to global memory (final); A'
        //      operands of rows past the window are zero
        for (int e = tid; e < NB * NB; e += 256) {
            const int c = e / NB, c2 = e - c * NB;
            W[e] = (c2 < c && c < nb) ? cmul(Pb[c2 * ld], Pb[c2 * ld + (c - c2)]) : zero;
            // entry (k + c + c2, k + c) of the block
            if (c < nb && c + c2 < nb && c2 <= kd) A[(size_t)(k + c) * ld + c2] = Pb[c * ld + c2];
        }
        for (int e = tid; e < (TT * TS - ntr) * NB; e += 256) {
            const int rr = ntr + e / NB, c = e % NB;
            Nsw[(rr / MM::ROWS * NB + c) * MM::ROWS + rr % MM::ROWS] = zero;
        }
        if (tid == 0) *ctr = 0;
        lds_barrier();
        // ---- 2. rows below the diagonal block
        for (int r = nb + tid; r < mrows; r += 256) {
            cpx<R> x[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = (c < nb) ? PV(c, r) : zero;
            const int rr = r - nb;
            row_solve<0, NB, MM::ROWS>(x, W, Dk, Nsw + (rr / MM::ROWS) * NB * MM::ROWS + rr % MM::ROWS);
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nb && r - c <= kd) A[(size_t)(k + c) * ld + (r - c)] = x[c];
        }
        lds_barrier();
        // ---- 3. first tile column -> next chunk; the next chunk's entries
        //      below the window from global memory (column c takes rows
        //      d >= ntr - c)
        for (int I = wave; I < TT; I += NW) tile_row(I, 0, 0, true);
        const int fl = min(ld, kd + 1 - ntr + nbn - 1);   // longest such run
        const int nfresh = nbn > 0 ? nbn * fl : 0;
        const cpx<R>* fsrc = A + (size_t)(k + nb) * ld;
        for (int e = tid; e < nfresh; e += 256) {
            const int c = e / fl, d = kd - (e - c * fl);
            if (d >= ntr - c) Pb[c * ld + d] = fsrc[c * ld + d];
        }
        lds_barrier();
        // ---- 4. next diagonal block (wave 0) beside the rest of the update
        if (wave == 0 && nbn > 0) diag(k + nb, nbn, Dn);
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(ctr, 1);
            t = __builtin_amdgcn_readfirstlane(t);
            const int I = TT - 1 - t;
            if (I < 1) break;
            tile_row(I, 1, I, false);
        }
        __syncthreads();
        par ^= 1;
    }
    if (tid == 0) info[l] = bad;
}

// ---------------------------------------------------------------------- sweeps
constexpr int SWEEP_QL = 11;       // 16-byte units per producer thread and panel
constexpr int SWEEP_BULK = 256;    // threads of waves 1-4
constexpr int SWEEP_PROD = 192;    // threads of waves 5-7

// One workgroup of 8 waves solves S_l x = g for NR right-hand sides:
// L y = g, z = D^{-1} y, L^T x = z.  The sweeps walk the factor panel by
// panel (NB columns); a panel, NB columns of band storage, is one contiguous
// chunk of memory.  Waves 5-7 are producers: they store into a ring of three
// LDS slots the panel they loaded one step earlier, then issue the loads of
// the next one.  Waves 0-4 are consumers; the rows within reach of the
// current panels live in an LDS ring of Sz slots per rhs (Sz a power of two
// >= kd + 2 NB).  The consumers pipeline two panels, so that each panel step
// needs a single LDS-only barrier (no wave waits there for global memory):
//  forward, step p   wave 0 subtracts the contributions of panel p-1 from
//                    the NB rows of panel p and solves their unit triangle
//                    (register broadcasts between lanes); waves 1-4 subtract
//                    the contributions of panel p-1 from the kd - NB rows
//                    below panel p and store the NB rows of g that enter
//                    (loaded one step earlier);
//  backward, step b  (panel p = last - b) wave 0 forms the dot products of the
//                    columns of panel p with the x of panel p+1, adds the far
//                    sums prepared one step earlier and solves the transposed
//                    triangle; waves 1-4 form the far sums of panel p-1: the
//                    dot products of its columns with the x of panels >= p+1,
//                    RL = 256/NB threads per column, whose partial sums wave 0
//                    adds up.  Each thread's rows are rotated by its column,
//                    so that the lanes of one LDS read hit distinct banks.
// In wave 0 a row (or column) of the panel is owned by a group of CG = 64/NB
// consecutive lanes; group sums use DPP lane permutations.  Needs NB <= kd.
template <class R, int NB, int NR, bool CONJ>
__global__ __launch_bounds__(512, 1) void k_sweep(const cpx<R>* __restrict__ band, Stencil st, const double* G,
                                                  double* U, long long rstride, int Sz) {
    typedef typename Unit<R>::T UT;
    constexpr int CPU = Unit<R>::CPU;
    constexpr int CG = 64 / NB;              // lanes per row (column) in wave 0
    constexpr int PER = (NB + CG - 1) / CG;  // columns (rows) per lane of a group
    constexpr int RL = SWEEP_BULK / NB;      // threads per column in the far sums
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = st.m, kd = st.n, n_x = m * m, ld = kd + 1;
    const int msk = Sz - 1;
    const int slot_units = (NB * ld + CPU - 1) / CPU;
    UT* ring = reinterpret_cast<UT*>(smem_raw);                       // 3 * slot_units
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(ring + 3 * slot_units);      // Y[rh*Sz + slot]
    cpx<R>* P = Y + NR * Sz;                                          // P[par][(t*NR + rh)*NB + c]
    const int l = blockIdx.x;
    const cpx<R>* Lb = band + (size_t)l * band_stride(st);
    const double2* g = reinterpret_cast<const double2*>(G) + (size_t)l * n_x;
    double2* u = reinterpret_cast<double2*>(U) + (size_t)l * n_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool producer = wave >= 5;
    const int ptid = tid - 64 - SWEEP_BULK;  // producer thread index
    const int t1 = tid - 64;                 // thread index within waves 1-4
    const int npanel = (n_x + NB - 1) / NB;
    const cpx<R> cz = {R(0), R(0)};

    // ---- producers
    UT q[SWEEP_QL];
    auto pload = [&](int p) {
        p = min(max(p, 0), npanel - 1);
        const int k = p * NB, nb = min(NB, n_x - k);
        const int units = (nb * ld + CPU - 1) / CPU;
        const UT* src = reinterpret_cast<const UT*>(Lb + (size_t)k * ld);
#pragma unroll
        for (int j = 0; j < SWEEP_QL; ++j) q[j] = src[min(ptid + SWEEP_PROD * j, units - 1)];
    };
    auto pstore = [&](int p, int slot) {
        const int k = p * NB, nb = min(NB, n_x - k);
        const int units = (nb * ld + CPU - 1) / CPU;
        UT* dst = ring + slot * slot_units;
#pragma unroll
        for (int j = 0; j < SWEEP_QL; ++j) {
            const int e = ptid + SWEEP_PROD * j;
            if (e < units) dst[e] = q[j];
        }
    };
    // ---- consumers: entry (k+r, k+c) of the panel in `slot`, 0 <= r - c <= kd
    auto PV = [&](int slot, int c, int r) -> cpx<R> {
        cpx<R> v = reinterpret_cast<const cpx<R>*>(ring + slot * slot_units)[c * ld + (r - c)];
        if (CONJ) v.y = -v.y;
        return v;
    };

    // ===================================================== forward sweep
    if (producer) {
        pload(0);
        pstore(0, 0);
        pload(1);
    } else {
        const int rows0 = min(NB + kd, n_x);
        for (int e = tid; e < NR * rows0; e += 64 + SWEEP_BULK) {
            const int rh = e / rows0, i = e - rh * rows0;
            const double2 v = g[(size_t)rh * rstride + i];
            Y[rh * Sz + (i & msk)] = {(R)v.x, (R)v.y};
        }
    }
    // rows of g that enter the window, loaded one step before they are
    // stored (threads t1 < NB * NR of waves 1-4): row kd + t1 % NB at step 0
    double2 gq = make_double2(0.0, 0.0);
    if (!producer && wave > 0 && t1 < NB * NR) {
        const int rh = t1 / NB, i = kd + (t1 % NB);
        if (i < n_x) gq = g[(size_t)rh * rstride + i];
    }
    lds_barrier();
    for (int p = 0; p < npanel; ++p) {
        const int k = p * NB, nb = min(NB, n_x - k), kp = k - NB;
        const int slot = p % 3, slotq = (p + 2) % 3;      // panels p and p-1
        if (producer) {
            if (p + 1 < npanel) pstore(p + 1, (p + 1) % 3);
            pload(p + 2);
        } else if (wave == 0) {
            const int r = lane / CG, cg = lane % CG;
            cpx<R> acc[NR];
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) acc[rh] = cz;
            if (p > 0) {
#pragma unroll
                for (int q2 = 0; q2 < PER; ++q2) {
                    const int c = cg + CG * q2;
                    if (c < NB && r < nb && NB + r - c <= kd) {
                        const cpx<R> lv = PV(slotq, c, NB + r);
#pragma unroll
                        for (int rh = 0; rh < NR; ++rh) acc[rh] = cfma(lv, Y[rh * Sz + ((kp + c) & msk)], acc[rh]);
                    }
                }
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) group_sum<CG>(acc[rh]);
            }
            const int ys = (k + min(r, nb - 1)) & msk;
            cpx<R> lrow[NB];                                  // L[k+r][k+c], c < r
#pragma unroll
            for (int c = 0; c < NB - 1; ++c) lrow[c] = (r > c && r < nb) ? PV(slot, c, r) : cz;
            const cpx<R> dv = (r < nb) ? PV(slot, r, r) : cpx<R>{R(1), R(0)};
            cpx<R> y[NR];
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) y[rh] = csub(Y[rh * Sz + ys], acc[rh]);
#pragma unroll
            for (int c = 0; c < NB - 1; ++c) {
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) y[rh] = csub(y[rh], cmul(lrow[c], rdlane(y[rh], c * CG)));
            }
            if (cg == 0 && r < nb) {
                bool ok;
                const cpx<R> dinv = cinv_or_zero(dv, ok);
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) {
                    Y[rh * Sz + ys] = y[rh];
                    const cpx<R> z = cmul(y[rh], dinv);
                    u[(size_t)rh * rstride + k + r] = make_double2((double)z.x, (double)z.y);
                }
            }
        } else {
            if (p > 0) {
                const int ihi = min(k - 1 + kd, n_x - 1);
                if constexpr (NR == 1) {
                    cpx<R> yq[NB];                            // y of panel p-1
#pragma unroll
                    for (int c = 0; c < NB; ++c) yq[c] = Y[(kp + c) & msk];
                    for (int i = k + NB + t1; i <= ihi; i += SWEEP_BULK) {
                        const int rr = i - kp;                // row offset in panel p-1
                        cpx<R> acc = cz;
#pragma unroll
                        for (int c = 0; c < NB; ++c) {
                            // in the slot for every c (rr < NB + kd); zero past the band
                            const cpx<R> lv = PV(slotq, c, rr);
                            acc = cfma(rr - c <= kd ? lv : cz, yq[c], acc);
                        }
                        cpx<R>& yi = Y[i & msk];
                        yi = csub(yi, acc);
                    }
                } else {
                    for (int i = k + NB + t1; i <= ihi; i += SWEEP_BULK) {
                        const int rr = i - kp;
                        cpx<R> acc[NR];
#pragma unroll
                        for (int rh = 0; rh < NR; ++rh) acc[rh] = cz;
#pragma unroll
                        for (int c = 0; c < NB; ++c) {
                            if (rr - c <= kd) {
                                const cpx<R> lv = PV(slotq, c, rr);
#pragma unroll
                                for (int rh = 0; rh < NR; ++rh)
                                    acc[rh] = cfma(lv, Y[rh * Sz + ((kp + c) & msk)], acc[rh]);
                            }
                        }
#pragma unroll
                        for (int rh = 0; rh < NR; ++rh) {
                            cpx<R>& yi = Y[rh * Sz + (i & msk)];
                            yi = csub(yi, acc[rh]);
                        }
                    }
                }
            }
            if (t1 < NB * NR) {                               // rows first reached at step p+1
                const int rh = t1 / NB, i = k + kd + (t1 % NB);
                if (i < n_x) Y[rh * Sz + (i & msk)] = {(R)gq.x, (R)gq.y};
                if (i + NB < n_x) gq = g[(size_t)rh * rstride + i + NB];   // for the next step
            }
        }
        lds_barrier();
    }

    // ==================================================== backward sweep
    // step b works on panel p = npanel-1-b (slot b % 3) and panel p-1 (slot
    // (b+1) % 3); the partial far sums of panel p are in P[b & 1]
    const int far_period = (kd - NB + RL - 1) / RL * RL;  // >= rows of the longest column
    cpx<R> zc[NR];
    if (producer) {
        pload(npanel - 1);
        pstore(npanel - 1, 0);
        pload(npanel - 2);
        if (npanel > 1) pstore(npanel - 2, 1);
        pload(npanel - 3);
    } else if (wave == 0) {
        const int k = (npanel - 1) * NB;
#pragma unroll
        for (int rh = 0; rh < NR; ++rh) {
            const double2 z = u[(size_t)rh * rstride + min(k + lane / CG, n_x - 1)];
            zc[rh] = {(R)z.x, (R)z.y};
        }
    } else {
        for (int e = t1; e < RL * NR * NB; e += SWEEP_BULK) P[e] = cz;
    }
    lds_barrier();
    for (int b = 0; b < npanel; ++b) {
        const int p = npanel - 1 - b;
        const int k = p * NB, nb = min(NB, n_x - k), kp = k - NB;
        const int slot = b % 3, slotq = (b + 1) % 3;      // panels p and p-1
        const cpx<R>* Pr = P + (b & 1) * RL * NR * NB;
        cpx<R>* Pw = P + ((b + 1) & 1) * RL * NR * NB;
        if (producer) {
            if (b + 2 < npanel) pstore(npanel - 3 - b, (b + 2) % 3);
            pload(npanel - 4 - b);
        } else if (wave == 0) {
            const int c = lane / CG, rg = lane % CG;
            cpx<R> acc[NR];
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) acc[rh] = cz;
#pragma unroll
            for (int q2 = 0; q2 < PER; ++q2) {                // rows of panel p+1
                const int j = rg + CG * q2, i = k + NB + j;
                if (j < NB && i < n_x && c < nb && NB + j - c <= kd) {
                    const cpx<R> lv = PV(slot, c, NB + j);
#pragma unroll
                    for (int rh = 0; rh < NR; ++rh) acc[rh] = cfma(lv, Y[rh * Sz + (i & msk)], acc[rh]);
                }
            }
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) {
                group_sum<CG>(acc[rh]);
#pragma unroll(16 / NR)
                for (int t = 0; t < RL; ++t) {                // far sums
                    const cpx<R> f = Pr[(t * NR + rh) * NB + c];
                    acc[rh].x += f.x;
                    acc[rh].y += f.y;
                }
            }
            const int r = c;
            cpx<R> lcol[NB];                                  // L[k+cc][k+r], cc > r
#pragma unroll
            for (int cc = 1; cc < NB; ++cc) lcol[cc] = (r < cc && cc < nb) ? PV(slot, r, cc) : cz;
            cpx<R> v[NR];
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) v[rh] = (r < nb) ? csub(zc[rh], acc[rh]) : cz;
#pragma unroll
            for (int cc = NB - 1; cc >= 1; --cc) {
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) v[rh] = csub(v[rh], cmul(lcol[cc], rdlane(v[rh], cc * CG)));
            }
            if (rg == 0 && r < nb) {
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) {
                    Y[rh * Sz + ((k + r) & msk)] = v[rh];
                    u[(size_t)rh * rstride + k + r] = make_double2((double)v[rh].x, (double)v[rh].y);
                }
            }
            if (p > 0) {                                      // z of panel p-1 for the next step
#pragma unroll
                for (int rh = 0; rh < NR; ++rh) {
                    const double2 z = u[(size_t)rh * rstride + kp + c];
                    zc[rh] = {(R)z.x, (R)z.y};
                }
            }
        } else if (p > 0) {
            // partial far sums of panel p-1: column c, rows k+NB+j for j = rl,
            // rl+RL, ... (rotated by c modulo far_period), j <= c + kd - 2 NB
            const int c = t1 % NB, rl = t1 / NB;
            const int ilast = min(kp + c + kd, n_x - 1);
            cpx<R> part[NR];
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) part[rh] = cz;
            int j = far_period > 0 ? (rl + c) % far_period : 0;
#pragma unroll 4
            for (int j0 = rl; j0 < far_period; j0 += RL) {
                const int i = k + NB + j;
                if (i <= ilast) {
                    const cpx<R> lv = PV(slotq, c, i - kp);
#pragma unroll
                    for (int rh = 0; rh < NR; ++rh) part[rh] = cfma(lv, Y[rh * Sz + (i & msk)], part[rh]);
                }
                j += RL;
                if (j >= far_period) j -= far_period;
            }
#pragma unroll
            for (int rh = 0; rh < NR; ++rh) Pw[(rl * NR + rh) * NB + c] = part[rh];
        }
        lds_barrier();
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

// Shifted spatial blocks of one chunk of eigen-indices, in FP64: system s
// (blockIdx.y) uses S_l = lambda_l M + A with l = l0 + s % cnt (conj:
// conj(lambda_l) M + A); Y_s = S_l X_s, or Y_s = B_s - S_l X_s if B != null.
__global__ __launch_bounds__(256) void k_shifted(const double2* __restrict__ X, double2* __restrict__ Y,
                                                 const double2* __restrict__ B, const double* __restrict__ lam,
                                                 int l0, int cnt, int conj, Stencil st) {
    const int n_x = st.m * st.m;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= n_x) return;
    const int sy = blockIdx.y;
    const size_t base = (size_t)sy * n_x;
    const int l = l0 + sy % cnt;
    const double lr = lam[2 * l], li = conj ? -lam[2 * l + 1] : lam[2 * l + 1];
    double2 Mv, Av;
    stencil_apply(X + base, x, st.m, st, Mv, Av);
    double2 v = make_double2(lr * Mv.x - li * Mv.y + Av.x, lr * Mv.y + li * Mv.x + Av.y);
    if (B) {
        const double2 b = B[base + x];
        v = make_double2(b.x - v.x, b.y - v.y);
    }
    Y[base + x] = v;
}

// ------------------------------------------------------------- Krylov vectors
// Vectors of the Krylov solvers: complex128, nrhs slices of N elements (slice
// r at offset r*N).  A basis holds nv such vectors, vstride complex elements
// apart.  Every reduction runs over gridDim.x (<= VEC_BLOCKS) workgroups per
// slice, then k_partial_reduce sums their partial results.

// Sum of a 64-lane wave, then of the 4 waves of a 256-thread workgroup
// (result valid in thread 0).  `red` holds 4 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// partial[(r*gridDim.x + bx)*2nv + 2i + {0,1}] = workgroup share of
// sum_e conj(V_i[r][e]) w[r][e]
__global__ __launch_bounds__(256) void k_mdot(const double2* __restrict__ V, long long vstride, int nv,
                                              const double2* __restrict__ w, long long N,
                                              double* __restrict__ partial) {
    const int r = blockIdx.y;
    const double2* wr = w + (size_t)r * N;
    const double2* Vr = V + (size_t)r * N;
    double2 acc[KRYLOV_MAX];
#pragma unroll
    for (int i = 0; i < KRYLOV_MAX; ++i) acc[i] = make_double2(0.0, 0.0);
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
        const double2 x = wr[e];
#pragma unroll
        for (int i = 0; i < KRYLOV_MAX; ++i) {
            if (i < nv) {
                const double2 v = Vr[(size_t)i * vstride + e];
                acc[i].x += v.x * x.x + v.y * x.y;
                acc[i].y += v.x * x.y - v.y * x.x;
            }
        }
    }
    __shared__ double red[4];
    double* out = partial + ((size_t)r * gridDim.x + blockIdx.x) * 2 * nv;
#pragma unroll
    for (int i = 0; i < KRYLOV_MAX; ++i) {
        if (i < nv) {
            const double re = block_sum(acc[i].x, red);
            const double im = block_sum(acc[i].y, red);
            if (threadIdx.x == 0) {
                out[2 * i] = re;
                out[2 * i + 1] = im;
            }
        }
    }
}

// w[r] = (accumulate ? w[r] : 0) + sign * sum_i coef[r][i] V_i[r]; with
// partial != null also the workgroup shares of ||w[r]||^2 (new values).
__global__ __launch_bounds__(256) void k_mcomb(double2* __restrict__ w, long long N, const double2* __restrict__ V,
                                               long long vstride, int nv, const double2* __restrict__ coef,
                                               double sign, int accumulate, double* __restrict__ partial) {
    const int r = blockIdx.y;
    double2* wr = w + (size_t)r * N;
    const double2* Vr = V + (size_t)r * N;
    __shared__ double2 c[KRYLOV_MAX];
    if (threadIdx.x < nv) {
        const double2 v = coef[(size_t)r * nv + threadIdx.x];
        c[threadIdx.x] = make_double2(sign * v.x, sign * v.y);
    }
    __syncthreads();
    double nrm = 0.0;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
        double2 x = accumulate ? wr[e] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < KRYLOV_MAX; ++i) {
            if (i < nv) {
                const double2 v = Vr[(size_t)i * vstride + e];
                x.x += c[i].x * v.x - c[i].y * v.y;
                x.y += c[i].x * v.y + c[i].y * v.x;
            }
        }
        wr[e] = x;
        nrm += x.x * x.x + x.y * x.y;
    }
    if (partial) {
        __shared__ double red[4];
        const double t = block_sum(nrm, red);
        if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
    }
}

// workgroup shares of ||x[r]||^2
__global__ __launch_bounds__(256) void k_vnorm2(const double2* __restrict__ x, long long N,
                                                double* __restrict__ partial) {
    const int r = blockIdx.y;
    const double2* xr = x + (size_t)r * N;
    double nrm = 0.0;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
        const double2 v = xr[e];
        nrm += v.x * v.x + v.y * v.y;
    }
    __shared__ double red[4];
    const double t = block_sum(nrm, red);
    if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
}

// y[r] = sc[r] x[r] (sc real, on the device); y may equal x
__global__ __launch_bounds__(256) void k_vscale(double2* y, const double2* x, long long N, const double* sc) {
    const int r = blockIdx.y;
    const double a = sc[r];
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
        const double2 v = x[(size_t)r * N + e];
        y[(size_t)r * N + e] = make_double2(a * v.x, a * v.y);
    }
}

// out[r*width + c] = sum over the nblk shares partial[(r*nblk + b)*width + c]
__global__ __launch_bounds__(256) void k_partial_reduce(const double* __restrict__ partial, int nblk, int width,
                                                        double* __restrict__ out) {
    const int r = blockIdx.x;
    __shared__ double red[4];
    for (int c = 0; c < width; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) v += partial[((size_t)r * nblk + b) * width + c];
        const double t = block_sum(v, red);
        if (threadIdx.x == 0) out[(size_t)r * width + c] = t;
    }
}

__global__ void k_fill_int(int* p, int count, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// LDS of the factorisation: the panel (NB (kd + 1) complex values), D^{-1}
// of two steps, the W table, the column broadcast buffer, the A' operands
// (ceil(kd / TS) tiles x TS rows x NB) and the tile-row counter.
template <class R, int NB>
size_t ldlt_lds_bytes(int kd) {
    constexpr int CPU = Unit<R>::CPU;
    const size_t panel = (size_t)(NB * (kd + 1) + CPU - 1) / CPU * CPU + 2 * NB;
    const size_t tiles = (size_t)(kd + Mma<R>::COLS - 1) / Mma<R>::COLS;
    return (panel + (size_t)NB * NB + 2 * NB + tiles * Mma<R>::COLS * NB) * sizeof(cpx<R>) + 16;
}

template <class R, int NB>
hipError_t launch_ldlt(void* band, int count, const Stencil& st, int* info, hipStream_t s) {
    const size_t lds = ldlt_lds_bytes<R, NB>(st.n);
    auto kern = k_ldlt<R, NB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(count), dim3(256), lds, s, (cpx<R>*)band, st, info);
    return hipGetLastError();
}

// Dynamic LDS of k_sweep: three panel slots, the Y ring, the far-sum partials.
template <class R, int NB, int NR>
size_t sweep_lds_bytes(int kd, int& Sz) {
    Sz = 1;
    while (Sz < kd + 2 * NB) Sz <<= 1;
    constexpr int CPU = Unit<R>::CPU;
    const size_t slot = (size_t)(NB * (kd + 1) + CPU - 1) / CPU;   // 16-byte units
    return 3 * slot * 16 + ((size_t)NR * Sz + 2 * (size_t)(SWEEP_BULK / NB) * NR * NB) * sizeof(cpx<R>);
}
constexpr size_t SWEEP_LDS_CAP = 160u * 1024u;

template <class R, int NB, int NR>
hipError_t launch_sweep_nr(const void* band, int count, const Stencil& st, const double* G, double* U, int conj,
                           long long rstride, hipStream_t s) {
    int Sz = 0;
    const size_t lds = sweep_lds_bytes<R, NB, NR>(st.n, Sz);
    if ((size_t)NB * (st.n + 1) > (size_t)SWEEP_QL * SWEEP_PROD * Unit<R>::CPU || lds > SWEEP_LDS_CAP)
        return hipErrorInvalidValue;
    auto kern = conj ? k_sweep<R, NB, NR, true> : k_sweep<R, NB, NR, false>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(count), dim3(512), lds, s, (const cpx<R>*)band, st, G, U, rstride, Sz);
    return hipGetLastError();
}

// Right-hand sides go through the kernel 4, then 2, then 1 at a time (fewer
// at once where the LDS of 4 or 2 would not fit).
template <class R, int NB>
hipError_t launch_sweep_nb(const void* band, int count, const Stencil& st, const double* G, double* U, int nrhs,
                           int conj, hipStream_t s) {
    const long long rstride = (long long)count * st.m * st.m;   // complex elements between rhs
    int Sz = 0;
    const bool fit4 = sweep_lds_bytes<R, NB, 4>(st.n, Sz) <= SWEEP_LDS_CAP;
    const bool fit2 = sweep_lds_bytes<R, NB, 2>(st.n, Sz) <= SWEEP_LDS_CAP;
    int r0 = 0;
    while (r0 < nrhs) {
        const int left = nrhs - r0;
        const double* Gr = G + (size_t)r0 * rstride * 2;
        double* Ur = U + (size_t)r0 * rstride * 2;
        hipError_t e;
        if (left >= 4 && fit4) {
            e = launch_sweep_nr<R, NB, 4>(band, count, st, Gr, Ur, conj, rstride, s);
            r0 += 4;
        } else if (left >= 2 && fit2) {
            e = launch_sweep_nr<R, NB, 2>(band, count, st, Gr, Ur, conj, rstride, s);
            r0 += 2;
        } else {
            e = launch_sweep_nr<R, NB, 1>(band, count, st, Gr, Ur, conj, rstride, s);
            r0 += 1;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Panel width of the sweeps: the widest of 16, 8, 4, 2 columns that is at
// most kd and whose panel (NB (kd + 1) complex values) fits the SWEEP_QL
// 16-byte loads per thread.
template <class R>
hipError_t launch_sweep(const void* band, int count, const Stencil& st, const double* G, double* U, int nrhs, int conj,
                        hipStream_t s) {
    const size_t cap = (size_t)SWEEP_QL * SWEEP_PROD * Unit<R>::CPU;
    const size_t ld = st.n + 1;
    const int kd = st.n;
    if (16 <= kd && 16 * ld <= cap) return launch_sweep_nb<R, 16>(band, count, st, G, U, nrhs, conj, s);
    if (8 <= kd && 8 * ld <= cap) return launch_sweep_nb<R, 8>(band, count, st, G, U, nrhs, conj, s);
    if (4 <= kd && 4 * ld <= cap) return launch_sweep_nb<R, 4>(band, count, st, G, U, nrhs, conj, s);
    if (2 <= kd && 2 * ld <= cap) return launch_sweep_nb<R, 2>(band, count, st, G, U, nrhs, conj, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t band_fill(int precision, void* band, const double* lambda, int count, const Stencil& st, hipStream_t s) {
    const long long per = (long long)st.m * st.m * (st.n + 1);
    const long long units = precision == 32 ? (per + 1) / 2 : per;
    const int bx = (int)std::min<long long>((units + 256LL * FILL_UPT - 1) / (256LL * FILL_UPT), 1024);
    if (precision == 32)
        hipLaunchKernelGGL(k_band_fill<float>, dim3(bx, count), dim3(256), 0, s, (cpx<float>*)band, lambda, st);
    else
        hipLaunchKernelGGL(k_band_fill<double>, dim3(bx, count), dim3(256), 0, s, (cpx<double>*)band, lambda, st);
    return hipGetLastError();
}

// Panel width: the widest of 32, 16, 8 columns (at most the tile size) whose
// LDS fits in 150 KiB.
hipError_t ldlt_factor(int precision, void* band, int count, const Stencil& st, int* info, hipStream_t s) {
    constexpr size_t cap = 150u * 1024u;
    if (precision == 32) {
        if (ldlt_lds_bytes<float, 32>(st.n) <= cap) return launch_ldlt<float, 32>(band, count, st, info, s);
        if (ldlt_lds_bytes<float, 16>(st.n) <= cap) return launch_ldlt<float, 16>(band, count, st, info, s);
        if (ldlt_lds_bytes<float, 8>(st.n) <= cap) return launch_ldlt<float, 8>(band, count, st, info, s);
    } else {
        if (ldlt_lds_bytes<double, 16>(st.n) <= cap) return launch_ldlt<double, 16>(band, count, st, info, s);
        if (ldlt_lds_bytes<double, 8>(st.n) <= cap) return launch_ldlt<double, 8>(band, count, st, info, s);
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

size_t krylov_partial_size(int nrhs) { return (size_t)nrhs * VEC_BLOCKS * 2 * KRYLOV_MAX; }

// workgroups per slice: about 8 elements per thread, at most VEC_BLOCKS
static int vec_grid(long long N) { return (int)std::min<long long>(VEC_BLOCKS, std::max<long long>(1, (N + 2047) / 2048)); }

hipError_t vec_mdot(const double* V, long long vstride, int nv, const double* w, long long N, int nrhs,
                    double* partial, double* out, hipStream_t s) {
    if (nv < 1 || nv > KRYLOV_MAX) return hipErrorInvalidValue;
    const int vb = vec_grid(N);
    hipLaunchKernelGGL(k_mdot, dim3(vb, nrhs), dim3(256), 0, s, (const double2*)V, vstride, nv, (const double2*)w, N,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_partial_reduce, dim3(nrhs), dim3(256), 0, s, (const double*)partial, vb, 2 * nv, out);
    return hipGetLastError();
}

hipError_t vec_mcomb(double* w, long long N, int nrhs, const double* V, long long vstride, int nv, const double* coef,
                     double sign, int accumulate, double* partial, double* norms, hipStream_t s) {
    if (nv < 0 || nv > KRYLOV_MAX) return hipErrorInvalidValue;
    const int vb = vec_grid(N);
    hipLaunchKernelGGL(k_mcomb, dim3(vb, nrhs), dim3(256), 0, s, (double2*)w, N, (const double2*)V, vstride, nv,
                       (const double2*)coef, sign, accumulate, norms ? partial : (double*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !norms) return e;
    hipLaunchKernelGGL(k_partial_reduce, dim3(nrhs), dim3(256), 0, s, (const double*)partial, vb, 1, norms);
    return hipGetLastError();
}

hipError_t vec_norm2(const double* x, long long N, int nrhs, double* partial, double* norms, hipStream_t s) {
    const int vb = vec_grid(N);
    hipLaunchKernelGGL(k_vnorm2, dim3(vb, nrhs), dim3(256), 0, s, (const double2*)x, N, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_partial_reduce, dim3(nrhs), dim3(256), 0, s, (const double*)partial, vb, 1, norms);
    return hipGetLastError();
}

hipError_t vec_scale(double* y, const double* x, long long N, int nrhs, const double* sc, hipStream_t s) {
    hipLaunchKernelGGL(k_vscale, dim3(vec_grid(N), nrhs), dim3(256), 0, s, (double2*)y, (const double2*)x, N, sc);
    return hipGetLastError();
}

hipError_t shifted_apply(const Stencil& st, const double* lambda, int l0, int cnt, int conj, const double* X,
                         double* Y, const double* B, int nsys, hipStream_t s) {
    const int n_x = st.m * st.m;
    if (nsys < 1 || nsys > 65535 || cnt < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_shifted, dim3((n_x + 255) / 256, nsys), dim3(256), 0, s, (const double2*)X, (double2*)Y,
                       (const double2*)B, lambda, l0, cnt, conj, st);
    return hipGetLastError();
}

hipError_t fill_int(int* p, int count, int value, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

}  // namespace gpu
}  // namespace stfem
