// Fast diagonalization solver (Sec. 3, Kronecker solver steps 1-4 with the
// eigenvalue decomposition) behind the C ABI of include/stfem.h.
//
// K = i B_t (x) M_x + M_t (x) A_x = (M_t X (x) I) blockdiag(S_l) (X^{-1} (x) I)
// with S_l = lambda_l M_x + A_x, hence
//   K^{-1}   = (X (x) I) blockdiag(S_l^{-1}) (W (x) I),        W = (M_t X)^{-1}
//   K^{-H}   = (W^H (x) I) blockdiag(conj(S_l)^{-1}) (X^H (x) I).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace stfem;

#define HIPCHECK(call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(STFEM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

// Pairs of HIP events around kernels of interest, summed per category once the
// stream has been synchronised.
class StageTimer {
  public:
    enum { FILL = 0, LDLT, SWEEP, GEMM, RESID, NCAT };
    ~StageTimer() { release(); }
    hipError_t begin(hipStream_t s) { return mark(s, true); }
    hipError_t end(hipStream_t s, int cat) {
        cats_.push_back(cat);
        return mark(s, false);
    }
    // call after the stream has completed
    void collect(double out[NCAT]) {
        for (int c = 0; c < NCAT; ++c) out[c] = 0;
        for (size_t i = 0; i < cats_.size() && 2 * i + 1 < used_; ++i) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev_[2 * i], ev_[2 * i + 1]) == hipSuccess) out[cats_[i]] += ms;
        }
        cats_.clear();
        used_ = 0;
    }
    void reset() {
        cats_.clear();
        used_ = 0;
    }
    void release() {
        for (auto e : ev_) (void)hipEventDestroy(e);
        ev_.clear();
        cats_.clear();
        used_ = 0;
    }
  private:
    hipError_t mark(hipStream_t s, bool) {
        if (used_ == ev_.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev_.push_back(e);
        }
        return hipEventRecord(ev_[used_++], s);
    }
    std::vector<hipEvent_t> ev_;
    std::vector<int> cats_;
    size_t used_ = 0;
};

struct stfem_blocks {
    int n = 0, m = 0, n_x = 0, kd = 0, count = 0, precision = 64;
    gpu::Stencil st{};
    void* band = nullptr;
    size_t band_bytes = 0;
    int* info = nullptr;
    double* lambda_dev = nullptr;
    std::vector<double> lambda;   // host copy, interleaved complex
    StageTimer timer;
    double ms_fill = 0, ms_ldlt = 0;
};

struct stfem_handle {
    int n_t = 0, n_x = 0, n = 0, w = 0;
    stfem_options opt{};
    TemporalDecomp dec;
    stfem_blocks* blk = nullptr;
    double* X_dev = nullptr;
    double* W_dev = nullptr;
    double* tM_dev = nullptr;
    double* tB_dev = nullptr;
    double* G_ws = nullptr;
    double* R_ws = nullptr;
    size_t ws_elems = 0;          // complex elements of each of G_ws, R_ws
    // GMRES refinement: basis V_0..V_m then Z_0..Z_{m-1}, each nrhs n_t n_x
    // complex128; small device arrays for coefficients and norms
    double* kry = nullptr;
    size_t kry_bytes = 0;
    int kry_nrhs = 0, kry_m = 0;
    double* kry_partial = nullptr;
    double* kry_small = nullptr;  // coef1, coef2 [nrhs][KRYLOV_MAX] complex; nrm, sc [nrhs]
    double* partial = nullptr;
    size_t partial_elems = 0;
    double* norms_dev = nullptr;
    int norms_cap = 0;
    double ms_eig = 0, ms_factor = 0;
    StageTimer timer;
};

namespace {

// Factor storage runs to tens of GB and the solve workspaces to several;
// allocating and releasing them costs milliseconds per GB.  Released buffers
// of >= 64 MiB are kept (at most CACHE_PER_DEVICE per device) and handed to
// the next request that fits in them without wasting more than a quarter; a
// failed allocation first gives them all back, and stfem_release_cache()
// returns them to the device.
struct CachedBuffer {
    void* ptr;
    size_t bytes;
    int device;
};
std::mutex g_cache_mutex;
std::vector<CachedBuffer> g_cache;
constexpr size_t CACHE_MIN_BYTES = (size_t)64 << 20;
constexpr int CACHE_PER_DEVICE = 6;

void release_cache_locked() {
    for (auto& c : g_cache) (void)hipFree(c.ptr);
    g_cache.clear();
}

hipError_t cached_alloc(void** p, size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_cache_mutex);
        for (size_t i = 0; i < g_cache.size(); ++i) {
            const CachedBuffer c = g_cache[i];
            if (c.device == dev && c.bytes >= bytes && c.bytes - bytes <= c.bytes / 4) {
                g_cache.erase(g_cache.begin() + i);
                *p = c.ptr;
                return hipSuccess;
            }
        }
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {   // give the cached buffers back and retry once
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(g_cache_mutex);
        release_cache_locked();
        e = hipMalloc(p, bytes);
    }
    return e;
}

void cached_free(void* p, size_t bytes) {
    if (!p) return;
    if (bytes < CACHE_MIN_BYTES) {
        (void)hipFree(p);
        return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    int same = 0;
    for (auto& c : g_cache) same += (c.device == dev);
    if (same >= CACHE_PER_DEVICE) {   // drop the oldest buffer of this device
        for (size_t i = 0; i < g_cache.size(); ++i)
            if (g_cache[i].device == dev) {
                (void)hipFree(g_cache[i].ptr);
                g_cache.erase(g_cache.begin() + i);
                break;
            }
    }
    g_cache.push_back({p, bytes, dev});
}

bool stencil_ok(const double* Ms, const double* As) {
    for (int q = 0; q < 7; ++q)
        if (!std::isfinite(Ms[q]) || !std::isfinite(As[q])) return false;
    // the factorisation is symmetric: east = west, north = south, NE = SW
    return Ms[STFEM_ST_E] == Ms[STFEM_ST_W] && Ms[STFEM_ST_N] == Ms[STFEM_ST_S] &&
           Ms[STFEM_ST_NE] == Ms[STFEM_ST_SW] && As[STFEM_ST_E] == As[STFEM_ST_W] &&
           As[STFEM_ST_N] == As[STFEM_ST_S] && As[STFEM_ST_NE] == As[STFEM_ST_SW];
}

gpu::Stencil make_stencil(int n, const double* Ms, const double* As) {
    gpu::Stencil st{};
    for (int q = 0; q < 7; ++q) {
        st.M[q] = Ms[q];
        st.A[q] = As[q];
    }
    st.n = n;
    st.m = n - 1;
    return st;
}

size_t elem_bytes(int precision) { return precision == 32 ? 8 : 16; }

void free_blocks(stfem_blocks* b) {
    if (!b) return;
    b->timer.release();
    cached_free(b->band, b->band_bytes);
    if (b->info) (void)hipFree(b->info);
    if (b->lambda_dev) (void)hipFree(b->lambda_dev);
    delete b;
}

// Allocate and enqueue band fill + LDL^T; does not synchronise.
int blocks_launch(int n, const double* Ms, const double* As, const double* lambda, int count, int precision,
                  hipStream_t s, stfem_blocks** out) {
    if (n < 2 || n > 1024) return fail(STFEM_EINVAL, "spatial size: need 2 <= n <= 1024");
    if (count < 1) return fail(STFEM_EINVAL, "block count must be >= 1");
    if (precision != 32 && precision != 64) return fail(STFEM_EINVAL, "precision must be 32 or 64");
    if (!Ms || !As || !lambda) return fail(STFEM_EINVAL, "null stencil or shift array");
    if (!stencil_ok(Ms, As)) return fail(STFEM_EINVAL, "stencils must be finite and symmetric (E=W, N=S, NE=SW)");
    for (int l = 0; l < count; ++l)
        if (!std::isfinite(lambda[2 * l]) || !(lambda[2 * l + 1] > 0.0) || !std::isfinite(lambda[2 * l + 1]))
            return fail(STFEM_EINVAL, "every shift needs a finite value with Im(lambda) > 0");
    auto* b = new stfem_blocks();
    b->n = n;
    b->m = n - 1;
    b->n_x = b->m * b->m;
    b->kd = n;
    b->count = count;
    b->precision = precision;
    b->st = make_stencil(n, Ms, As);
    b->lambda.assign(lambda, lambda + 2 * count);
    const size_t bytes = (size_t)count * gpu::band_stride_host(n) * elem_bytes(precision);
    b->band_bytes = bytes;
    if (cached_alloc(&b->band, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b->band = nullptr;
        free_blocks(b);
        return fail(STFEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes of factors failed");
    }
    if (hipMalloc(&b->info, sizeof(int) * count) != hipSuccess ||
        hipMalloc(&b->lambda_dev, sizeof(double) * 2 * count) != hipSuccess) {
        (void)hipGetLastError();
        free_blocks(b);
        return fail(STFEM_ENOMEM, "device allocation failed");
    }
    hipError_t e = hipMemcpyAsync(b->lambda_dev, lambda, sizeof(double) * 2 * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = gpu::fill_int(b->info, count, 0, s);
    b->timer.reset();
    if (e == hipSuccess) e = b->timer.begin(s);
    if (e == hipSuccess) e = gpu::band_fill(precision, b->band, b->lambda_dev, count, b->st, s);
    if (e == hipSuccess) e = b->timer.end(s, StageTimer::FILL);
    if (e == hipSuccess) e = b->timer.begin(s);
    if (e == hipSuccess) e = gpu::ldlt_factor(precision, b->band, count, b->st, b->info, s);
    if (e == hipSuccess) e = b->timer.end(s, StageTimer::LDLT);
    if (e != hipSuccess) {
        free_blocks(b);
        return fail(STFEM_EHIP, std::string("factor launch: ") + hipGetErrorString(e));
    }
    *out = b;
    return STFEM_OK;
}

// Synchronise and check the pivot flags.
int blocks_finish(stfem_blocks* b, hipStream_t s) {
    HIPCHECK(hipStreamSynchronize(s));
    double t[StageTimer::NCAT];
    b->timer.collect(t);
    b->ms_fill = t[StageTimer::FILL];
    b->ms_ldlt = t[StageTimer::LDLT];
    std::vector<int> info(b->count);
    HIPCHECK(hipMemcpy(info.data(), b->info, sizeof(int) * b->count, hipMemcpyDeviceToHost));
    for (int l = 0; l < b->count; ++l)
        if (info[l] != 0)
            return fail(STFEM_EBREAKDOWN, "zero or non-finite pivot in block " + std::to_string(l) + " at column " +
                                              std::to_string(info[l] - 1));
    return STFEM_OK;
}

int ensure_workspace(stfem_handle* h, int nrhs) {
    const size_t need = (size_t)nrhs * h->n_t * h->n_x;
    if (need > h->ws_elems) {
        cached_free(h->G_ws, h->ws_elems * 16);
        cached_free(h->R_ws, h->ws_elems * 16);
        h->G_ws = h->R_ws = nullptr;
        h->ws_elems = 0;
        if (cached_alloc((void**)&h->G_ws, need * 16) != hipSuccess ||
            cached_alloc((void**)&h->R_ws, need * 16) != hipSuccess) {
            (void)hipGetLastError();
            cached_free(h->G_ws, need * 16);
            h->G_ws = h->R_ws = nullptr;
            return fail(STFEM_ENOMEM, "solve workspace allocation failed");
        }
        h->ws_elems = need;
    }
    const size_t pneed = gpu::residual_partial_size(nrhs, h->n_t, h->n_x);
    if (pneed > h->partial_elems) {
        if (h->partial) (void)hipFree(h->partial);
        h->partial = nullptr;
        if (hipMalloc(&h->partial, pneed * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            h->partial_elems = 0;
            return fail(STFEM_ENOMEM, "residual scratch allocation failed");
        }
        h->partial_elems = pneed;
    }
    if (nrhs > h->norms_cap) {
        if (h->norms_dev) (void)hipFree(h->norms_dev);
        h->norms_dev = nullptr;
        if (hipMalloc(&h->norms_dev, sizeof(double) * 2 * nrhs) != hipSuccess) {
            (void)hipGetLastError();
            h->norms_cap = 0;
            return fail(STFEM_ENOMEM, "norm buffer allocation failed");
        }
        h->norms_cap = nrhs;
    }
    return STFEM_OK;
}

// max over rhs of ||R||/||F|| (from the device norm pairs); synchronises.
int read_relres(stfem_handle* h, int nrhs, hipStream_t s, double& rel) {
    std::vector<double> nv(2 * nrhs);
    HIPCHECK(hipMemcpyAsync(nv.data(), h->norms_dev, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    rel = 0;
    for (int r = 0; r < nrhs; ++r) {
        const double ff = nv[2 * r + 1], rr = nv[2 * r];
        const double v = ff > 0 ? std::sqrt(rr / ff) : (rr > 0 ? INFINITY : 0.0);
        rel = std::max(rel, std::isfinite(v) ? v : INFINITY);
    }
    return STFEM_OK;
}

// One application of K^{-1} (adjoint: K^{-H}) to `in`, written to (or added
// to) `out`, using G_ws as the transformed buffer.
int apply_inverse(stfem_handle* h, const double* in, double* out, int nrhs, int adjoint, int accumulate,
                  hipStream_t s) {
    const int nt = h->n_t, nx = h->n_x;
    const long long N = (long long)nt * nx;
    stfem_blocks* b = h->blk;
    StageTimer& T = h->timer;
    const double* first = adjoint ? h->X_dev : h->W_dev;
    const double* second = adjoint ? h->W_dev : h->X_dev;
    HIPCHECK(T.begin(s));
    HIPCHECK(gpu::zgemm_small_left(nt, nx, nrhs, first, adjoint, in, N, h->G_ws, N, 0, s));
    HIPCHECK(T.end(s, StageTimer::GEMM));
    HIPCHECK(T.begin(s));
    HIPCHECK(gpu::sweep_solve(b->precision, b->band, b->count, b->st, h->G_ws, h->G_ws, nrhs, adjoint, s));
    HIPCHECK(T.end(s, StageTimer::SWEEP));
    HIPCHECK(T.begin(s));
    HIPCHECK(gpu::zgemm_small_left(nt, nx, nrhs, second, adjoint, h->G_ws, N, out, N, accumulate, s));
    HIPCHECK(T.end(s, StageTimer::GEMM));
    return STFEM_OK;
}

// ------------------------------------------------------- GMRES refinement
// Krylov storage for nrhs right-hand sides: 2m+1 arrays of nrhs n_t n_x
// complex128, m <= KRYLOV_MAX - 1 and within KRYLOV_BUDGET.
constexpr size_t KRYLOV_BUDGET = (size_t)16 << 30;

int ensure_krylov(stfem_handle* h, int nrhs) {
    const size_t vec = (size_t)nrhs * h->n_t * h->n_x * 16;
    const size_t fit = KRYLOV_BUDGET / vec >= 3 ? (KRYLOV_BUDGET / vec - 1) / 2 : 1;
    const size_t want = h->opt.restart > 0 ? (size_t)h->opt.restart : (size_t)h->opt.max_iter + 1;
    const int m = (int)std::max<size_t>(1, std::min<size_t>({want, (size_t)gpu::KRYLOV_MAX - 1, fit}));
    const size_t need = (2 * (size_t)m + 1) * vec;
    if (need > h->kry_bytes) {
        cached_free(h->kry, h->kry_bytes);
        h->kry = nullptr;
        h->kry_bytes = 0;
        if (cached_alloc((void**)&h->kry, need) != hipSuccess) {
            (void)hipGetLastError();
            h->kry = nullptr;
            return fail(STFEM_ENOMEM, "Krylov basis allocation failed");
        }
        h->kry_bytes = need;
    }
    if (nrhs > h->kry_nrhs) {
        if (h->kry_partial) (void)hipFree(h->kry_partial);
        if (h->kry_small) (void)hipFree(h->kry_small);
        h->kry_partial = h->kry_small = nullptr;
        h->kry_nrhs = 0;
        if (hipMalloc(&h->kry_partial, gpu::krylov_partial_size(nrhs) * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->kry_small, ((size_t)4 * gpu::KRYLOV_MAX + 2) * nrhs * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(STFEM_ENOMEM, "Krylov scratch allocation failed");
        }
        h->kry_nrhs = nrhs;
    }
    h->kry_m = m;
    return STFEM_OK;
}

typedef std::complex<double> zd;

// Flexible GMRES on K Psi = F (adjoint: K^H) with the FDM inverse as right
// preconditioner, started from Psi = 0 and restarted every m columns; each
// rhs has its own Hessenberg matrix, all rhs share the batched kernels.  Every
// residual and basis vector is FP64; the preconditioner runs in the factor
// precision.  Orthogonalisation: classical Gram-Schmidt, twice.
int refine_gmres(stfem_handle* h, const double* F, double* Psi, int nrhs, int adjoint, hipStream_t s, int& applied,
                 double& rel, double* hist) {
    int st = ensure_krylov(h, nrhs);
    if (st) return st;
    const int m = h->kry_m, KM = gpu::KRYLOV_MAX;
    const long long N = (long long)h->n_t * h->n_x;
    const long long vs = (long long)nrhs * N;                  // complex elements per basis array
    double* V = h->kry;
    double* Z = h->kry + 2 * (size_t)(m + 1) * vs;
    auto Vp = [&](int i) { return V + 2 * (size_t)i * vs; };
    auto Zp = [&](int i) { return Z + 2 * (size_t)i * vs; };
    double* coef1 = h->kry_small;                              // [nrhs][KM] complex
    double* coef2 = coef1 + 2 * (size_t)KM * nrhs;
    double* nrm = coef2 + 2 * (size_t)KM * nrhs;               // [nrhs]
    double* sc = nrm + nrhs;                                   // [nrhs]
    double* part = h->kry_partial;
    StageTimer& T = h->timer;
    const int max_apply = 1 + h->opt.max_iter;
    const double tol = h->opt.tol;

    std::vector<double> fn(nrhs), beta(nrhs), nh(nrhs), sh(nrhs);
    std::vector<double> c1(2 * (size_t)KM * nrhs), c2(2 * (size_t)KM * nrhs);
    HIPCHECK(T.begin(s));
    HIPCHECK(gpu::vec_norm2(F, N, nrhs, part, nrm, s));
    HIPCHECK(T.end(s, StageTimer::RESID));
    HIPCHECK(hipMemcpyAsync(fn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) beta[r] = fn[r] = std::sqrt(fn[r]);

    std::vector<zd> H((size_t)nrhs * (m + 1) * m), g((size_t)nrhs * (m + 1)), sn((size_t)nrhs * m);
    std::vector<double> cs((size_t)nrhs * m);
    auto Hat = [&](int r, int i, int j) -> zd& { return H[((size_t)r * (m + 1) + i) * m + j]; };
    const double* r0 = F;
    bool first = true;
    applied = 0;
    rel = INFINITY;
    for (;;) {
        // V_0 = r0 / beta
        for (int r = 0; r < nrhs; ++r) sh[r] = beta[r] > 0 && std::isfinite(beta[r]) ? 1.0 / beta[r] : 0.0;
        HIPCHECK(hipMemcpyAsync(sc, sh.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::vec_scale(Vp(0), r0, N, nrhs, sc, s));
        HIPCHECK(T.end(s, StageTimer::RESID));
        std::fill(H.begin(), H.end(), zd(0));
        std::fill(g.begin(), g.end(), zd(0));
        for (int r = 0; r < nrhs; ++r) g[(size_t)r * (m + 1)] = beta[r];
        int ncol = 0;
        while (ncol < m && applied < max_apply) {
            const int j = ncol;
            st = apply_inverse(h, Vp(j), Zp(j), nrhs, adjoint, 0, s);
            if (st) return st;
            ++applied;
            HIPCHECK(T.begin(s));
            HIPCHECK(gpu::kron_apply(Zp(j), Vp(j + 1), nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev, h->blk->st, adjoint,
                                     s));
            HIPCHECK(gpu::vec_mdot(V, vs, j + 1, Vp(j + 1), N, nrhs, part, coef1, s));
            HIPCHECK(gpu::vec_mcomb(Vp(j + 1), N, nrhs, V, vs, j + 1, coef1, -1.0, 1, part, nullptr, s));
            HIPCHECK(gpu::vec_mdot(V, vs, j + 1, Vp(j + 1), N, nrhs, part, coef2, s));
            HIPCHECK(gpu::vec_mcomb(Vp(j + 1), N, nrhs, V, vs, j + 1, coef2, -1.0, 1, part, nrm, s));
            HIPCHECK(T.end(s, StageTimer::RESID));
            const size_t cb = sizeof(double) * 2 * (size_t)(j + 1) * nrhs;
            HIPCHECK(hipMemcpyAsync(c1.data(), coef1, cb, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipMemcpyAsync(c2.data(), coef2, cb, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipMemcpyAsync(nh.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            double est = 0;
            for (int r = 0; r < nrhs; ++r) {
                for (int i = 0; i <= j; ++i) {
                    const size_t q = 2 * ((size_t)r * (j + 1) + i);
                    Hat(r, i, j) = zd(c1[q] + c2[q], c1[q + 1] + c2[q + 1]);
                }
                const double hn = std::sqrt(nh[r]);
                sh[r] = hn > 0 && std::isfinite(1.0 / hn) ? 1.0 / hn : 0.0;
                // previous rotations, then the one that zeroes H[j+1][j]
                for (int i = 0; i < j; ++i) {
                    const double c = cs[(size_t)r * m + i];
                    const zd sv = sn[(size_t)r * m + i];
                    const zd a = Hat(r, i, j), b = Hat(r, i + 1, j);
                    Hat(r, i, j) = c * a + sv * b;
                    Hat(r, i + 1, j) = -std::conj(sv) * a + c * b;
                }
                const zd a = Hat(r, j, j);
                const double rho = std::hypot(std::abs(a), hn);
                double c = 1.0;
                zd sv = 0.0;
                if (rho > 0) {
                    if (std::abs(a) > 0) {
                        c = std::abs(a) / rho;
                        sv = (a / std::abs(a)) * hn / rho;
                    } else {
                        c = 0.0;
                        sv = 1.0;
                    }
                }
                cs[(size_t)r * m + j] = c;
                sn[(size_t)r * m + j] = sv;
                Hat(r, j, j) = c * a + sv * hn;
                zd& gj = g[(size_t)r * (m + 1) + j];
                g[(size_t)r * (m + 1) + j + 1] = -std::conj(sv) * gj;
                gj = c * gj;
                if (fn[r] > 0) est = std::max(est, std::abs(g[(size_t)r * (m + 1) + j + 1]) / fn[r]);
            }
            HIPCHECK(hipMemcpyAsync(sc, sh.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
            HIPCHECK(T.begin(s));
            HIPCHECK(gpu::vec_scale(Vp(j + 1), Vp(j + 1), N, nrhs, sc, s));
            HIPCHECK(T.end(s, StageTimer::RESID));
            if (applied <= 16) hist[applied - 1] = est;
            ++ncol;
            if (!(est > 0.5 * tol)) break;      // also stops on NaN
        }
        // y = R^{-1} g per rhs, then Psi (+)= Z y
        for (int r = 0; r < nrhs; ++r) {
            std::vector<zd> y(ncol);
            for (int i = ncol - 1; i >= 0; --i) {
                zd t = g[(size_t)r * (m + 1) + i];
                for (int k = i + 1; k < ncol; ++k) t -= Hat(r, i, k) * y[k];
                const zd d = Hat(r, i, i);
                y[i] = std::abs(d) > 0 ? t / d : zd(0);
            }
            for (int i = 0; i < ncol; ++i) {
                c1[2 * ((size_t)r * ncol + i)] = y[i].real();
                c1[2 * ((size_t)r * ncol + i) + 1] = y[i].imag();
            }
        }
        HIPCHECK(hipMemcpyAsync(coef1, c1.data(), sizeof(double) * 2 * (size_t)ncol * nrhs, hipMemcpyHostToDevice, s));
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::vec_mcomb(Psi, N, nrhs, Z, vs, ncol, coef1, 1.0, first ? 0 : 1, part, nullptr, s));
        first = false;
        // recomputed residual
        HIPCHECK(gpu::kron_residual(Psi, F, h->R_ws, nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev, h->blk->st, adjoint,
                                    h->partial, h->norms_dev, s));
        HIPCHECK(T.end(s, StageTimer::RESID));
        std::vector<double> nv(2 * (size_t)nrhs);
        HIPCHECK(hipMemcpyAsync(nv.data(), h->norms_dev, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        rel = 0;
        for (int r = 0; r < nrhs; ++r) {
            beta[r] = std::sqrt(nv[2 * r]);
            const double v = fn[r] > 0 ? beta[r] / fn[r] : (beta[r] > 0 ? INFINITY : 0.0);
            rel = std::max(rel, std::isfinite(v) ? v : INFINITY);
        }
        if (applied >= 1 && applied <= 16) hist[applied - 1] = rel;
        if (rel <= tol || applied >= max_apply || !std::isfinite(rel)) break;
        r0 = h->R_ws;
    }
    return STFEM_OK;
}

int solve_common(stfem_handle* h, const void* F_dev, void* Psi_dev, int nrhs, void* stream, stfem_report* rep,
                 int adjoint) {
    clear_error();
    const double t0 = now_ms();
    if (!h || !F_dev || !Psi_dev || nrhs < 1) return fail(STFEM_EINVAL, "fdm_solve: null handle/array or nrhs < 1");
    if (F_dev == Psi_dev) return fail(STFEM_EINVAL, "fdm_solve: F and Psi must not overlap");
    hipStream_t s = (hipStream_t)stream;
    h->timer.reset();
    int st = ensure_workspace(h, nrhs);
    if (st) return st;
    const double* F = (const double*)F_dev;
    double* Psi = (double*)Psi_dev;
    int it = 0;
    double rel = -1.0;
    double hist[16];
    for (double& x : hist) x = -1.0;
    if (h->opt.tol > 0 && h->opt.refine == STFEM_REFINE_GMRES) {
        int applied = 0;
        st = refine_gmres(h, F, Psi, nrhs, adjoint, s, applied, rel, hist);
        if (st) return st;
        it = applied - 1;
    } else {
        st = apply_inverse(h, F, Psi, nrhs, adjoint, 0, s);
        if (st) return st;
        if (h->opt.tol > 0) {
            for (;;) {
                HIPCHECK(h->timer.begin(s));
                HIPCHECK(gpu::kron_residual(Psi, F, h->R_ws, nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev,
                                            h->blk->st, adjoint, h->partial, h->norms_dev, s));
                HIPCHECK(h->timer.end(s, StageTimer::RESID));
                st = read_relres(h, nrhs, s, rel);
                if (st) return st;
                if (it < 16) hist[it] = rel;
                if (rel <= h->opt.tol || it >= h->opt.max_iter || !std::isfinite(rel)) break;
                st = apply_inverse(h, h->R_ws, Psi, nrhs, adjoint, 1, s);
                if (st) return st;
                ++it;
            }
        }
    }
    HIPCHECK(hipStreamSynchronize(s));
    double t[StageTimer::NCAT];
    h->timer.collect(t);
    if (rep) {
        rep->ms_band_fill = h->blk->ms_fill;
        rep->ms_ldlt = h->blk->ms_ldlt;
        rep->ms_sweeps = t[StageTimer::SWEEP];
        rep->ms_transforms = t[StageTimer::GEMM];
        rep->ms_residual = t[StageTimer::RESID];
        rep->iterations = it;
        std::memcpy(rep->history, hist, sizeof hist);
        rep->rel_residual = rel;
        rep->kappa_x = h->dec.kappa;
        rep->ms_eig = h->ms_eig;
        rep->ms_factor = h->ms_factor;
        rep->ms_total = now_ms() - t0;
    }
    if (h->opt.tol > 0 && !(rel <= h->opt.tol)) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "refinement stopped at relative residual %.3e (tolerance %.3e) after %d applications of the "
                      "inverse", rel, h->opt.tol, it + 1);
        return fail(STFEM_ENOCONV, msg);
    }
    return STFEM_OK;
}

}  // namespace

// ======================================================== batched shifted blocks
extern "C" int shifted_factor(int n, const double* M_stencil, const double* A_stencil, const double* lambda, int count,
                              int precision, void* stream, stfem_blocks** out) {
    clear_error();
    if (!out) return fail(STFEM_EINVAL, "shifted_factor: null output handle");
    *out = nullptr;
    stfem_blocks* b = nullptr;
    int st = blocks_launch(n, M_stencil, A_stencil, lambda, count, precision, (hipStream_t)stream, &b);
    if (st) return st;
    st = blocks_finish(b, (hipStream_t)stream);
    if (st) {
        free_blocks(b);
        return st;
    }
    *out = b;
    return STFEM_OK;
}

extern "C" int shifted_solve(stfem_blocks* b, const void* G_dev, void* U_dev, int nrhs, int conj, void* stream) {
    clear_error();
    if (!b || !G_dev || !U_dev || nrhs < 1) return fail(STFEM_EINVAL, "shifted_solve: null argument or nrhs < 1");
    HIPCHECK(gpu::sweep_solve(b->precision, b->band, b->count, b->st, (const double*)G_dev, (double*)U_dev, nrhs,
                              conj ? 1 : 0, (hipStream_t)stream));
    return STFEM_OK;
}

extern "C" int shifted_factor_band(const stfem_blocks* b, int l, double* band) {
    clear_error();
    if (!b || !band || l < 0 || l >= b->count) return fail(STFEM_EINVAL, "shifted_factor_band: bad argument");
    const size_t per = (size_t)b->n_x * (b->kd + 1);
    const size_t stride = (size_t)gpu::band_stride_host(b->n);
    if (b->precision == 64) {
        HIPCHECK(hipMemcpy(band, (const char*)b->band + (size_t)l * stride * 16, per * 16, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * per);
        HIPCHECK(hipMemcpy(tmp.data(), (const char*)b->band + (size_t)l * stride * 8, per * 8, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < 2 * per; ++i) band[i] = tmp[i];
    }
    return STFEM_OK;
}

extern "C" void shifted_destroy(stfem_blocks* b) { free_blocks(b); }

// ===================================================================== FDM
extern "C" int fdm_temporal(const double* M_t, const double* B_t, int n_t, double* lambda, double* X, double* W,
                            double* kappa, int* iters) {
    clear_error();
    if (!M_t || !B_t || n_t < 1) return fail(STFEM_EINVAL, "fdm_temporal: null temporal matrices or n_t < 1");
    TemporalDecomp d;
    int st = temporal_decompose(M_t, B_t, n_t, d);
    if (st) return st;
    const size_t n = n_t;
    if (lambda) std::memcpy(lambda, d.lambda.data(), n * 16);
    if (X) std::memcpy(X, d.X.data(), n * n * 16);
    if (W) std::memcpy(W, d.W.data(), n * n * 16);
    if (kappa) *kappa = temporal_kappa(d);
    if (iters) *iters = d.aberth_iters;
    return STFEM_OK;
}

extern "C" int fdm_factor(const double* M_t, const double* B_t, int n_t, const double* M_stencil,
                          const double* A_stencil, int n, const stfem_options* opt, void* stream, stfem_handle** out) {
    clear_error();
    if (!out) return fail(STFEM_EINVAL, "fdm_factor: null output handle");
    *out = nullptr;
    if (!M_t || !B_t || n_t < 1) return fail(STFEM_EINVAL, "fdm_factor: null temporal matrices or n_t < 1");
    stfem_options o{64, 0, 0.0, STFEM_REFINE_GMRES, 0};
    if (opt) o = *opt;
    if (o.precision != 32 && o.precision != 64) return fail(STFEM_EINVAL, "fdm_factor: precision must be 32 or 64");
    if (o.max_iter < 0) return fail(STFEM_EINVAL, "fdm_factor: max_iter must be >= 0");
    if (o.refine != STFEM_REFINE_GMRES && o.refine != STFEM_REFINE_PLAIN)
        return fail(STFEM_EINVAL, "fdm_factor: refine must be STFEM_REFINE_GMRES or STFEM_REFINE_PLAIN");
    if (o.restart < 0) return fail(STFEM_EINVAL, "fdm_factor: restart must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const double t0 = now_ms();
    auto* h = new stfem_handle();
    h->n_t = n_t;
    h->n = n;
    h->n_x = (n - 1) * (n - 1);
    h->opt = o;
    int st = temporal_decompose(M_t, B_t, n_t, h->dec);
    if (st) {
        delete h;
        return st;
    }
    h->w = h->dec.band_w;
    const double t1 = now_ms();
    h->ms_eig = t1 - t0;
    std::vector<double> lam(2 * n_t);
    for (int l = 0; l < n_t; ++l) {
        lam[2 * l] = h->dec.lambda[l].re;
        lam[2 * l + 1] = h->dec.lambda[l].im;
    }
    st = blocks_launch(n, M_stencil, A_stencil, lam.data(), n_t, o.precision, s, &h->blk);
    if (st) {
        delete h;
        return st;
    }
    // host work overlapping the GPU factorisation
    h->dec.kappa = temporal_kappa(h->dec);
    const int bw = 2 * h->w + 1;
    std::vector<double> tM((size_t)n_t * bw, 0.0), tB((size_t)n_t * bw, 0.0);
    for (int i = 0; i < n_t; ++i)
        for (int j = std::max(0, i - h->w); j <= std::min(n_t - 1, i + h->w); ++j) {
            tM[(size_t)i * bw + (j - i + h->w)] = M_t[(size_t)i * n_t + j];
            tB[(size_t)i * bw + (j - i + h->w)] = B_t[(size_t)i * n_t + j];
        }
    auto cleanup = [&](int code) {
        fdm_destroy(h);
        return code;
    };
    const size_t mat = (size_t)n_t * n_t * 16;
    if (hipMalloc(&h->X_dev, mat) != hipSuccess || hipMalloc(&h->W_dev, mat) != hipSuccess ||
        hipMalloc(&h->tM_dev, tM.size() * 8) != hipSuccess || hipMalloc(&h->tB_dev, tB.size() * 8) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(STFEM_ENOMEM, "fdm_factor: device allocation failed"));
    }
    if (hipMemcpyAsync(h->X_dev, h->dec.X.data(), mat, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->W_dev, h->dec.W.data(), mat, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->tM_dev, tM.data(), tM.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->tB_dev, tB.data(), tB.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(STFEM_EHIP, "fdm_factor: upload failed"));
    st = blocks_finish(h->blk, s);
    if (st) return cleanup(st);
    h->ms_factor = now_ms() - t1;
    *out = h;
    return STFEM_OK;
}

extern "C" int fdm_solve(stfem_handle* h, const void* F_dev, void* Psi_dev, int nrhs, void* stream,
                         stfem_report* rep) {
    return solve_common(h, F_dev, Psi_dev, nrhs, stream, rep, 0);
}

extern "C" int fdm_solve_adjoint(stfem_handle* h, const void* G_dev, void* Lam_dev, int nrhs, void* stream,
                                 stfem_report* rep) {
    return solve_common(h, G_dev, Lam_dev, nrhs, stream, rep, 1);
}

extern "C" int fdm_apply(stfem_handle* h, const void* Psi_dev, void* Y_dev, int nrhs, int adjoint, void* stream) {
    clear_error();
    if (!h || !Psi_dev || !Y_dev || nrhs < 1 || Psi_dev == Y_dev)
        return fail(STFEM_EINVAL, "fdm_apply: bad argument (arrays must not overlap)");
    HIPCHECK(gpu::kron_apply((const double*)Psi_dev, (double*)Y_dev, nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev,
                             h->blk->st, adjoint ? 1 : 0, (hipStream_t)stream));
    return STFEM_OK;
}

extern "C" int fdm_decomposition(const stfem_handle* h, double* lambda, double* X, double* W, double* kappa) {
    clear_error();
    if (!h) return fail(STFEM_EINVAL, "fdm_decomposition: null handle");
    const size_t n = h->n_t;
    if (lambda) std::memcpy(lambda, h->dec.lambda.data(), n * 16);
    if (X) std::memcpy(X, h->dec.X.data(), n * n * 16);
    if (W) std::memcpy(W, h->dec.W.data(), n * n * 16);
    if (kappa) *kappa = h->dec.kappa;
    return STFEM_OK;
}

extern "C" int fdm_sizes(const stfem_handle* h, int* n_t, int* n_x, int* n, int* precision) {
    clear_error();
    if (!h) return fail(STFEM_EINVAL, "fdm_sizes: null handle");
    if (n_t) *n_t = h->n_t;
    if (n_x) *n_x = h->n_x;
    if (n) *n = h->n;
    if (precision) *precision = h->opt.precision;
    return STFEM_OK;
}

extern "C" void fdm_destroy(stfem_handle* h) {
    if (!h) return;
    h->timer.release();
    free_blocks(h->blk);
    cached_free(h->G_ws, h->ws_elems * 16);
    cached_free(h->R_ws, h->ws_elems * 16);
    cached_free(h->kry, h->kry_bytes);
    for (double* p : {h->X_dev, h->W_dev, h->tM_dev, h->tB_dev, h->partial, h->norms_dev, h->kry_partial,
                      h->kry_small})
        if (p) (void)hipFree(p);
    delete h;
}

extern "C" void stfem_release_cache(void) {
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    release_cache_locked();
}

// ============================================================ spatial apply
extern "C" int apply_spatial(int n, const double* M_stencil, const double* A_stencil, double alpha_re, double alpha_im,
                             double beta_re, double beta_im, const void* X_dev, void* Y_dev, int count, void* stream) {
    clear_error();
    if (n < 2 || !M_stencil || !A_stencil || !X_dev || !Y_dev || count < 1 || X_dev == Y_dev)
        return fail(STFEM_EINVAL, "apply_spatial: bad argument (arrays must not overlap)");
    gpu::Stencil st = make_stencil(n, M_stencil, A_stencil);
    HIPCHECK(gpu::spatial_apply(st, alpha_re, alpha_im, beta_re, beta_im, (const double*)X_dev, (double*)Y_dev, count,
                                (hipStream_t)stream));
    return STFEM_OK;
}
