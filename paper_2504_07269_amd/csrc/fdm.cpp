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
#include <functional>
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
    int cap = 0;                  // blocks the factor buffer holds
    int l0 = 0, nf = 0;           // eigen-indices [l0, l0 + nf) in the factor buffer
    bool factored = false;        // ... and factored without breakdown
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
    double* kry_small = nullptr;  // coef1, coef2 [nsys][KRYLOV_MAX] complex; nrm, sc [nsys]
    // eigen-chunking: the factors of blk->cap blocks at a time, recomputed
    // chunk by chunk in every solve (nchunks > 1)
    int nchunks = 1;
    double amp_fwd = 1.0, amp_adj = 1.0;  // ||M_t X||_2 and ||X^{-1}||_2
    double* U_ws = nullptr;               // transformed solution, all eigen-indices
    size_t u_elems = 0;
    double* Gc = nullptr;                 // one chunk: rhs, solution, residual
    double* Uc = nullptr;
    double* Rc = nullptr;
    size_t chunk_elems = 0;
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
constexpr int CACHE_PER_DEVICE = 12;

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

// Bytes held by the cache for the current device.
size_t cached_bytes() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    size_t t = 0;
    for (auto& c : g_cache)
        if (c.device == dev) t += c.bytes;
    return t;
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
// Validate, allocate factor storage for `cap` blocks and upload the `count`
// shifts; nothing is factored yet.
int blocks_create(int n, const double* Ms, const double* As, const double* lambda, int count, int cap, int precision,
                  hipStream_t s, stfem_blocks** out) {
    if (n < 2 || n > 1024) return fail(STFEM_EINVAL, "spatial size: need 2 <= n <= 1024");
    if (count < 1 || cap < 1 || cap > count) return fail(STFEM_EINVAL, "block count must be >= 1");
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
    b->cap = cap;
    b->precision = precision;
    b->st = make_stencil(n, Ms, As);
    b->lambda.assign(lambda, lambda + 2 * count);
    const size_t bytes = (size_t)cap * gpu::band_stride_host(n) * elem_bytes(precision);
    b->band_bytes = bytes;
    if (cached_alloc(&b->band, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b->band = nullptr;
        free_blocks(b);
        return fail(STFEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes of factors failed");
    }
    if (hipMalloc(&b->info, sizeof(int) * cap) != hipSuccess ||
        hipMalloc(&b->lambda_dev, sizeof(double) * 2 * count) != hipSuccess) {
        (void)hipGetLastError();
        free_blocks(b);
        return fail(STFEM_ENOMEM, "device allocation failed");
    }
    if (hipMemcpyAsync(b->lambda_dev, lambda, sizeof(double) * 2 * count, hipMemcpyHostToDevice, s) != hipSuccess) {
        free_blocks(b);
        return fail(STFEM_EHIP, "shift upload failed");
    }
    *out = b;
    return STFEM_OK;
}

// Enqueue band fill + LDL^T of the shifts [l0, l0 + nf) into the factor
// buffer; does not synchronise.
int blocks_factor(stfem_blocks* b, int l0, int nf, hipStream_t s) {
    if (l0 < 0 || nf < 1 || nf > b->cap || l0 + nf > b->count) return fail(STFEM_EINVAL, "bad block range");
    b->l0 = l0;
    b->nf = nf;
    b->factored = false;
    hipError_t e = gpu::fill_int(b->info, nf, 0, s);
    b->timer.reset();
    if (e == hipSuccess) e = b->timer.begin(s);
    if (e == hipSuccess) e = gpu::band_fill(b->precision, b->band, b->lambda_dev + 2 * (size_t)l0, nf, b->st, s);
    if (e == hipSuccess) e = b->timer.end(s, StageTimer::FILL);
    if (e == hipSuccess) e = b->timer.begin(s);
    if (e == hipSuccess) e = gpu::ldlt_factor(b->precision, b->band, nf, b->st, b->info, s);
    if (e == hipSuccess) e = b->timer.end(s, StageTimer::LDLT);
    if (e != hipSuccess) return fail(STFEM_EHIP, std::string("factor launch: ") + hipGetErrorString(e));
    return STFEM_OK;
}

// All `count` shifts at once; does not synchronise.
int blocks_launch(int n, const double* Ms, const double* As, const double* lambda, int count, int precision,
                  hipStream_t s, stfem_blocks** out) {
    stfem_blocks* b = nullptr;
    int st = blocks_create(n, Ms, As, lambda, count, count, precision, s, &b);
    if (st) return st;
    st = blocks_factor(b, 0, count, s);
    if (st) {
        free_blocks(b);
        return st;
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
    std::vector<int> info(b->nf);
    HIPCHECK(hipMemcpy(info.data(), b->info, sizeof(int) * b->nf, hipMemcpyDeviceToHost));
    for (int l = 0; l < b->nf; ++l)
        if (info[l] != 0)
            return fail(STFEM_EBREAKDOWN, "zero or non-finite pivot in block " + std::to_string(b->l0 + l) +
                                              " at column " + std::to_string(info[l] - 1));
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
    HIPCHECK(gpu::sweep_solve(b->precision, b->band, b->nf, b->st, h->G_ws, h->G_ws, nrhs, adjoint, s));
    HIPCHECK(T.end(s, StageTimer::SWEEP));
    HIPCHECK(T.begin(s));
    HIPCHECK(gpu::zgemm_small_left(nt, nx, nrhs, second, adjoint, h->G_ws, N, out, N, accumulate, s));
    HIPCHECK(T.end(s, StageTimer::GEMM));
    return STFEM_OK;
}

// ------------------------------------------------------- flexible GMRES
// nsys independent systems A_s x_s = b_s of N complex128 unknowns each, stored
// one after the other and solved together: batched kernels, one Hessenberg
// matrix per system on the host.  Right preconditioner M^{-1} (flexible:
// the preconditioned vectors Z are kept), started from x = 0, restarted every
// m columns; every cycle ends with a recomputed residual.  A system whose
// recomputed residual did not halve over a cycle has reached the accuracy
// its FP64 residual allows and stops.  Orthogonalisation: classical
// Gram-Schmidt, applied twice.
struct KrylovSystems {
    int nsys = 0;
    long long N = 0;
    std::function<int(const double* in, double* out)> prec;   // out = M^{-1} in
    std::function<int(const double* in, double* out)> op;     // out = A in
    // out = b - A x and rr[s] = ||out_s||^2 on the host (synchronises)
    std::function<int(const double* x, double* out, std::vector<double>& rr)> residual;
    std::vector<double> bnorm;    // ||b_s||
    std::vector<double> target;   // converged when ||b_s - A_s x_s|| <= target[s]
    int max_apply = 1;            // applications of M^{-1}
    int restart = 0;              // columns per cycle (0: max_apply)
};

// Krylov storage: 2m+1 arrays of nsys N complex128, m <= KRYLOV_MAX - 1 and
// within KRYLOV_BUDGET bytes.
constexpr size_t KRYLOV_BUDGET = (size_t)16 << 30;

int ensure_krylov(stfem_handle* h, int nsys, long long N, int want, int& m) {
    const size_t vec = (size_t)nsys * N * 16;
    const size_t fit = KRYLOV_BUDGET / vec >= 3 ? (KRYLOV_BUDGET / vec - 1) / 2 : 1;
    m = (int)std::max<size_t>(1, std::min<size_t>({(size_t)want, (size_t)gpu::KRYLOV_MAX - 1, fit}));
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
    if (nsys > h->kry_nrhs) {
        if (h->kry_partial) (void)hipFree(h->kry_partial);
        if (h->kry_small) (void)hipFree(h->kry_small);
        h->kry_partial = h->kry_small = nullptr;
        h->kry_nrhs = 0;
        if (hipMalloc(&h->kry_partial, gpu::krylov_partial_size(nsys) * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->kry_small, ((size_t)4 * gpu::KRYLOV_MAX + 2) * nsys * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(STFEM_ENOMEM, "Krylov scratch allocation failed");
        }
        h->kry_nrhs = nsys;
    }
    return STFEM_OK;
}

typedef std::complex<double> zd;

// x = (approximately) A^{-1} b.  rbuf: nsys N complex128 of scratch (holds the
// last residual).  applied: applications of M^{-1}; rn[s]: final residual
// norms; hist[k] (k < 16): max_s of the residual estimate / bnorm after k+1
// applications (the recomputed value at the end of a cycle).
int gmres_batched(stfem_handle* h, KrylovSystems& K, const double* b, double* x, double* rbuf, hipStream_t s,
                  int& applied, std::vector<double>& rn, double* hist) {
    const int ns = K.nsys, KM = gpu::KRYLOV_MAX;
    const long long N = K.N, vs = (long long)ns * N;      // complex elements per basis array
    int m = 0;
    int st = ensure_krylov(h, ns, N, K.restart > 0 ? K.restart : K.max_apply, m);
    if (st) return st;
    double* V = h->kry;
    double* Z = h->kry + 2 * (size_t)(m + 1) * vs;
    auto Vp = [&](int i) { return V + 2 * (size_t)i * vs; };
    auto Zp = [&](int i) { return Z + 2 * (size_t)i * vs; };
    double* coef1 = h->kry_small;                          // [ns][<= KM] complex
    double* coef2 = coef1 + 2 * (size_t)KM * ns;
    double* nrm = coef2 + 2 * (size_t)KM * ns;             // [ns]
    double* sc = nrm + ns;                                 // [ns]
    double* part = h->kry_partial;
    StageTimer& T = h->timer;

    std::vector<double> beta(K.bnorm), nh(ns), sh(ns);
    std::vector<double> c1(2 * (size_t)KM * ns), c2(2 * (size_t)KM * ns);
    std::vector<zd> H((size_t)ns * (m + 1) * m), g((size_t)ns * (m + 1)), sn((size_t)ns * m);
    std::vector<double> cs((size_t)ns * m);
    auto Hat = [&](int r, int i, int j) -> zd& { return H[((size_t)r * (m + 1) + i) * m + j]; };
    auto relmax = [&](const std::vector<double>& v) {
        double e = 0;
        for (int r = 0; r < ns; ++r)
            if (K.bnorm[r] > 0) e = std::max(e, std::isfinite(v[r]) ? v[r] / K.bnorm[r] : INFINITY);
        return e;
    };
    std::vector<char> stalled(ns, 0);
    auto done = [&](const std::vector<double>& v, double factor) {
        for (int r = 0; r < ns; ++r)
            if (!stalled[r] && !(v[r] <= factor * K.target[r])) return false;
        return true;
    };
    const double* r0 = b;
    bool first = true;
    applied = 0;
    rn = beta;
    if (done(rn, 1.0)) {        // b within target (b = 0): x = 0
        HIPCHECK(hipMemsetAsync(x, 0, (size_t)vs * 16, s));
        return STFEM_OK;
    }
    for (;;) {
        // V_0 = r0 / beta
        for (int r = 0; r < ns; ++r) sh[r] = beta[r] > 0 && std::isfinite(beta[r]) ? 1.0 / beta[r] : 0.0;
        HIPCHECK(hipMemcpyAsync(sc, sh.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::vec_scale(Vp(0), r0, N, ns, sc, s));
        HIPCHECK(T.end(s, StageTimer::RESID));
        std::fill(H.begin(), H.end(), zd(0));
        std::fill(g.begin(), g.end(), zd(0));
        for (int r = 0; r < ns; ++r) g[(size_t)r * (m + 1)] = beta[r];
        int ncol = 0;
        std::vector<double> est(ns, 0.0);
        while (ncol < m && applied < K.max_apply) {
            const int j = ncol;
            st = K.prec(Vp(j), Zp(j));
            if (st) return st;
            ++applied;
            HIPCHECK(T.begin(s));
            st = K.op(Zp(j), Vp(j + 1));
            if (st) return st;
            HIPCHECK(gpu::vec_mdot(V, vs, j + 1, Vp(j + 1), N, ns, part, coef1, s));
            HIPCHECK(gpu::vec_mcomb(Vp(j + 1), N, ns, V, vs, j + 1, coef1, -1.0, 1, part, nullptr, s));
            HIPCHECK(gpu::vec_mdot(V, vs, j + 1, Vp(j + 1), N, ns, part, coef2, s));
            HIPCHECK(gpu::vec_mcomb(Vp(j + 1), N, ns, V, vs, j + 1, coef2, -1.0, 1, part, nrm, s));
            HIPCHECK(T.end(s, StageTimer::RESID));
            const size_t cb = sizeof(double) * 2 * (size_t)(j + 1) * ns;
            HIPCHECK(hipMemcpyAsync(c1.data(), coef1, cb, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipMemcpyAsync(c2.data(), coef2, cb, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipMemcpyAsync(nh.data(), nrm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            for (int r = 0; r < ns; ++r) {
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
                    const zd a = Hat(r, i, j), bb = Hat(r, i + 1, j);
                    Hat(r, i, j) = c * a + sv * bb;
                    Hat(r, i + 1, j) = -std::conj(sv) * a + c * bb;
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
                est[r] = std::abs(g[(size_t)r * (m + 1) + j + 1]);
            }
            HIPCHECK(hipMemcpyAsync(sc, sh.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
            HIPCHECK(T.begin(s));
            HIPCHECK(gpu::vec_scale(Vp(j + 1), Vp(j + 1), N, ns, sc, s));
            HIPCHECK(T.end(s, StageTimer::RESID));
            if (applied <= 16) hist[applied - 1] = relmax(est);
            ++ncol;
            if (done(est, 0.5)) break;
        }
        // y = R^{-1} g per system, then x (+)= Z y
        for (int r = 0; r < ns; ++r) {
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
        HIPCHECK(hipMemcpyAsync(coef1, c1.data(), sizeof(double) * 2 * (size_t)ncol * ns, hipMemcpyHostToDevice, s));
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::vec_mcomb(x, N, ns, Z, vs, ncol, coef1, 1.0, first ? 0 : 1, part, nullptr, s));
        HIPCHECK(T.end(s, StageTimer::RESID));
        first = false;
        std::vector<double> rr(ns);
        st = K.residual(x, rbuf, rr);
        if (st) return st;
        for (int r = 0; r < ns; ++r) {
            const double v = std::sqrt(rr[r]);
            if (!(v <= 0.5 * beta[r])) stalled[r] = 1;
            rn[r] = beta[r] = v;
        }
        if (applied >= 1 && applied <= 16) hist[applied - 1] = relmax(rn);
        bool finite = true;
        for (double v : rn) finite = finite && std::isfinite(v);
        if (done(rn, 1.0) || applied >= K.max_apply || !finite) break;
        r0 = rbuf;
    }
    return STFEM_OK;
}

// GMRES on the global system K Psi = F (adjoint: K^H) preconditioned by the
// factored FDM inverse, to ||F - K Psi|| <= tol ||F|| for every rhs.
int refine_gmres(stfem_handle* h, const double* F, double* Psi, int nrhs, int adjoint, hipStream_t s, int& applied,
                 double& rel, double* hist) {
    const long long N = (long long)h->n_t * h->n_x;
    int m = 0;
    int st = ensure_krylov(h, nrhs, N, h->opt.restart > 0 ? h->opt.restart : 1 + h->opt.max_iter, m);
    if (st) return st;
    double* nrm = h->kry_small;
    std::vector<double> fn(nrhs);
    HIPCHECK(gpu::vec_norm2(F, N, nrhs, h->kry_partial, nrm, s));
    HIPCHECK(hipMemcpyAsync(fn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    KrylovSystems K;
    K.nsys = nrhs;
    K.N = N;
    K.max_apply = 1 + h->opt.max_iter;
    K.restart = h->opt.restart;
    for (int r = 0; r < nrhs; ++r) {
        K.bnorm.push_back(std::sqrt(fn[r]));
        K.target.push_back(h->opt.tol * std::sqrt(fn[r]));
    }
    K.prec = [&](const double* in, double* out) -> int { return apply_inverse(h, in, out, nrhs, adjoint, 0, s); };
    K.op = [&](const double* in, double* out) -> int {
        HIPCHECK(gpu::kron_apply(in, out, nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev, h->blk->st, adjoint, s));
        return STFEM_OK;
    };
    K.residual = [&](const double* x, double* out, std::vector<double>& rr) -> int {
        HIPCHECK(h->timer.begin(s));
        HIPCHECK(gpu::kron_residual(x, F, out, nrhs, h->n_t, h->w, h->tM_dev, h->tB_dev, h->blk->st, adjoint,
                                    h->partial, h->norms_dev, s));
        HIPCHECK(h->timer.end(s, StageTimer::RESID));
        std::vector<double> nv(2 * (size_t)nrhs);
        HIPCHECK(hipMemcpyAsync(nv.data(), h->norms_dev, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r) rr[r] = nv[2 * r];
        return STFEM_OK;
    };
    std::vector<double> rn;
    st = gmres_batched(h, K, F, Psi, h->R_ws, s, applied, rn, hist);
    if (st) return st;
    rel = 0;
    for (int r = 0; r < nrhs; ++r) {
        const double v = K.bnorm[r] > 0 ? rn[r] / K.bnorm[r] : (rn[r] > 0 ? INFINITY : 0.0);
        rel = std::max(rel, std::isfinite(v) ? v : INFINITY);
    }
    return STFEM_OK;
}


// Spectral norm of the n x n operator y = A v given by `apply` and its adjoint
// `apply_h`: power iteration on A^H A from a fixed start (80 steps), plus 5 %.
template <class F1, class F2>
double spectral_norm(int n, F1 apply, F2 apply_h) {
    std::vector<cplx> v(n), y(n), z(n);
    for (int i = 0; i < n; ++i) v[i] = cplx(1.0 + 0.01 * (i % 7), 0.003 * (i % 5));
    double sigma = 0;
    for (int it = 0; it < 80; ++it) {
        double nv = 0;
        for (auto& c : v) nv += abs2(c);
        nv = std::sqrt(nv);
        if (!(nv > 0)) return 0;
        for (auto& c : v) c = (1.0 / nv) * c;
        apply(v, y);
        apply_h(y, z);
        double nz = 0;
        for (auto& c : z) nz += abs2(c);
        sigma = std::sqrt(std::sqrt(nz));
        v.swap(z);
    }
    return 1.05 * sigma;
}

// Solve with the factors computed chunk by chunk (the factors of all n_t
// blocks exceed the budget), or with resident factors as one chunk when the
// block refinement is chosen.  The transformed rhs G = W F (adjoint: X^H F) is
// formed once; then per chunk of eigen-indices: band fill + LDL^T of its
// blocks, and GMRES on each block system S_l u_l = g_l (adjoint: conj(S_l))
// preconditioned by the chunk's factors, with FP64 block residuals, to
//   ||g_l - S_l u_l|| <= tol ||F|| / (a sqrt(n_t)),  a = ||M_t X||_2
// (adjoint: ||X^{-1}||_2).  Since F - K Psi = (M_t X (x) I)(g - S u) for
// Psi = (X (x) I) u (adjoint: G - K^H Lam = (X^{-H} (x) I)(g - conj(S) u)),
// this bounds the global residual by tol ||F||.  Nearly singular blocks may
// not reach their bound in FP64 (their large solutions cancel in the
// back-transform); the global residual is therefore recomputed, and if it
// is still above tol the solve is repeated on it (at most CHUNK_ROUNDS rounds).
constexpr int CHUNK_ROUNDS = 3;

int solve_chunked(stfem_handle* h, const double* F, double* Psi, int nrhs, int adjoint, hipStream_t s, int& applied,
                  double& rel, double* hist) {
    stfem_blocks* b = h->blk;
    const int nt = h->n_t, nx = h->n_x, cap = b->cap;
    const long long N = (long long)nt * nx;
    const size_t need = (size_t)nrhs * N, cneed = (size_t)nrhs * cap * nx;
    if (need > h->u_elems) {
        cached_free(h->U_ws, h->u_elems * 16);
        h->U_ws = nullptr;
        h->u_elems = 0;
        if (cached_alloc((void**)&h->U_ws, need * 16) != hipSuccess) {
            (void)hipGetLastError();
            h->U_ws = nullptr;
            return fail(STFEM_ENOMEM, "chunked solve: workspace allocation failed");
        }
        h->u_elems = need;
    }
    if (cneed > h->chunk_elems) {
        for (double** p : {&h->Gc, &h->Uc, &h->Rc}) {
            cached_free(*p, h->chunk_elems * 16);
            *p = nullptr;
        }
        h->chunk_elems = 0;
        for (double** p : {&h->Gc, &h->Uc, &h->Rc})
            if (cached_alloc((void**)p, cneed * 16) != hipSuccess) {
                (void)hipGetLastError();
                *p = nullptr;
                return fail(STFEM_ENOMEM, "chunked solve: chunk buffer allocation failed");
            }
        h->chunk_elems = cneed;
    }
    int m = 0;
    int st = ensure_krylov(h, nrhs * cap, nx, h->opt.restart > 0 ? h->opt.restart : 1 + h->opt.max_iter, m);
    if (st) return st;
    StageTimer& T = h->timer;
    double* nrm = h->kry_small;
    std::vector<double> fn(nrhs);
    HIPCHECK(gpu::vec_norm2(F, N, nrhs, h->kry_partial, nrm, s));
    HIPCHECK(hipMemcpyAsync(fn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (double& v : fn) v = std::sqrt(v);
    const double amp = adjoint ? h->amp_adj : h->amp_fwd;
    const double* first = adjoint ? h->X_dev : h->W_dev;
    const double* second = adjoint ? h->W_dev : h->X_dev;
    const double tol = h->opt.tol;
    double ms_fill = 0, ms_ldlt = 0;
    applied = 0;
    rel = INFINITY;
    const double* rhs = F;
    for (int round = 0; round < CHUNK_ROUNDS; ++round) {
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::zgemm_small_left(nt, nx, nrhs, first, adjoint, rhs, N, h->G_ws, N, 0, s));
        HIPCHECK(T.end(s, StageTimer::GEMM));
        int round_apply = 0;
        for (int c = 0; c < h->nchunks; ++c) {
            // odd rounds walk the chunks backwards and start with the one
            // whose factors are still in place
            const int l0 = (round % 2 == 0 ? c : h->nchunks - 1 - c) * cap;
            const int cnt = std::min(cap, nt - l0), ns = nrhs * cnt;
            if (!(b->l0 == l0 && b->nf == cnt && b->factored)) {
                st = blocks_factor(b, l0, cnt, s);
                if (st) return st;
                st = blocks_finish(b, s);
                if (st) return st;
                b->factored = true;
                ms_fill += b->ms_fill;
                ms_ldlt += b->ms_ldlt;
            }
            const size_t row = (size_t)cnt * nx * 16;
            HIPCHECK(hipMemcpy2DAsync(h->Gc, row, h->G_ws + 2 * (size_t)l0 * nx, (size_t)N * 16, row, nrhs,
                                      hipMemcpyDeviceToDevice, s));
            auto prec = [&](const double* in, double* out) -> int {
                HIPCHECK(T.begin(s));
                HIPCHECK(gpu::sweep_solve(b->precision, b->band, cnt, b->st, in, out, nrhs, adjoint, s));
                HIPCHECK(T.end(s, StageTimer::SWEEP));
                return STFEM_OK;
            };
            if (tol > 0) {
                KrylovSystems K;
                K.nsys = ns;
                K.N = nx;
                K.max_apply = 1 + h->opt.max_iter;
                K.restart = h->opt.restart;
                std::vector<double> gn(ns);
                HIPCHECK(gpu::vec_norm2(h->Gc, nx, ns, h->kry_partial, nrm, s));
                HIPCHECK(hipMemcpyAsync(gn.data(), nrm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                for (int q = 0; q < ns; ++q) {
                    K.bnorm.push_back(std::sqrt(gn[q]));
                    K.target.push_back(tol * fn[q / cnt] / (amp * std::sqrt((double)nt)));
                }
                K.prec = prec;
                K.op = [&](const double* in, double* out) -> int {
                    HIPCHECK(gpu::shifted_apply(b->st, b->lambda_dev, l0, cnt, adjoint, in, out, nullptr, ns, s));
                    return STFEM_OK;
                };
                K.residual = [&](const double* x, double* out, std::vector<double>& rr) -> int {
                    HIPCHECK(T.begin(s));
                    HIPCHECK(gpu::shifted_apply(b->st, b->lambda_dev, l0, cnt, adjoint, x, out, h->Gc, ns, s));
                    HIPCHECK(gpu::vec_norm2(out, nx, ns, h->kry_partial, nrm, s));
                    HIPCHECK(T.end(s, StageTimer::RESID));
                    HIPCHECK(hipMemcpyAsync(rr.data(), nrm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
                    HIPCHECK(hipStreamSynchronize(s));
                    return STFEM_OK;
                };
                int a = 0;
                std::vector<double> rn;
                double hloc[16];
                st = gmres_batched(h, K, h->Gc, h->Uc, h->Rc, s, a, rn, hloc);
                if (st) return st;
                round_apply = std::max(round_apply, a);
            } else {
                st = prec(h->Gc, h->Uc);
                if (st) return st;
                round_apply = 1;
            }
            HIPCHECK(hipMemcpy2DAsync(h->U_ws + 2 * (size_t)l0 * nx, (size_t)N * 16, h->Uc, row, row, nrhs,
                                      hipMemcpyDeviceToDevice, s));
        }
        applied += round_apply;
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::zgemm_small_left(nt, nx, nrhs, second, adjoint, h->U_ws, N, Psi, N, round > 0, s));
        HIPCHECK(T.end(s, StageTimer::GEMM));
        if (!(tol > 0)) break;
        HIPCHECK(T.begin(s));
        HIPCHECK(gpu::kron_residual(Psi, F, h->R_ws, nrhs, nt, h->w, h->tM_dev, h->tB_dev, b->st, adjoint, h->partial,
                                    h->norms_dev, s));
        HIPCHECK(T.end(s, StageTimer::RESID));
        st = read_relres(h, nrhs, s, rel);
        if (st) return st;
        if (round < 16) hist[round] = rel;
        if (rel <= tol || !std::isfinite(rel)) break;
        rhs = h->R_ws;
    }
    if (h->nchunks > 1) {   // resident factors keep their factorisation times
        b->ms_fill = ms_fill;
        b->ms_ldlt = ms_ldlt;
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
    if (h->nchunks > 1 || (h->opt.tol > 0 && h->opt.refine == STFEM_REFINE_BLOCK)) {
        int applied = 0;
        st = solve_chunked(h, F, Psi, nrhs, adjoint, s, applied, rel, hist);
        if (st) return st;
        it = applied - 1;
    } else if (h->opt.tol > 0 && h->opt.refine == STFEM_REFINE_GMRES) {
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
        rep->chunks = h->nchunks;
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
    HIPCHECK(gpu::sweep_solve(b->precision, b->band, b->nf, b->st, (const double*)G_dev, (double*)U_dev, nrhs,
                              conj ? 1 : 0, (hipStream_t)stream));
    return STFEM_OK;
}

extern "C" int shifted_factor_band(const stfem_blocks* b, int l, double* band) {
    clear_error();
    if (!b || !band || l < 0 || l >= b->nf) return fail(STFEM_EINVAL, "shifted_factor_band: bad argument");
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
    stfem_options o{64, 0, 0.0, STFEM_REFINE_GMRES, 0, 0.0};
    if (opt) o = *opt;
    if (o.precision != 32 && o.precision != 64) return fail(STFEM_EINVAL, "fdm_factor: precision must be 32 or 64");
    if (o.max_iter < 0) return fail(STFEM_EINVAL, "fdm_factor: max_iter must be >= 0");
    if (o.refine != STFEM_REFINE_GMRES && o.refine != STFEM_REFINE_PLAIN && o.refine != STFEM_REFINE_BLOCK)
        return fail(STFEM_EINVAL, "fdm_factor: refine must be STFEM_REFINE_GMRES, _PLAIN or _BLOCK");
    if (o.restart < 0) return fail(STFEM_EINVAL, "fdm_factor: restart must be >= 0");
    if (!(o.factor_budget >= 0)) return fail(STFEM_EINVAL, "fdm_factor: factor_budget must be >= 0");
    if (n < 2 || n > 1024) return fail(STFEM_EINVAL, "fdm_factor: need 2 <= n <= 1024");
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
    // factor storage for all n_t blocks if it fits the budget, else chunks of
    // eigen-indices that are factored again in every solve
    const size_t per_block = (size_t)gpu::band_stride_host(n) * elem_bytes(o.precision);
    size_t budget = (size_t)o.factor_budget;
    if (!(o.factor_budget > 0)) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        free_b += cached_bytes();
        const size_t reserve = (size_t)6 * n_t * h->n_x * 16 + KRYLOV_BUDGET + ((size_t)4 << 30);
        budget = free_b > reserve ? free_b - reserve : 0;
    }
    int cap = n_t;
    if ((size_t)n_t * per_block > budget) {
        cap = (int)std::min<size_t>(n_t, budget / per_block);
        if (cap < 1) {
            delete h;
            return fail(STFEM_ENOMEM, "fdm_factor: the factor budget holds less than one spatial block");
        }
        h->nchunks = (n_t + cap - 1) / cap;
        cap = (n_t + h->nchunks - 1) / h->nchunks;
    }
    if (h->nchunks > 1) {
        st = blocks_create(n, M_stencil, A_stencil, lam.data(), n_t, cap, o.precision, s, &h->blk);
    } else {
        st = blocks_launch(n, M_stencil, A_stencil, lam.data(), n_t, o.precision, s, &h->blk);
    }
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
    if (h->nchunks > 1 || o.refine == STFEM_REFINE_BLOCK) {
        // ||M_t X||_2 and ||X^{-1}||_2 = ||W M_t||_2 for the block tolerances
        const std::vector<cplx>& X = h->dec.X;
        const std::vector<cplx>& W = h->dec.W;
        auto mt = [&](const std::vector<cplx>& v, std::vector<cplx>& y) {   // y = M_t v (M_t symmetric)
            for (int i = 0; i < n_t; ++i) {
                cplx a;
                for (int j = std::max(0, i - h->w); j <= std::min(n_t - 1, i + h->w); ++j)
                    a += M_t[(size_t)i * n_t + j] * v[j];
                y[i] = a;
            }
        };
        auto mul = [&](const std::vector<cplx>& A, bool herm, const std::vector<cplx>& v, std::vector<cplx>& y) {
            for (int i = 0; i < n_t; ++i) {
                cplx a;
                for (int j = 0; j < n_t; ++j)
                    a += (herm ? conj(A[(size_t)j * n_t + i]) : A[(size_t)i * n_t + j]) * v[j];
                y[i] = a;
            }
        };
        std::vector<cplx> tmp(n_t);
        h->amp_fwd = spectral_norm(
            n_t, [&](const std::vector<cplx>& v, std::vector<cplx>& y) { mul(X, false, v, tmp); mt(tmp, y); },
            [&](const std::vector<cplx>& v, std::vector<cplx>& y) { mt(v, tmp); mul(X, true, tmp, y); });
        h->amp_adj = spectral_norm(
            n_t, [&](const std::vector<cplx>& v, std::vector<cplx>& y) { mt(v, tmp); mul(W, false, tmp, y); },
            [&](const std::vector<cplx>& v, std::vector<cplx>& y) { mul(W, true, v, tmp); mt(tmp, y); });
        HIPCHECK(hipStreamSynchronize(s));
    }
    if (h->nchunks == 1) {
        st = blocks_finish(h->blk, s);
        if (st) return cleanup(st);
        h->blk->factored = true;
    }
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
    cached_free(h->U_ws, h->u_elems * 16);
    for (double* q : {h->Gc, h->Uc, h->Rc}) cached_free(q, h->chunk_elems * 16);
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
