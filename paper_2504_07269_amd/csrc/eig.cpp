// Host FP64 temporal eigen-decomposition for fast diagonalization (Sec. 3,
// solver step 1 with the eigenvalue decomposition as the choice of X_t, S_t).
//
// The library diagonalises M^{-1} (i B) = X diag(lambda) X^{-1}; the paper's
// (i B_t)^{-1} M_t = X_t S_t X_t^{-1} has the same eigenvectors and
// S_t = diag(1/lambda).  Both temporal matrices are banded (bandwidth p), so
// everything here costs O(n^2) instead of the O(n^3) of a dense
// Hessenberg-QR:
//
//  1. eigenvalues: simultaneous Newton iteration with Aberth's correction
//     (Ehrlich-Aberth) on det(i B - z M) = 0.  The Newton quotient uses
//     d/dz log det(i B - z M), obtained from a banded LU with partial
//     pivoting that carries first derivatives (forward-mode) of its entries;
//  2. right eigenvectors x_l and left eigenvectors y_l (y_l^T (iB - lambda_l M) = 0)
//     by two steps of inverse iteration with the banded LU, then the two-sided
//     Rayleigh quotient lambda_l = y_l^T iB x_l / y_l^T M x_l;
//  3. W = (M X)^{-1} = diag(1 / y_l^T M x_l) Y^T, because left and right
//     eigenvectors of a diagonalisable pencil are M-biorthogonal.
// Eigenvalues are sorted by real part (then imaginary part) so that the
// block order is reproducible.
#include <algorithm>
#include <cstdio>
#include <atomic>
#include <numeric>

#include "common.h"

namespace stfem {
namespace {

// Banded n x n complex matrix with half-bandwidth w: a[i*(2w+1) + (j-i+w)].
struct Band {
    int n = 0, w = 0;
    std::vector<double> m, b;   // real M and B in band storage
    double M(int i, int j) const { return m[(size_t)i * (2 * w + 1) + (j - i + w)]; }
    double B(int i, int j) const { return b[(size_t)i * (2 * w + 1) + (j - i + w)]; }
};

// LU with partial pivoting of T = i B - z M (or its derivative-carrying
// variant).  Row i keeps the columns [i-w, i+2w]; after step k row k holds U's
// row k in columns [k, k+2w]; mult[k*w + r] is the multiplier of row k+1+r.
struct BandPLU {
    int n = 0, w = 0, ww = 0;
    std::vector<cplx> u, mult;
    std::vector<int> piv;
    bool singular = false;

    cplx& at(int i, int j) { return u[(size_t)i * ww + (j - i + w)]; }

    void factor(const Band& P, cplx z) {
        n = P.n; w = P.w; ww = 3 * w + 1;
        u.assign((size_t)n * ww, cplx());
        mult.assign((size_t)n * std::max(w, 1), cplx());
        piv.assign(n, 0);
        singular = false;
        for (int i = 0; i < n; ++i)
            for (int j = std::max(0, i - w); j <= std::min(n - 1, i + w); ++j)
                at(i, j) = cplx(0.0, P.B(i, j)) - z * P.M(i, j);
        for (int k = 0; k < n; ++k) {
            const int last = std::min(n - 1, k + w), jmax = std::min(n - 1, k + 2 * w);
            int p = k;
            double best = abs2(at(k, k));
            for (int r = k + 1; r <= last; ++r) {
                double v = abs2(at(r, k));
                if (v > best) { best = v; p = r; }
            }
            piv[k] = p;
            if (p != k)
                for (int j = k; j <= jmax; ++j) std::swap(at(k, j), at(p, j));
            cplx d = at(k, k);
            if (best == 0.0) { singular = true; d = cplx(1e-300, 0.0); at(k, k) = d; }
            for (int r = k + 1; r <= last; ++r) {
                cplx l = at(r, k) / d;
                mult[(size_t)k * w + (r - k - 1)] = l;
                at(r, k) = cplx();
                for (int j = k + 1; j <= jmax; ++j) at(r, j) -= l * at(k, j);
            }
        }
    }
    // x <- T^{-1} x
    void solve(std::vector<cplx>& x) {
        for (int k = 0; k < n; ++k) {
            if (piv[k] != k) std::swap(x[k], x[piv[k]]);
            const int last = std::min(n - 1, k + w);
            for (int r = k + 1; r <= last; ++r) x[r] -= mult[(size_t)k * w + (r - k - 1)] * x[k];
        }
        for (int k = n - 1; k >= 0; --k) {
            cplx s = x[k];
            const int jmax = std::min(n - 1, k + 2 * w);
            for (int j = k + 1; j <= jmax; ++j) s -= at(k, j) * x[j];
            x[k] = s / at(k, k);
        }
    }
    // x <- T^{-T} x  (plain transpose, no conjugation)
    void solve_transpose(std::vector<cplx>& x) {
        for (int k = 0; k < n; ++k) {           // U^T is lower triangular
            cplx s = x[k];
            for (int i = std::max(0, k - 2 * w); i < k; ++i) s -= at(i, k) * x[i];
            x[k] = s / at(k, k);
        }
        for (int k = n - 1; k >= 0; --k) {
            const int last = std::min(n - 1, k + w);
            cplx s = x[k];
            for (int r = k + 1; r <= last; ++r) s -= mult[(size_t)k * w + (r - k - 1)] * x[r];
            x[k] = s;
            if (piv[k] != k) std::swap(x[k], x[piv[k]]);
        }
    }
};

// d/dz log det(i B - z M) by banded LU with partial pivoting on dual numbers
// (value, d/dz); the derivative of every entry of i B - z M is -M.
// Returns false if an exact zero pivot occurs.
bool logdet_derivative(const Band& P, cplx z, std::vector<cplx>& va, std::vector<cplx>& da, cplx& out) {
    const int n = P.n, w = P.w, ww = 3 * w + 1;
    va.assign((size_t)n * ww, cplx());
    da.assign((size_t)n * ww, cplx());
    auto idx = [&](int i, int j) { return (size_t)i * ww + (j - i + w); };
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - w); j <= std::min(n - 1, i + w); ++j) {
            va[idx(i, j)] = cplx(0.0, P.B(i, j)) - z * P.M(i, j);
            da[idx(i, j)] = cplx(-P.M(i, j), 0.0);
        }
    cplx s;
    for (int k = 0; k < n; ++k) {
        const int last = std::min(n - 1, k + w), jmax = std::min(n - 1, k + 2 * w);
        int p = k;
        double best = abs2(va[idx(k, k)]);
        for (int r = k + 1; r <= last; ++r) {
            double v = abs2(va[idx(r, k)]);
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) return false;
        if (p != k)
            for (int j = k; j <= jmax; ++j) {
                std::swap(va[idx(k, j)], va[idx(p, j)]);
                std::swap(da[idx(k, j)], da[idx(p, j)]);
            }
        const cplx dv = va[idx(k, k)], dd = da[idx(k, k)];
        const cplx inv = conj(dv) * (1.0 / best);          // 1 / dv
        const cplx q = dd * inv;
        s += q;
        for (int r = k + 1; r <= last; ++r) {
            const cplx l = va[idx(r, k)] * inv;
            const cplx ld = (da[idx(r, k)] - l * dd) * inv;
            for (int j = k + 1; j <= jmax; ++j) {
                const cplx kv = va[idx(k, j)], kdv = da[idx(k, j)];
                va[idx(r, j)] -= l * kv;
                da[idx(r, j)] -= ld * kv + l * kdv;
            }
        }
    }
    out = s;
    return true;
}

// A fixed team of host threads that repeatedly runs body(thread, nthreads)
// separated by barriers; used for the Jacobi-style Aberth sweeps so that the
// threads are created once per decomposition rather than once per sweep.
class SpinBarrier {
  public:
    explicit SpinBarrier(int n) : n_(n), count_(0), gen_(0) {}
    void wait() {
        const int g = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_acq_rel);
            return;
        }
        int spins = 0;
        while (gen_.load(std::memory_order_acquire) == g)
            if (++spins > 256) std::this_thread::yield();
    }
  private:
    int n_;
    std::atomic<int> count_, gen_;
};

// Deterministic start vector for inverse iteration.
void start_vector(std::vector<cplx>& x, int seed) {
    for (size_t k = 0; k < x.size(); ++k) {
        double a = 0.7548776662 * (double)(k + 1) + 0.5698402910 * (double)(seed + 1);
        a -= std::floor(a);
        x[k] = cplx(std::cos(6.283185307179586 * a), std::sin(6.283185307179586 * a * 1.6180339887));
    }
}

double norm2(const std::vector<cplx>& x) {
    double s = 0;
    for (auto& v : x) s += abs2(v);
    return std::sqrt(s);
}

void dense_matvec(const std::vector<cplx>& A, int n, const std::vector<cplx>& v, std::vector<cplx>& r, bool herm) {
    for (int i = 0; i < n; ++i) {
        cplx s;
        if (!herm)
            for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * v[k];
        else
            for (int k = 0; k < n; ++k) s += conj(A[(size_t)k * n + i]) * v[k];
        r[i] = s;
    }
}

void band_M(const Band& P, const std::vector<cplx>& v, std::vector<cplx>& r, bool transpose) {
    const int n = P.n, w = P.w;
    for (int i = 0; i < n; ++i) {
        cplx s;
        for (int k = std::max(0, i - w); k <= std::min(n - 1, i + w); ++k)
            s += (transpose ? P.M(k, i) : P.M(i, k)) * v[k];
        r[i] = s;
    }
}

}  // namespace

int temporal_decompose(const double* Md, const double* Bd, int n, TemporalDecomp& out) {
    if (n < 1) return fail(STFEM_EINVAL, "temporal_decompose: n < 1");
    // bandwidth of the pencil
    int w = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (Md[(size_t)i * n + j] != 0.0 || Bd[(size_t)i * n + j] != 0.0) w = std::max(w, std::abs(i - j));
    if (w > 4) return fail(STFEM_EINVAL, "fdm_factor: temporal matrices must be banded with bandwidth <= 4");
    w = std::max(w, 1);
    Band P;
    P.n = n; P.w = w;
    P.m.assign((size_t)n * (2 * w + 1), 0.0);
    P.b.assign((size_t)n * (2 * w + 1), 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - w); j <= std::min(n - 1, i + w); ++j) {
            P.m[(size_t)i * (2 * w + 1) + (j - i + w)] = Md[(size_t)i * n + j];
            P.b[(size_t)i * (2 * w + 1) + (j - i + w)] = Bd[(size_t)i * n + j];
        }

    // ---- spectral radius estimate by power iteration on M^{-1} (i B)
    double R = 0;
    {
        BandPLU Mlu;
        Band Mneg = P;                      // factor  i*0 - (-1) M = M
        std::fill(Mneg.b.begin(), Mneg.b.end(), 0.0);
        Mlu.factor(Mneg, cplx(-1.0, 0.0));
        if (Mlu.singular) return fail(STFEM_ENOTDIAG, "fdm_factor: temporal mass matrix is singular");
        std::vector<cplx> v(n), t(n);
        start_vector(v, 7);
        double nv = norm2(v);
        for (auto& e : v) e = e * (1.0 / nv);
        for (int it = 0; it < 60; ++it) {
            for (int i = 0; i < n; ++i) {
                cplx s;
                for (int j = std::max(0, i - w); j <= std::min(n - 1, i + w); ++j) s += cplx(0.0, P.B(i, j)) * v[j];
                t[i] = s;
            }
            Mlu.solve(t);
            double nt = norm2(t);
            if (!(nt > 0) || !std::isfinite(nt)) break;
            R = std::max(R, nt);
            for (int i = 0; i < n; ++i) v[i] = t[i] * (1.0 / nt);
        }
        if (!(R > 0)) return fail(STFEM_ENOTDIAG, "fdm_factor: could not estimate the temporal spectrum");
    }

    // ---- Ehrlich-Aberth iteration: Jacobi sweeps (every root updated from
    //      the previous sweep's roots, so the result does not depend on the
    //      number of threads), split over a fixed team of host threads.
    std::vector<cplx> zbuf0(n), zbuf1(n);
    const double pi = 3.141592653589793;
    for (int j = 0; j < n; ++j) {
        const double th = pi * (j + 0.5) / n;
        zbuf0[j] = cplx(1.05 * R * std::cos(th), 0.05 * R * std::sin(th));
    }
    std::vector<char> conv(n, 0);
    const double tol = 1e-12;
    const int maxit = 800;
    unsigned hc = std::thread::hardware_concurrency();
    const int team = std::max(1, std::min<int>({(int)(hc ? hc : 1), 16, n / 16 + 1}));
    SpinBarrier barrier(team);
    std::atomic<int> done(0), iters(0);
    auto worker = [&](int t) {
        const int lo = (int)((long long)n * t / team), hi = (int)((long long)n * (t + 1) / team);
        std::vector<cplx> va, da;
        for (int it = 0; it < maxit; ++it) {
            const std::vector<cplx>& z = (it & 1) ? zbuf1 : zbuf0;
            std::vector<cplx>& zn = (it & 1) ? zbuf0 : zbuf1;
            for (int j = lo; j < hi; ++j) {
                const cplx zj = z[j];
                zn[j] = zj;
                if (conv[j]) continue;
                cplx dlog;
                if (!logdet_derivative(P, zj, va, da, dlog)) {   // exact pole: nudge
                    zn[j] = zj + cplx(1e-10 * R, 1e-10 * R);
                    continue;
                }
                // Newton quotient N = det/det' = 1/dlog; Aberth step
                // N / (1 - N sum_k 1/(z_j - z_k))
                const cplx N = conj(dlog) * (1.0 / abs2(dlog));
                cplx S;
                for (int k = 0; k < n; ++k) {
                    if (k == j) continue;
                    const cplx d = zj - z[k];
                    S += conj(d) * (1.0 / abs2(d));
                }
                cplx step = N / (cplx(1.0, 0.0) - N * S);
                if (!finite(step)) step = N;
                zn[j] = zj - step;
                if (cabs(step) <= tol * cabs(zj)) conv[j] = 1;
            }
            barrier.wait();
            if (t == 0) {
                bool all = true;
                for (int j = 0; j < n && all; ++j) all = conv[j];
                iters.store(it + 1);
                if (all) done.store(1);
            }
            barrier.wait();
            if (done.load()) break;
        }
    };
    {
        std::vector<std::thread> pool;
        for (int t = 1; t < team; ++t) pool.emplace_back(worker, t);
        worker(0);
        for (auto& th : pool) th.join();
    }
    const int it = iters.load();
    std::vector<cplx>& z = (it & 1) ? zbuf1 : zbuf0;
    for (int j = 0; j < n; ++j)
        if (!finite(z[j])) return fail(STFEM_ENOTDIAG, "fdm_factor: eigenvalue iteration diverged");
    if (!done.load()) {
        int nc = 0;
        for (int j = 0; j < n; ++j) nc += !conv[j];
        // Roots that stagnate at rounding level are polished below; refuse
        // only if the iteration clearly did not settle.
        if (nc > n / 4) return fail(STFEM_ENOTDIAG, "fdm_factor: eigenvalue iteration did not converge");
    }
    out.aberth_iters = it;

    // ---- eigenvectors by inverse iteration, two-sided Rayleigh quotient
    std::vector<cplx> X((size_t)n * n), Y((size_t)n * n), lam(n), ymx(n);
    std::vector<int> bad(n, 0);
    parallel_for(n, [&](int j) {
        BandPLU lu;
        cplx zj = z[j];
        lu.factor(P, zj);
        if (lu.singular) {
            zj = zj * cplx(1.0 + 1e-14, 1e-14);
            lu.factor(P, zj);
        }
        std::vector<cplx> x(n), y(n), mx(n), mty(n);
        start_vector(x, 2 * j);
        start_vector(y, 2 * j + 1);
        for (int s = 0; s < 2; ++s) {
            // x <- T^{-1} M x ;  y <- T^{-T} M^T y
            for (int i = 0; i < n; ++i) {
                cplx a, b;
                for (int k = std::max(0, i - w); k <= std::min(n - 1, i + w); ++k) {
                    a += P.M(i, k) * x[k];
                    b += P.M(k, i) * y[k];
                }
                mx[i] = a;
                mty[i] = b;
            }
            lu.solve(mx);
            lu.solve_transpose(mty);
            x.swap(mx);
            y.swap(mty);
            double nx = norm2(x), ny = norm2(y);
            if (!(nx > 0) || !(ny > 0) || !std::isfinite(nx) || !std::isfinite(ny)) { bad[j] = 1; return; }
            for (int i = 0; i < n; ++i) { x[i] = x[i] * (1.0 / nx); y[i] = y[i] * (1.0 / ny); }
        }
        cplx num, den;
        for (int i = 0; i < n; ++i) {
            cplx bx, mx;
            for (int k = std::max(0, i - w); k <= std::min(n - 1, i + w); ++k) {
                bx += cplx(0.0, P.B(i, k)) * x[k];
                mx += P.M(i, k) * x[k];
            }
            num += y[i] * bx;
            den += y[i] * mx;
        }
        if (cabs(den) == 0.0) { bad[j] = 1; return; }
        lam[j] = num / den;
        ymx[j] = den;
        for (int i = 0; i < n; ++i) {
            X[(size_t)i * n + j] = x[i];
            Y[(size_t)i * n + j] = y[i];
        }
    });
    for (int j = 0; j < n; ++j)
        if (bad[j] || !finite(lam[j]))
            return fail(STFEM_ENOTDIAG, "fdm_factor: inverse iteration failed (pencil not diagonalisable?)");

    // ---- order by real part, then imaginary part
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (lam[a].re != lam[b].re) return lam[a].re < lam[b].re;
        return lam[a].im < lam[b].im;
    });
    out.n = n;
    out.lambda.resize(n);
    out.X.assign((size_t)n * n, cplx());
    out.W.assign((size_t)n * n, cplx());
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        out.lambda[jj] = lam[j];
        const cplx sc = cplx(1.0, 0.0) / ymx[j];
        for (int i = 0; i < n; ++i) {
            out.X[(size_t)i * n + jj] = X[(size_t)i * n + j];
            out.W[(size_t)jj * n + i] = sc * Y[(size_t)i * n + j];
        }
    }

    // ---- check W M X = I on a probe vector (O(n^2))
    std::vector<cplx> v(n), t1(n), t2(n);
    start_vector(v, 12345);
    dense_matvec(out.X, n, v, t1, false);
    band_M(P, t1, t2, false);
    dense_matvec(out.W, n, t2, t1, false);
    double err = 0;
    for (int i = 0; i < n; ++i) err += abs2(t1[i] - v[i]);
    if (!(std::sqrt(err) <= 1e-6 * norm2(v)))
        return fail(STFEM_ENOTDIAG, "fdm_factor: W M X != I (eigenvectors nearly dependent)");
    out.band_w = w;
    out.Mband = P.m;
    return STFEM_OK;
}

// kappa_2(X) estimate: sqrt of the largest eigenvalue of X^H X times that of
// (W M)^H (W M), each by power iteration (X^{-1} = W M).
double temporal_kappa(const TemporalDecomp& d, int iters) {
    const int n = d.n;
    Band P;
    P.n = n; P.w = d.band_w; P.m = d.Mband;
    std::vector<cplx> v(n), t1(n), t2(n);
    auto power = [&](bool inverse) {
        start_vector(v, inverse ? 99 : 98);
        double sig = 0;
        for (int s = 0; s < iters; ++s) {
            double nv = norm2(v);
            for (auto& e : v) e = e * (1.0 / nv);
            if (!inverse) {
                dense_matvec(d.X, n, v, t1, false);
                dense_matvec(d.X, n, t1, v, true);
            } else {
                band_M(P, v, t1, false);
                dense_matvec(d.W, n, t1, t2, false);
                dense_matvec(d.W, n, t2, t1, true);
                band_M(P, t1, v, true);
            }
            sig = std::sqrt(norm2(v));
        }
        return sig;
    };
    return power(false) * power(true);
}

}  // namespace stfem
