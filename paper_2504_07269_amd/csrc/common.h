// Shared host-side helpers of the stfem library: a small complex type, status
// and error-message plumbing, wall-clock timing and a parallel-for.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stfem.h"

namespace stfem {

// Plain complex double with inline arithmetic (no inf/nan recovery path).
struct cplx {
    double re, im;
    cplx() : re(0), im(0) {}
    cplx(double r, double i = 0.0) : re(r), im(i) {}
};
inline cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
inline cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
inline cplx operator-(cplx a) { return {-a.re, -a.im}; }
inline cplx operator*(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
inline cplx operator*(cplx a, double s) { return {s * a.re, s * a.im}; }
inline cplx conj(cplx a) { return {a.re, -a.im}; }
inline double abs2(cplx a) { return a.re * a.re + a.im * a.im; }
inline double cabs(cplx a) { return std::hypot(a.re, a.im); }
inline cplx operator/(cplx a, cplx b) {
    // Smith's algorithm
    if (std::fabs(b.re) >= std::fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
inline cplx& operator+=(cplx& a, cplx b) { a.re += b.re; a.im += b.im; return a; }
inline cplx& operator-=(cplx& a, cplx b) { a.re -= b.re; a.im -= b.im; return a; }
inline bool finite(cplx a) { return std::isfinite(a.re) && std::isfinite(a.im); }

// Thread-local message of the last failure; returns the status for chaining.
int fail(int status, const std::string& msg);
void clear_error();

inline double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Run body(i) for i in [0, n) on up to `threads` host threads (static blocks).
template <class F>
void parallel_for(int n, F body, int threads = 0) {
    if (threads <= 0) {
        unsigned hc = std::thread::hardware_concurrency();
        threads = (int)std::min<unsigned>(hc ? hc : 1, 16u);
    }
    threads = std::max(1, std::min(threads, n));
    if (threads == 1) {
        for (int i = 0; i < n; ++i) body(i);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(threads);
    for (int t = 0; t < threads; ++t) {
        pool.emplace_back([=, &body]() {
            int lo = (int)((long long)n * t / threads), hi = (int)((long long)n * (t + 1) / threads);
            for (int i = lo; i < hi; ++i) body(i);
        });
    }
    for (auto& th : pool) th.join();
}

// Temporal eigen-decomposition M^{-1} (i B) = X diag(lambda) X^{-1} with
// W = (M X)^{-1}; all arrays row-major n x n (X, W) or length n (lambda).
struct TemporalDecomp {
    int n = 0;
    std::vector<cplx> lambda, X, W;
    double kappa = 0.0;       // estimate of ||X||_2 ||X^{-1}||_2 (temporal_kappa)
    int aberth_iters = 0;
    int band_w = 0;           // temporal bandwidth
    std::vector<double> Mband;   // M in band storage, kept for temporal_kappa
};

int temporal_decompose(const double* M, const double* B, int n, TemporalDecomp& out);
double temporal_kappa(const TemporalDecomp& d, int iters = 25);

}  // namespace stfem
