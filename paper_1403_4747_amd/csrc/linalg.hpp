// Host-side dense complex linear algebra used while building a plan:
// column-major matrices, products and a thread pool loop.  (The SVDs of the
// equivalent-to-check maps run on the GPU, in rocSOLVER.)
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <functional>
#include <thread>
#include <vector>

namespace fda {

using cplx = std::complex<double>;

struct Mat {
    int m = 0, n = 0;
    std::vector<cplx> a;  // column-major, a[i + j*m]
    Mat() = default;
    Mat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_) {}
    cplx &operator()(int i, int j) { return a[(size_t)i + (size_t)j * m]; }
    const cplx &operator()(int i, int j) const { return a[(size_t)i + (size_t)j * m]; }
    cplx *col(int j) { return a.data() + (size_t)j * m; }
    const cplx *col(int j) const { return a.data() + (size_t)j * m; }
};

// C = op(A) * op(B), op = 'N' (none) or 'C' (conjugate transpose).
inline Mat matmul(const Mat &A, char ta, const Mat &B, char tb) {
    const int m = (ta == 'N') ? A.m : A.n;
    const int kk = (ta == 'N') ? A.n : A.m;
    const int n = (tb == 'N') ? B.n : B.m;
    Mat C(m, n);
    if (ta == 'N' && tb == 'N') {
        for (int j = 0; j < n; ++j) {
            cplx *c = C.col(j);
            for (int p = 0; p < kk; ++p) {
                const cplx b = B(p, j);
                if (b == cplx(0)) continue;
                const cplx *a = A.col(p);
                for (int i = 0; i < m; ++i) c[i] += a[i] * b;
            }
        }
    } else if (ta == 'C' && tb == 'N') {
        for (int j = 0; j < n; ++j) {
            const cplx *b = B.col(j);
            for (int i = 0; i < m; ++i) {
                const cplx *a = A.col(i);
                cplx s = 0;
                for (int p = 0; p < kk; ++p) s += std::conj(a[p]) * b[p];
                C(i, j) = s;
            }
        }
    } else if (ta == 'N' && tb == 'C') {
        for (int j = 0; j < n; ++j) {
            cplx *c = C.col(j);
            for (int p = 0; p < kk; ++p) {
                const cplx b = std::conj(B(j, p));
                const cplx *a = A.col(p);
                for (int i = 0; i < m; ++i) c[i] += a[i] * b;
            }
        }
    } else {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                cplx s = 0;
                for (int p = 0; p < kk; ++p) s += std::conj(A(p, i)) * std::conj(B(j, p));
                C(i, j) = s;
            }
    }
    return C;
}

// Run f(i) for i in [0, n) on up to `threads` host threads.
inline void parallel_for(int64_t n, const std::function<void(int64_t)> &f, int threads = 0) {
    if (threads <= 0) {
        threads = (int)std::thread::hardware_concurrency();
        if (threads <= 0) threads = 4;
        threads = std::min(threads, 32);
    }
    if (n <= 1 || threads == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> pool;
    std::atomic<int64_t> next(0);
    for (int t = 0; t < threads && t < n; ++t)
        pool.emplace_back([&]() {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                f(i);
            }
        });
    for (auto &th : pool) th.join();
}

}  // namespace fda
