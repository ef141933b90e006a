// Host-side dense complex linear algebra used while building a plan:
// column-major matrices, products, Householder QR and a one-sided Jacobi
// SVD.  The SVDs factor the equivalent-to-check maps G_up and G_dn and their
// truncation follows eqs. (eq_svdg), (eq_epsg), (eq_invg).
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

// Householder QR of a tall matrix A (m >= n): returns Q (m x n, orthonormal
// columns) and R (n x n, upper triangular) with A = Q R.
inline void qr_thin(const Mat &A, Mat &Q, Mat &R) {
    const int m = A.m, n = A.n;
    Mat W = A;
    std::vector<std::vector<cplx>> vs(n);
    std::vector<cplx> betas(n);
    for (int j = 0; j < n; ++j) {
        double nrm = 0;
        for (int i = j; i < m; ++i) nrm += std::norm(W(i, j));
        nrm = std::sqrt(nrm);
        std::vector<cplx> v(m - j);
        for (int i = j; i < m; ++i) v[i - j] = W(i, j);
        cplx x0 = v[0];
        double ax0 = std::abs(x0);
        cplx phase = (ax0 > 0) ? x0 / ax0 : cplx(1.0);
        cplx alpha = -phase * nrm;
        v[0] -= alpha;
        double vn = 0;
        for (auto &z : v) vn += std::norm(z);
        if (vn > 0) {
            for (int jj = j; jj < n; ++jj) {
                cplx s = 0;
                for (int i = j; i < m; ++i) s += std::conj(v[i - j]) * W(i, jj);
                s *= 2.0 / vn;
                for (int i = j; i < m; ++i) W(i, jj) -= s * v[i - j];
            }
        }
        vs[j] = std::move(v);
        betas[j] = (vn > 0) ? cplx(2.0 / vn) : cplx(0.0);
    }
    R = Mat(n, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) R(i, j) = W(i, j);
    Q = Mat(m, n);
    for (int j = 0; j < n; ++j) Q(j, j) = 1.0;
    for (int j = n - 1; j >= 0; --j) {
        const auto &v = vs[j];
        if (betas[j] == cplx(0.0)) continue;
        for (int jj = 0; jj < n; ++jj) {
            cplx s = 0;
            for (int i = j; i < m; ++i) s += std::conj(v[i - j]) * Q(i, jj);
            s *= betas[j];
            for (int i = j; i < m; ++i) Q(i, jj) -= s * v[i - j];
        }
    }
}

// One-sided (Hestenes) Jacobi SVD of a square matrix: A = U diag(s) V^H,
// singular values in descending order.
inline void jacobi_svd_square(const Mat &A, Mat &U, std::vector<double> &s, Mat &V) {
    const int n = A.n, m = A.m;
    Mat W = A;
    V = Mat(n, n);
    for (int j = 0; j < n; ++j) V(j, j) = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                cplx *ap = W.col(p), *aq = W.col(q);
                double al = 0, be = 0;
                cplx ga = 0;
                for (int i = 0; i < m; ++i) {
                    al += std::norm(ap[i]);
                    be += std::norm(aq[i]);
                    ga += std::conj(ap[i]) * aq[i];
                }
                double ag = std::abs(ga);
                if (ag == 0.0 || ag <= 1e-15 * std::sqrt(al * be)) continue;
                off = std::max(off, ag / std::sqrt(al * be));
                cplx ph = ga / ag;  // exp(i phi)
                double zeta = (be - al) / (2.0 * ag);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                cplx phc = std::conj(ph);
                for (int i = 0; i < m; ++i) {
                    cplx x = ap[i], y = aq[i] * phc;
                    ap[i] = c * x - sn * y;
                    aq[i] = sn * x + c * y;
                }
                cplx *vp = V.col(p), *vq = V.col(q);
                for (int i = 0; i < n; ++i) {
                    cplx x = vp[i], y = vq[i] * phc;
                    vp[i] = c * x - sn * y;
                    vq[i] = sn * x + c * y;
                }
            }
        }
        if (off < 1e-14) break;
    }
    std::vector<double> nr(n);
    for (int j = 0; j < n; ++j) {
        double z = 0;
        for (int i = 0; i < m; ++i) z += std::norm(W(i, j));
        nr[j] = std::sqrt(z);
    }
    std::vector<int> ord(n);
    for (int j = 0; j < n; ++j) ord[j] = j;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return nr[a] > nr[b]; });
    U = Mat(m, n);
    Mat V2(n, n);
    s.assign(n, 0.0);
    for (int jj = 0; jj < n; ++jj) {
        int j = ord[jj];
        s[jj] = nr[j];
        double inv = nr[j] > 0 ? 1.0 / nr[j] : 0.0;
        for (int i = 0; i < m; ++i) U(i, jj) = W(i, j) * inv;
        for (int i = 0; i < n; ++i) V2(i, jj) = V(i, j);
    }
    V = V2;
}

// Truncated SVD A ~ U diag(s) V^H keeping s_i >= eps * s_0 (eq. (eq_epsg),
// with s_0 the largest singular value).  Works for any shape.
inline void svd_truncated(const Mat &A, double eps, Mat &U, std::vector<double> &s, Mat &V) {
    Mat Uf, Vf;
    std::vector<double> sf;
    if (A.m >= A.n) {
        Mat Q, R;
        qr_thin(A, Q, R);
        Mat Ur;
        jacobi_svd_square(R, Ur, sf, Vf);
        Uf = matmul(Q, 'N', Ur, 'N');
    } else {
        // A^H = Q R -> A = R^H Q^H; svd of R^H
        Mat AH(A.n, A.m);
        for (int j = 0; j < A.n; ++j)
            for (int i = 0; i < A.m; ++i) AH(j, i) = std::conj(A(i, j));
        Mat Q, R;
        qr_thin(AH, Q, R);
        Mat RH(R.n, R.m);
        for (int j = 0; j < R.n; ++j)
            for (int i = 0; i < R.m; ++i) RH(j, i) = std::conj(R(i, j));
        Mat Ur;
        jacobi_svd_square(RH, Uf, sf, Ur);
        Vf = matmul(Q, 'N', Ur, 'N');
    }
    int kk = 0;
    while (kk < (int)sf.size() && sf[kk] >= eps * sf[0]) ++kk;
    if (kk == 0) kk = 1;
    U = Mat(Uf.m, kk);
    V = Mat(Vf.m, kk);
    s.assign(sf.begin(), sf.begin() + kk);
    std::memcpy(U.a.data(), Uf.a.data(), sizeof(cplx) * (size_t)Uf.m * kk);
    std::memcpy(V.a.data(), Vf.a.data(), sizeof(cplx) * (size_t)Vf.m * kk);
}

}  // namespace fda
