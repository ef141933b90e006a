// Device part of fda_build: the truncated SVDs of G_up per level and
// direction (eqs. (eq_svdg), (eq_epsg), (eq_invg); rocSOLVER), and the
// reduced / compressed translation matrices (eq. (eq_cmpm2l) and the
// compressed M2M, L2L matrices of Section 4.3), formed as batched products
// of device-generated kernel matrices (rocBLAS).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "dsetup.hpp"

namespace fda {

static const double kRin = 1.05, kRout = 2.95;
static const double kSat = 0.7;

// out[b][i + j m] = G(X_i + t_b, Y_j)
__global__ void k_green_batched(const double *X, int m, const double *Y, int n, const double *t, double k,
                                double2 *out) {
    const int b = blockIdx.y;
    const int64_t mn = (int64_t)m * n;
    const double t0 = t[3 * b], t1 = t[3 * b + 1], t2 = t[3 * b + 2];
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < mn; idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx % m), j = (int)(idx / m);
        double a = X[3 * i] + t0 - Y[3 * j], c = X[3 * i + 1] + t1 - Y[3 * j + 1], d = X[3 * i + 2] + t2 - Y[3 * j + 2];
        double R = sqrt(a * a + c * c + d * d);
        double s, cs;
        sincos(k * R, &s, &cs);
        double inv = 1.0 / (4.0 * 3.14159265358979323846 * R);
        out[(int64_t)b * mn + idx] = make_double2(cs * inv, s * inv);
    }
}

namespace {

struct Err {
    int code;
    std::string msg;
};

void hchk(hipError_t e, const char *w) {
    if (e != hipSuccess) throw BuildError{FDA_EHIP, std::string(w) + ": " + hipGetErrorString(e)};
}
void rchk(rocblas_status s, const char *w) {
    if (s != rocblas_status_success) throw BuildError{FDA_EHIP, std::string(w) + ": rocBLAS/rocSOLVER status " + std::to_string((int)s)};
}

struct DBuf {
    void *p = nullptr;
    DBuf() = default;
    explicit DBuf(size_t bytes) {
        if (bytes == 0) bytes = 16;
        if (hipMalloc(&p, bytes) != hipSuccess) throw BuildError{FDA_ENOMEM, "device allocation in build failed"};
    }
    ~DBuf() {
        if (p) hipFree(p);
    }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p) { o.p = nullptr; }
    template <class T>
    T *as() const { return (T *)p; }
};

template <class T>
DBuf to_dev(const std::vector<T> &v) {
    DBuf b(sizeof(T) * std::max<size_t>(1, v.size()));
    if (!v.empty()) hchk(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "h2d");
    return b;
}

DBuf mat_to_dev(const Mat &M) {
    DBuf b(sizeof(double2) * std::max<size_t>(1, M.a.size()));
    hchk(hipMemcpy(b.p, M.a.data(), sizeof(double2) * M.a.size(), hipMemcpyHostToDevice), "h2d");
    return b;
}

void green_batched(const DBuf &X, int m, const DBuf &Y, int n, const std::vector<double> &t, double k, double2 *out) {
    int batch = (int)t.size() / 3;
    DBuf dt = to_dev(t);
    int64_t mn = (int64_t)m * n;
    int gx = (int)std::min<int64_t>((mn + 255) / 256, 2048);
    hipLaunchKernelGGL(k_green_batched, dim3(gx, batch), dim3(256), 0, nullptr, X.as<double>(), m, Y.as<double>(), n,
                       dt.as<double>(), k, out);
    hchk(hipGetLastError(), "green kernel");
}

std::vector<double> scaled(const std::vector<double> &P, double s) {
    std::vector<double> o(P);
    for (auto &v : o) v *= s;
    return o;
}

void rot_to(const double *u, double R[9]) {
    double c = u[2];
    double v[3] = {-u[1], u[0], 0.0};
    double vn = std::sqrt(v[0] * v[0] + v[1] * v[1]);
    if (vn < 1e-14) {
        double s = c > 0 ? 1.0 : -1.0;
        double I[9] = {1, 0, 0, 0, s, 0, 0, 0, s};
        std::memcpy(R, I, sizeof(I));
        return;
    }
    double V[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int q = 0; q < 3; ++q) s += V[3 * i + q] * V[3 * q + j];
            R[3 * i + j] = (i == j ? 1.0 : 0.0) + V[3 * i + j] + s / (1.0 + c);
        }
}

std::vector<double> rotated(const std::vector<double> &P, const double *u, double sign) {
    double R[9];
    rot_to(u, R);
    std::vector<double> o(P.size());
    for (size_t i = 0; i < P.size() / 3; ++i)
        for (int a = 0; a < 3; ++a)
            o[3 * i + a] = sign * (R[3 * a] * P[3 * i] + R[3 * a + 1] * P[3 * i + 1] + R[3 * a + 2] * P[3 * i + 2]);
    return o;
}

std::vector<double> cube_points(int p) {
    std::vector<double> out;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k)
                if (i == 0 || j == 0 || k == 0 || i == p - 1 || j == p - 1 || k == p - 1) {
                    out.push_back(-1.0 + 2.0 * i / (p - 1));
                    out.push_back(-1.0 + 2.0 * j / (p - 1));
                    out.push_back(-1.0 + 2.0 * k / (p - 1));
                }
    return out;
}

// Batched thin SVD A = U diag(S) V^H of column-major matrices (rocSOLVER):
// method 1 = one-sided Jacobi (gesvdj), otherwise bidiagonalisation + QR
// (gesvd).  V receives V^H (rows = right singular vectors); S descends.
// E is workspace of min(m, n) doubles per matrix.
void batched_svd(rocblas_handle h, int method, int m, int n, rocblas_double_complex *A, int lda, rocblas_stride sA,
                 double *S, rocblas_stride sS, rocblas_double_complex *U, int ldu, rocblas_stride sU,
                 rocblas_double_complex *V, int ldv, rocblas_stride sV, double *E, rocblas_int *info, int batch,
                 const char *what) {
    if (method == 1) {
        DBuf res(sizeof(double) * (size_t)batch), sweeps(sizeof(rocblas_int) * (size_t)batch);
        rchk(rocsolver_zgesvdj_strided_batched(h, rocblas_svect_singular, rocblas_svect_singular, m, n, A, lda, sA,
                                               0.0, res.as<double>(), 100, sweeps.as<rocblas_int>(), S, sS, U, ldu,
                                               sU, V, ldv, sV, info, batch),
             what);
    } else {
        rchk(rocsolver_zgesvd_strided_batched(h, rocblas_svect_singular, rocblas_svect_singular, m, n, A, lda, sA, S,
                                              sS, U, ldu, sU, V, ldv, sV, E, std::min(m, n), rocblas_outofplace,
                                              info, batch),
             what);
    }
}

// Batched SVD of `batch` m x n matrices (m >= n) stored contiguously in A
// (destroyed).  Returns host copies of S (batch x n), U (batch x m x n) and
// V^H (batch x n x n).
void svd_batched(rocblas_handle h, int method, double2 *A, int m, int n, int batch, std::vector<double> &S,
                 std::vector<cplx> &U, std::vector<cplx> &Vh) {
    DBuf dS(sizeof(double) * (size_t)batch * n), dU(sizeof(double2) * (size_t)batch * m * n),
        dV(sizeof(double2) * (size_t)batch * n * n), dE(sizeof(double) * (size_t)batch * n),
        dinfo(sizeof(rocblas_int) * batch);
    batched_svd(h, method, m, n, (rocblas_double_complex *)A, m, (rocblas_stride)m * n, dS.as<double>(), n,
                dU.as<rocblas_double_complex>(), m, (rocblas_stride)m * n, dV.as<rocblas_double_complex>(), n,
                (rocblas_stride)n * n, dE.as<double>(), dinfo.as<rocblas_int>(), batch, "zgesvd");
    S.resize((size_t)batch * n);
    U.resize((size_t)batch * m * n);
    Vh.resize((size_t)batch * n * n);
    std::vector<rocblas_int> info(batch);
    hchk(hipMemcpy(S.data(), dS.p, sizeof(double) * S.size(), hipMemcpyDeviceToHost), "d2h");
    hchk(hipMemcpy(U.data(), dU.p, sizeof(double2) * U.size(), hipMemcpyDeviceToHost), "d2h");
    hchk(hipMemcpy(Vh.data(), dV.p, sizeof(double2) * Vh.size(), hipMemcpyDeviceToHost), "d2h");
    hchk(hipMemcpy(info.data(), dinfo.p, sizeof(rocblas_int) * batch, hipMemcpyDeviceToHost), "d2h");
    for (int b = 0; b < batch; ++b)
        if (info[b] != 0) throw BuildError{FDA_EHIP, "SVD did not converge"};
}

int trunc_rank(const double *s, int n, double eps) {
    int r = 0;
    while (r < n && s[r] >= eps * s[0]) ++r;
    return std::max(r, 1);
}

// C_b = op(A) * B_b (+ strides), complex double, column-major.
void zgemm_sb(rocblas_handle h, rocblas_operation ta, int m, int n, int kk, const double2 *A, int lda,
              int64_t sa, const double2 *B, int ldb, int64_t sb, double2 *C, int ldc, int64_t sc, int batch) {
    rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    rchk(rocblas_zgemm_strided_batched(h, ta, rocblas_operation_none, m, n, kk, &one, (const rocblas_double_complex *)A,
                                       lda, sa, (const rocblas_double_complex *)B, ldb, sb, &zero,
                                       (rocblas_double_complex *)C, ldc, sc, batch),
         "zgemm");
}

// Zero-padded copy of the first `cols` columns of an (m x c) host matrix to
// (m x padc), optionally scaling column j by 1/s[j].
Mat padded(const Mat &M, int padc, const std::vector<double> *inv_scale) {
    Mat P(M.m, padc);
    for (int j = 0; j < std::min(M.n, padc); ++j)
        for (int i = 0; i < M.m; ++i) P(i, j) = inv_scale ? M(i, j) / (*inv_scale)[j] : M(i, j);
    return P;
}

}  // namespace

// Outgoing check points of a level / slot, relative to the box centre: on a
// directional level the cone far set turned to the slot's orbit
// representative, then carried onto the slot by its cube symmetry.
static std::vector<double> cone_points(const Level &lv, int slot, double sign) {
    const int r = lv.rep_slot.empty() ? slot : lv.rep_slot[slot];
    const int g = lv.sym.empty() ? 0 : lv.sym[slot];
    std::vector<double> X = rotated(lv.far, &lv.dirvec[3 * lv.active[r]], sign);
    for (size_t i = 0; i < X.size() / 3; ++i) {
        double w[3];
        cube_sym_apply(g, &X[3 * i], w);
        for (int a = 0; a < 3; ++a) X[3 * i + a] = w[a];
    }
    return X;
}
std::vector<double> out_check(const Level &lv, int slot) {
    if (!lv.hf) return scaled(lv.cube, kRout * lv.r);
    return cone_points(lv, slot, 1.0);
}
// Incoming equivalent points: the outgoing check points reflected through
// the centre.
std::vector<double> in_equiv(const Level &lv, int slot) {
    if (!lv.hf) return scaled(lv.cube, kRout * lv.r);
    return cone_points(lv, slot, -1.0);
}

// Permutation of the cube-surface points (p per edge) under cube symmetry
// g: point k goes to point perm[k].
static std::vector<int> cube_perm(const std::vector<double> &cube, int p, int g) {
    const int n = (int)cube.size() / 3;
    auto key = [&](const double *x) {
        int64_t k = 0;
        for (int a = 0; a < 3; ++a) k = k * 4096 + (int64_t)std::lround((x[a] + 1.0) * 0.5 * (p - 1));
        return k;
    };
    std::unordered_map<int64_t, int> idx;
    for (int k = 0; k < n; ++k) idx[key(&cube[3 * k])] = k;
    std::vector<int> perm(n);
    for (int k = 0; k < n; ++k) {
        double w[3];
        cube_sym_apply(g, &cube[3 * k], w);
        auto it = idx.find(key(w));
        if (it == idx.end()) throw BuildError{FDA_EINVAL, "internal: cube points not symmetric"};
        perm[k] = it->second;
    }
    return perm;
}

void device_factors(HostPlan &hp, rocblas_handle h) {
    const int L = hp.depth;
    const double k = hp.k;
    const int pmin = hp.opt.p_min > 0 ? hp.opt.p_min
                                      : (int)std::ceil(std::log10(1.0 / hp.eps) - 1e-12) + hp.opt.p0;
    for (int l = hp.top; l <= L; ++l) {
        Level &lv = hp.lv[l];
        // adaptive p: smallest p whose G_up rank stays below kSat of the points
        int p = std::max(3, pmin);
        for (;; ++p) {
            std::vector<double> cube = cube_points(p);
            int nc = (int)cube.size() / 3;
            std::vector<double> X = lv.hf ? rotated(lv.far, &lv.dirvec[3 * lv.active[0]], 1.0) : scaled(cube, kRout * lv.r);
            int m = (int)X.size() / 3;
            DBuf dX = to_dev(X), dY = to_dev(scaled(cube, kRin * lv.r));
            DBuf G(sizeof(double2) * (size_t)m * nc);
            green_batched(dX, m, dY, nc, {0.0, 0.0, 0.0}, k, G.as<double2>());
            std::vector<double> S;
            std::vector<cplx> U, Vh;
            svd_batched(h, hp.opt.svd_method, G.as<double2>(), m, nc, 1, S, U, Vh);
            int r = trunc_rank(S.data(), nc, hp.svd_eps);
            lv.cube = cube;
            if (hp.opt.p_fixed || (double)r <= kSat * nc || p >= 14) break;
        }
        lv.p = p;
        const int nc = (int)lv.cube.size() / 3;
        std::vector<int> negp(nc);
        for (int i = 0; i < nc; ++i) negp[i] = nc - 1 - i;
        // G_up for every orbit representative slot, batched; the other slots
        // take their representative's factors carried over by their cube
        // symmetry g: their check points are g X_rep, so G_up,s = G_up,rep
        // with its columns (equivalent points) permuted, and V_up,s is
        // V_up,rep with its rows permuted the same way
        std::vector<int> reps;
        for (int s = 0; s < lv.nslot; ++s)
            if (lv.rep_slot.empty() || lv.rep_slot[s] == s) reps.push_back(s);
        const int nrep = (int)reps.size();
        std::vector<double> X0 = out_check(lv, reps[0]);
        const int m = (int)X0.size() / 3;
        DBuf dY = to_dev(scaled(lv.cube, kRin * lv.r));
        DBuf G(sizeof(double2) * (size_t)nrep * m * nc);
        for (int i = 0; i < nrep; ++i) {
            DBuf dX = to_dev(out_check(lv, reps[i]));
            green_batched(dX, m, dY, nc, {0.0, 0.0, 0.0}, k, G.as<double2>() + (size_t)i * m * nc);
        }
        std::vector<double> S;
        std::vector<cplx> U, Vh;
        svd_batched(h, hp.opt.svd_method, G.as<double2>(), m, nc, nrep, S, U, Vh);
        lv.Uu.assign(lv.nslot, Mat());
        lv.Vu.assign(lv.nslot, Mat());
        lv.Ud.assign(lv.nslot, Mat());
        lv.Vd.assign(lv.nslot, Mat());
        lv.su.assign(lv.nslot, {});
        lv.sd.assign(lv.nslot, {});
        lv.ku_s.assign(lv.nslot, 0);
        lv.kd_s.assign(lv.nslot, 0);
        // G_dn = Pi G_up^T: U_dn = Pi conj(V_up), V_dn = conj(U_up)
        auto set_dn = [&](int s) {
            const int r = lv.Uu[s].n;
            Mat Ud(nc, r), Vd(m, r);
            for (int j = 0; j < r; ++j) {
                for (int i = 0; i < nc; ++i) Ud(i, j) = std::conj(lv.Vu[s](lv.hf ? negp[i] : i, j));
                for (int i = 0; i < m; ++i) Vd(i, j) = std::conj(lv.Uu[s](i, j));
            }
            lv.Ud[s] = std::move(Ud);
            lv.Vd[s] = std::move(Vd);
        };
        for (int i = 0; i < nrep; ++i) {
            const int s = reps[i];
            const double *Ss = S.data() + (size_t)i * nc;
            int r = trunc_rank(Ss, nc, hp.svd_eps);
            Mat Uu(m, r), Vu(nc, r);
            const cplx *Us = U.data() + (size_t)i * m * nc;
            const cplx *Vs = Vh.data() + (size_t)i * nc * nc;  // V^H, n x n column-major
            for (int j = 0; j < r; ++j) {
                for (int q = 0; q < m; ++q) Uu(q, j) = Us[q + (size_t)j * m];
                for (int q = 0; q < nc; ++q) Vu(q, j) = std::conj(Vs[j + (size_t)q * nc]);
            }
            lv.Uu[s] = std::move(Uu);
            lv.Vu[s] = std::move(Vu);
            lv.su[s].assign(Ss, Ss + r);
            lv.sd[s] = lv.su[s];
            lv.ku_s[s] = lv.kd_s[s] = r;
            set_dn(s);
        }
        for (int s = 0; s < lv.nslot; ++s) {
            if (lv.rep_slot.empty() || lv.rep_slot[s] == s) continue;
            const int rs = lv.rep_slot[s];
            // G(g X, Y_j) = G(X, g^-1 Y_j): column j of G_up,s is column
            // perm^-1(j) of G_up,rep, where g Y_k = Y_perm(k)
            const std::vector<int> perm = cube_perm(lv.cube, lv.p, lv.sym[s]);
            const Mat &Vr = lv.Vu[rs];
            Mat Vu(nc, Vr.n);
            for (int j = 0; j < Vr.n; ++j)
                for (int q = 0; q < nc; ++q) Vu(perm[q], j) = Vr(q, j);
            lv.Uu[s] = lv.Uu[rs];
            lv.Vu[s] = std::move(Vu);
            lv.su[s] = lv.su[rs];
            lv.sd[s] = lv.sd[rs];
            lv.ku_s[s] = lv.kd_s[s] = lv.ku_s[rs];
            set_dn(s);
        }
        lv.ku = *std::max_element(lv.ku_s.begin(), lv.ku_s.end());
        lv.kd = lv.ku;
    }
}

void device_translations(const HostPlan &hp, rocblas_handle h, DevTranslations &out) {
    const int L = hp.depth;
    const double k = hp.k;
    out.K.assign(L + 1, nullptr);
    out.M.assign(L + 1, nullptr);
    out.Lo.assign(L + 1, nullptr);
    auto keep = [&](size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess) throw BuildError{FDA_ENOMEM, "hipMalloc failed"};
        out.allocs.push_back(q);
        out.bytes += (int64_t)bytes;
        return (double2 *)q;
    };
    for (int l = hp.top; l <= L; ++l) {
        const Level &lv = hp.lv[l];
        const int nc = (int)lv.cube.size() / 3;
        const size_t ksz = (size_t)lv.kd * lv.ku;
        double2 *K = keep(sizeof(double2) * lv.offsets.size() * ksz);
        out.K[l] = K;
        DBuf dcube = to_dev(scaled(lv.cube, kRin * lv.r));
        // offsets are numbered slot by slot (host_setup sorts them)
        size_t o0 = 0;
        for (int s = 0; s < lv.nslot && o0 < lv.offsets.size(); ++s) {
            size_t o1 = o0;
            while (o1 < lv.offsets.size() && (lv.hf ? lv.slot_of_dir[lv.offset_dir[o1]] : 0) == s) ++o1;
            if (o1 == o0) continue;
            Mat Vu = padded(lv.Vu[s], lv.ku, nullptr), Ud = padded(lv.Ud[s], lv.kd, nullptr);
            DBuf dVu = mat_to_dev(Vu), dUd = mat_to_dev(Ud);
            const size_t chunk = std::max<size_t>(1, (size_t)(1u << 30) / (sizeof(double2) * (size_t)nc * nc));
            for (size_t c0 = o0; c0 < o1; c0 += chunk) {
                size_t c1 = std::min(o1, c0 + chunk);
                int batch = (int)(c1 - c0);
                std::vector<double> t(3 * batch);
                for (int b = 0; b < batch; ++b)
                    for (int q = 0; q < 3; ++q) t[3 * b + q] = lv.offsets[c0 + b][q] * lv.w;
                DBuf Gd(sizeof(double2) * (size_t)batch * nc * nc), W(sizeof(double2) * (size_t)batch * nc * lv.ku);
                green_batched(dcube, nc, dcube, nc, t, k, Gd.as<double2>());
                zgemm_sb(h, rocblas_operation_none, nc, lv.ku, nc, Gd.as<double2>(), nc, (int64_t)nc * nc,
                         dVu.as<double2>(), nc, 0, W.as<double2>(), nc, (int64_t)nc * lv.ku, batch);
                zgemm_sb(h, rocblas_operation_conjugate_transpose, lv.kd, lv.ku, nc, dUd.as<double2>(), nc, 0,
                         W.as<double2>(), nc, (int64_t)nc * lv.ku, K + c0 * ksz, lv.kd, (int64_t)ksz, batch);
                hchk(hipDeviceSynchronize(), "K batch");
            }
            o0 = o1;
        }
    }
    // M2M and L2L towards each child level
    for (int l = hp.top; l < L; ++l) {
        const Level &P = hp.lv[l], &C = hp.lv[l + 1];
        const int ncC = (int)C.cube.size() / 3;
        const size_t msz = (size_t)P.ku * C.ku, lsz = (size_t)C.kd * P.kd;
        double2 *M = keep(sizeof(double2) * 8 * P.nslot * msz);
        double2 *Lo = keep(sizeof(double2) * 8 * P.nslot * lsz);
        out.M[l] = M;
        out.Lo[l] = Lo;
        DBuf dcin = to_dev(scaled(C.cube, kRin * C.r));
        std::vector<double> t(24);
        for (int o = 0; o < 8; ++o) {
            t[3 * o] = (o & 4) ? C.r : -C.r;
            t[3 * o + 1] = (o & 2) ? C.r : -C.r;
            t[3 * o + 2] = (o & 1) ? C.r : -C.r;
        }
        std::vector<double> negt(t);
        for (auto &v : negt) v = -v;
        for (int s = 0; s < P.nslot; ++s) {
            const int cs = hp.cslot_of(l, s);
            std::vector<double> X = out_check(P, s), Y = in_equiv(P, s);
            const int nX = (int)X.size() / 3, nY = (int)Y.size() / 3;
            DBuf dX = to_dev(X), dYp = to_dev(Y);
            // M~_o = S_P^-1 U_P^H G(X, child equiv + off_o) V_C
            {
                Mat Us = padded(P.Uu[s], P.ku, &P.su[s]);  // U S^-1: U^H then carries S^-1
                Mat Vc = padded(C.Vu[cs], C.ku, nullptr);
                DBuf dU = mat_to_dev(Us), dV = mat_to_dev(Vc);
                DBuf E(sizeof(double2) * 8 * (size_t)nX * ncC), W(sizeof(double2) * 8 * (size_t)nX * C.ku);
                // E_o[i, j] = G(X_i, cin_j + off_o) = G(X_i - off_o, cin_j)
                green_batched(dX, nX, dcin, ncC, negt, k, E.as<double2>());
                zgemm_sb(h, rocblas_operation_none, nX, C.ku, ncC, E.as<double2>(), nX, (int64_t)nX * ncC,
                         dV.as<double2>(), ncC, 0, W.as<double2>(), nX, (int64_t)nX * C.ku, 8);
                zgemm_sb(h, rocblas_operation_conjugate_transpose, P.ku, C.ku, nX, dU.as<double2>(), nX, 0,
                         W.as<double2>(), nX, (int64_t)nX * C.ku, M + (size_t)s * msz, P.ku,
                         (int64_t)P.nslot * msz, 8);
                hchk(hipDeviceSynchronize(), "M batch");
            }
            // L~_o = U_C^H G(child check + off_o, Y) V_dn,P S_P^-1
            {
                Mat Vd = padded(P.Vd[s], P.kd, &P.sd[s]);
                Mat Uc = padded(C.Ud[cs], C.kd, nullptr);
                DBuf dV = mat_to_dev(Vd), dU = mat_to_dev(Uc);
                DBuf E(sizeof(double2) * 8 * (size_t)ncC * nY), W(sizeof(double2) * 8 * (size_t)ncC * P.kd);
                green_batched(dcin, ncC, dYp, nY, t, k, E.as<double2>());
                zgemm_sb(h, rocblas_operation_none, ncC, P.kd, nY, E.as<double2>(), ncC, (int64_t)ncC * nY,
                         dV.as<double2>(), nY, 0, W.as<double2>(), ncC, (int64_t)ncC * P.kd, 8);
                zgemm_sb(h, rocblas_operation_conjugate_transpose, C.kd, P.kd, ncC, dU.as<double2>(), ncC, 0,
                         W.as<double2>(), ncC, (int64_t)ncC * P.kd, Lo + (size_t)s * lsz, C.kd,
                         (int64_t)P.nslot * lsz, 8);
                hchk(hipDeviceSynchronize(), "L batch");
            }
        }
    }
}

// Pack U^ = U[:, :r] and V^ = diag(s[:r]) V^H[:r, :] per translation; V^
// gets zero columns up to nld (ku rounded up to 4).
__global__ void k_pack_lowrank(const double2 *U, const double *S, const double2 *Vh, const int32_t *rank, int kd,
                               int ku, int nld, int mn, int rmax, double2 *Ulr, double2 *Vlr) {
    const int op = blockIdx.y;
    const int r = rank[op];
    const double2 *Uo = U + (int64_t)op * kd * mn;
    const double2 *Vo = Vh + (int64_t)op * mn * ku;
    const double *So = S + (int64_t)op * mn;
    double2 *Uout = Ulr + (int64_t)op * kd * rmax;
    double2 *Vout = Vlr + (int64_t)op * rmax * nld;
    const int64_t nU = (int64_t)kd * rmax, nV = (int64_t)rmax * nld;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nU + nV; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nU) {
            const int i = (int)(e % kd), j = (int)(e / kd);
            Uout[e] = (j < r && j < mn) ? Uo[i + (int64_t)j * kd] : make_double2(0.0, 0.0);
        } else {
            const int64_t f = e - nU;
            const int j = (int)(f % rmax), c = (int)(f / rmax);
            double2 v = make_double2(0.0, 0.0);
            if (j < r && j < mn && c < ku) {
                const double2 q = Vo[j + (int64_t)c * mn];
                v = make_double2(So[j] * q.x, So[j] * q.y);
            }
            Vout[f] = v;
        }
    }
}

// Truncated SVD factors of `count` column-major m x n matrices (stride m*n):
// A = U^ V^ with U^ = U[:, :r] (m x rmax) and V^ = diag(s[:r]) V^H[:r, :]
// (rmax x n, stored with n rounded up to a multiple of 4 and zero columns
// there), r the number of singular values >= m2l_svd_eps * s_0, padded to a
// multiple of 4.  rmax = 0 (nothing kept) when some rank exceeds max_rank or
// 2 r >= min(m, n) (the factors would not pay; Section 4.2).
LowRank factor_batch(const HostPlan &hp, rocblas_handle h, const double2 *mats, int m, int n, int count,
                     int max_rank, DevTranslations &out, const char *what) {
    LowRank lr;
    const int mn = std::min(m, n);
    const size_t msz = (size_t)m * n;
    DBuf A(sizeof(double2) * msz * count), dS(sizeof(double) * (size_t)mn * count),
        dU(sizeof(double2) * (size_t)m * mn * count), dV(sizeof(double2) * (size_t)mn * n * count),
        dE(sizeof(double) * (size_t)mn * count), dinfo(sizeof(rocblas_int) * count);
    hchk(hipMemcpy(A.p, mats, sizeof(double2) * msz * count, hipMemcpyDeviceToDevice), "copy");
    batched_svd(h, hp.opt.svd_method, m, n, A.as<rocblas_double_complex>(), m, (rocblas_stride)msz, dS.as<double>(),
                mn, dU.as<rocblas_double_complex>(), m, (rocblas_stride)m * mn, dV.as<rocblas_double_complex>(), mn,
                (rocblas_stride)mn * n, dE.as<double>(), dinfo.as<rocblas_int>(), count, what);
    std::vector<double> S((size_t)mn * count);
    std::vector<rocblas_int> info(count);
    hchk(hipMemcpy(S.data(), dS.p, sizeof(double) * S.size(), hipMemcpyDeviceToHost), "d2h");
    hchk(hipMemcpy(info.data(), dinfo.p, sizeof(rocblas_int) * count, hipMemcpyDeviceToHost), "d2h");
    std::vector<int32_t> rank(count);
    lr.rtrue.assign(count, 0);
    int rmax = 0, rtmax = 0;
    double rsum = 0;
    for (int o = 0; o < count; ++o) {
        if (info[o] != 0) throw BuildError{FDA_EHIP, std::string("SVD did not converge: ") + what};
        const double *so = S.data() + (size_t)o * mn;
        int r = 0;
        while (r < mn && so[r] >= hp.m2l_svd_eps * so[0] && so[0] > 0) ++r;
        r = std::max(r, 1);
        rsum += r;
        lr.rtrue[o] = r;
        rtmax = std::max(rtmax, r);
        r = std::min(mn, (r + 3) / 4 * 4);
        rank[o] = r;
        rmax = std::max(rmax, r);
    }
    lr.mean = rsum / std::max(1, count);
    lr.rtrue_max = rtmax;
    if (rmax > max_rank || 2 * rmax >= mn) return lr;
    auto keep = [&](size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess) throw BuildError{FDA_ENOMEM, "hipMalloc failed"};
        out.allocs.push_back(q);
        out.bytes += (int64_t)bytes;
        return q;
    };
    lr.U = (double2 *)keep(sizeof(double2) * (size_t)m * rmax * count);
    const int nld = (n + 3) / 4 * 4;
    lr.V = (double2 *)keep(sizeof(double2) * (size_t)rmax * nld * count);
    lr.rank = (int32_t *)keep(sizeof(int32_t) * count);
    hchk(hipMemcpy(lr.rank, rank.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice), "h2d");
    hipLaunchKernelGGL(k_pack_lowrank, dim3(64, count), dim3(256), 0, nullptr, dU.as<double2>(), dS.as<double>(),
                       dV.as<double2>(), lr.rank, m, n, nld, mn, rmax, lr.U, lr.V);
    hchk(hipGetLastError(), "pack");
    hchk(hipDeviceSynchronize(), "pack sync");
    lr.rmax = rmax;
    return lr;
}

void device_lowrank_m2l(const HostPlan &hp, rocblas_handle h, DevTranslations &out, int max_rank) {
    const int L = hp.depth;
    out.Ulr.assign(L + 1, nullptr);
    out.Vlr.assign(L + 1, nullptr);
    out.lr_rank.assign(L + 1, nullptr);
    out.rmax.assign(L + 1, 0);
    out.mean_rank.assign(L + 1, 0.0);
    out.true_rank.assign(L + 1, {});
    for (int l = hp.top; l <= L; ++l) {
        const Level &lv = hp.lv[l];
        const int noff = (int)lv.offsets.size();
        if (noff == 0) continue;
        LowRank lr = factor_batch(hp, h, out.K[l], lv.kd, lv.ku, noff, max_rank, out, "zgesvd (M2L)");
        out.mean_rank[l] = lr.mean;
        if (lr.rmax == 0) continue;
        out.true_rank[l] = lr.rtrue;
        out.Ulr[l] = lr.U;
        out.Vlr[l] = lr.V;
        out.lr_rank[l] = lr.rank;
        out.rmax[l] = lr.rmax;
    }
}

}  // namespace fda
