// HIP kernels of the fast directional BEM matvec and of the GMRES solver
// (gfx950).  Complex values are interleaved double2 (re, im).
//
// Matvec pipeline (Algorithm, Steps 2-4), all in element tree order:
//   near field (S2T, eq. (eq_sum)) -> leaf S2M -> M2M up the tree ->
//   M2L per level -> L2L down the tree -> leaf L2T (eq. (eq_l2t)).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace fda {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(double2 &acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// ------------------------------------------------------------ quadrature

__constant__ double c_r7b[7][3];
__constant__ double c_r7w[7];
__constant__ double c_glx[32];
__constant__ double c_glw[32];

// exp(i k R) / (4 pi R) and the derivative factor G'(R) = G (ikR - 1)/R.
__device__ __forceinline__ void green_pair(double k, double R, double2 &g, double2 &gp) {
    double s, c;
    sincos(k * R, &s, &c);
    double inv = 1.0 / (4.0 * 3.14159265358979323846 * R);
    g = make_double2(c * inv, s * inv);
    // (ikR - 1)/R
    double2 f = make_double2(-1.0 / R, k);
    gp = cmul(g, f);
}

// [dG/dn_y + alpha d2G/dn_x dn_y](x, y) (paper normal convention).
__device__ __forceinline__ double2 lhs_kernel(const double *x, const double *y, const double *nx, const double *ny,
                                              double k, double2 alpha) {
    double r0 = x[0] - y[0], r1 = x[1] - y[1], r2 = x[2] - y[2];
    double R = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    double2 g, gp;
    green_pair(k, R, g, gp);
    double rnx = (r0 * nx[0] + r1 * nx[1] + r2 * nx[2]) / R;
    double rny = (r0 * ny[0] + r1 * ny[1] + r2 * ny[2]) / R;
    double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
    double2 d1 = make_double2(-gp.x * rny, -gp.y * rny);
    // g/R^2 [ (1 - ikR) nn - (3 - 3ikR - k^2R^2) rnx rny ]
    double kR = k * R;
    double2 br = make_double2(nn - (3.0 - kR * kR) * rnx * rny, -kR * nn + 3.0 * kR * rnx * rny);
    double2 d2 = cmul(g, br);
    double iR2 = 1.0 / (R * R);
    d2.x *= iR2;
    d2.y *= iR2;
    double2 ad2 = cmul(alpha, d2);
    return make_double2(d1.x + ad2.x, d1.y + ad2.y);
}

// Near-field entry A_ij (i != j): 7-point rule on 4^level midpoint
// sub-triangles of triangle j.
__device__ double2 near_entry(const double *tv, double area, const double *x, const double *nx, const double *ny,
                              double k, double2 alpha, int level) {
    double2 acc = make_double2(0.0, 0.0);
    const int nsub = 1 << (2 * level);
    const double asub = area / nsub;
    for (int t = 0; t < nsub; ++t) {
        double a[3], b[3], c[3];
        for (int q = 0; q < 3; ++q) {
            a[q] = tv[q];
            b[q] = tv[3 + q];
            c[q] = tv[6 + q];
        }
        for (int d = level - 1; d >= 0; --d) {
            int digit = (t >> (2 * d)) & 3;
            double ab[3], bc[3], ca[3];
            for (int q = 0; q < 3; ++q) {
                ab[q] = 0.5 * (a[q] + b[q]);
                bc[q] = 0.5 * (b[q] + c[q]);
                ca[q] = 0.5 * (c[q] + a[q]);
            }
            for (int q = 0; q < 3; ++q) {
                double na, nb, nc;
                if (digit == 0) { na = a[q]; nb = ab[q]; nc = ca[q]; }
                else if (digit == 1) { na = b[q]; nb = bc[q]; nc = ab[q]; }
                else if (digit == 2) { na = c[q]; nb = ca[q]; nc = bc[q]; }
                else { na = ab[q]; nb = bc[q]; nc = ca[q]; }
                a[q] = na;
                b[q] = nb;
                c[q] = nc;
            }
        }
        for (int p = 0; p < 7; ++p) {
            double y[3];
            for (int q = 0; q < 3; ++q) y[q] = c_r7b[p][0] * a[q] + c_r7b[p][1] * b[q] + c_r7b[p][2] * c[q];
            double2 v = lhs_kernel(x, y, nx, ny, k, alpha);
            double w = c_r7w[p] * asub;
            acc.x += w * v.x;
            acc.y += w * v.y;
        }
    }
    return acc;
}

// Diagonal entry: 1/2 + alpha * f.p. int d2G over the element's own flat
// triangle at its centroid = 1/2 + alpha (ik/2 - (1/4pi) int exp(ikR)/R dtheta),
// the angular integral taken edge by edge with 32-point Gauss-Legendre.
__device__ double2 self_entry(const double *tv, const double *x, double k, double2 alpha) {
    double2 s = make_double2(0.0, 0.0);
    for (int e = 0; e < 3; ++e) {
        const double *p = tv + 3 * e, *q = tv + 3 * ((e + 1) % 3);
        double ev[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        double L = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        double eh[3] = {ev[0] / L, ev[1] / L, ev[2] / L};
        double t = (x[0] - p[0]) * eh[0] + (x[1] - p[1]) * eh[1] + (x[2] - p[2]) * eh[2];
        double f[3] = {p[0] + t * eh[0] - x[0], p[1] + t * eh[1] - x[1], p[2] + t * eh[2] - x[2]};
        double d = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        double ph1 = atan2(-t, d), ph2 = atan2(L - t, d);
        double half = 0.5 * (ph2 - ph1), mid = 0.5 * (ph2 + ph1);
        for (int g = 0; g < 32; ++g) {
            double R = d / cos(mid + half * c_glx[g]);
            double sn, cs;
            sincos(k * R, &sn, &cs);
            double w = half * c_glw[g] / R;
            s.x += w * cs;
            s.y += w * sn;
        }
    }
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
    double2 hyp = make_double2(-s.x * inv4pi, 0.5 * k - s.y * inv4pi);
    double2 ah = cmul(alpha, hyp);
    return make_double2(0.5 + ah.x, ah.y);
}

__global__ void k_near_blocks(const int64_t *leaf_off, const int64_t *col_off, const int32_t *cols,
                              const int64_t *blk_off, const double *tri, const double *cen, const double *nrm,
                              const double *area, double k, double2 alpha, double h, double2 *vals) {
    const int b = blockIdx.x;
    const int64_t t0 = leaf_off[b];
    const int nt = (int)(leaf_off[b + 1] - t0);
    const int64_t c0 = col_off[b];
    const int nc = (int)(col_off[b + 1] - c0);
    double2 *blk = vals + blk_off[b];
    for (int idx = threadIdx.x; idx < nt * nc; idx += blockDim.x) {
        int i = idx / nc, c = idx - i * nc;
        int64_t ti = t0 + i, tj = cols[c0 + c];
        const double *x = cen + 3 * ti;
        double2 v;
        if (ti == tj) {
            v = self_entry(tri + 9 * tj, x, k, alpha);
        } else {
            const double *cj = cen + 3 * tj;
            double dd = sqrt((x[0] - cj[0]) * (x[0] - cj[0]) + (x[1] - cj[1]) * (x[1] - cj[1]) +
                             (x[2] - cj[2]) * (x[2] - cj[2]));
            int level = (dd < h) ? 3 : (dd < 1.75 * h) ? 2 : (dd < 2.5 * h) ? 1 : 0;
            v = near_entry(tri + 9 * tj, area[tj], x, nrm + 3 * ti, nrm + 3 * tj, k, alpha, level);
        }
        blk[idx] = v;
    }
}

// ------------------------------------------------------------ matvec

// y_tree[i] = sum over the near leaves of the block entries times x.
__global__ void k_p2p(const int64_t *leaf_off, const int32_t *nl_off, const int32_t *nl, const int64_t *blk_off,
                      const double2 *vals, const double2 *x, double2 *y, int64_t N) {
    extern __shared__ double2 xs[];
    const int b = blockIdx.x;
    const double2 *xr = x + (int64_t)blockIdx.y * N;
    double2 *yr = y + (int64_t)blockIdx.y * N;
    int nc = 0;
    for (int q = nl_off[b]; q < nl_off[b + 1]; ++q) {
        int s = nl[q];
        int64_t s0 = leaf_off[s];
        int ns = (int)(leaf_off[s + 1] - s0);
        for (int i = threadIdx.x; i < ns; i += blockDim.x) xs[nc + i] = xr[s0 + i];
        nc += ns;
    }
    __syncthreads();
    const int64_t t0 = leaf_off[b];
    const int nt = (int)(leaf_off[b + 1] - t0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double2 *blk = vals + blk_off[b];
    for (int i = wv; i < nt; i += nw) {
        double2 acc = make_double2(0.0, 0.0);
        const double2 *row = blk + (int64_t)i * nc;
        for (int c = lane; c < nc; c += 64) cfma(acc, row[c], xs[c]);
        for (int o = 32; o > 0; o >>= 1) {
            acc.x += __shfl_down(acc.x, o, 64);
            acc.y += __shfl_down(acc.y, o, 64);
        }
        if (lane == 0) yr[t0 + i] = acc;
    }
}

// s_leaf = S~ x_leaf
__global__ void k_s2m(const int64_t *leaf_off, const double2 *S, int ku, const double2 *x, double2 *s, int64_t N,
                      int64_t sstride) {
    extern __shared__ double2 xs[];
    const int b = blockIdx.x;
    const double2 *xr = x + (int64_t)blockIdx.y * N;
    const int64_t e0 = leaf_off[b];
    const int nl = (int)(leaf_off[b + 1] - e0);
    for (int i = threadIdx.x; i < nl; i += blockDim.x) xs[i] = xr[e0 + i];
    __syncthreads();
    const double2 *Sb = S + (int64_t)ku * e0;
    double2 *sr = s + (int64_t)blockIdx.y * sstride + (int64_t)b * ku;
    for (int r = threadIdx.x; r < ku; r += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < nl; ++j) cfma(acc, Sb[r + (int64_t)j * ku], xs[j]);
        sr[r] = acc;
    }
}

#define FDA_MAXR 4  // rows per thread: ranks up to 4 * blockDim

// Parent outgoing states from the children (M2M).
__global__ void k_m2m(int nslotP, int kuP, const int32_t *child_begin, const int32_t *octant, int nslotC, int kuC,
                      const int32_t *cslot, const double2 *M, const double2 *sC, double2 *sP, int64_t strideC,
                      int64_t strideP) {
    extern __shared__ double2 v[];
    const int g = blockIdx.x;
    const int P = g / nslotP, sl = g - P * nslotP;
    const int cs = cslot[sl];
    const double2 *sCr = sC + (int64_t)blockIdx.y * strideC;
    double2 acc[FDA_MAXR];
    for (int q = 0; q < FDA_MAXR; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int c = child_begin[P]; c < child_begin[P + 1]; ++c) {
        __syncthreads();
        for (int j = threadIdx.x; j < kuC; j += blockDim.x) v[j] = sCr[((int64_t)c * nslotC + cs) * kuC + j];
        __syncthreads();
        const double2 *Mo = M + ((int64_t)octant[c] * nslotP + sl) * kuP * kuC;
        for (int q = 0; q < FDA_MAXR; ++q) {
            int r = threadIdx.x + q * blockDim.x;
            if (r >= kuP) break;
            for (int j = 0; j < kuC; ++j) cfma(acc[q], Mo[r + (int64_t)j * kuP], v[j]);
        }
    }
    double2 *out = sP + (int64_t)blockIdx.y * strideP + ((int64_t)P * nslotP + sl) * kuP;
    for (int q = 0; q < FDA_MAXR; ++q) {
        int r = threadIdx.x + q * blockDim.x;
        if (r < kuP) out[r] = acc[q];
    }
}

// Reduced M2L translations grouped by translation (eq. (eq_m2l) in the
// compressed form of eq. (eq_cmpm2l)): every interaction pair with the same
// lattice offset shares one matrix K~, so each work item multiplies K~ by up
// to M2L_NB gathered source states (a small complex GEMM) and writes the
// products to a per-pair buffer.  Work items of one translation are mapped
// to the same XCD so K~ is shared through that XCD's L2.
#define M2L_NB 32
#define M2L_J 32
__global__ void __launch_bounds__(256) k_m2l_gemm(const int4 *work, const int32_t *pp_src, const double2 *K, int kd,
                                                  int ku, const double2 *s, double2 *tmp, int64_t sstride,
                                                  int64_t tstride, int nwork) {
    __shared__ double2 S[M2L_J][M2L_NB];
    // XCD-aware mapping: consecutive hardware workgroups go round-robin over
    // the 8 XCDs; give each XCD a contiguous range of work items (the grid is
    // a multiple of 8, so each XCD runs exactly `per` workgroups).
    const int nx = 8;
    const int per = gridDim.x / nx;
    const int w = (blockIdx.x % nx) * per + blockIdx.x / nx;
    if (w >= nwork) return;
    const int4 wk = work[w];  // (op, first pair, pair count, 0)
    const double2 *Kp = K + (int64_t)wk.x * kd * ku;
    const double2 *sr = s + (int64_t)blockIdx.y * sstride;
    const int p0 = wk.y, nb = wk.z;
    for (int r0 = 0; r0 < kd; r0 += blockDim.x) {
        const int r = r0 + threadIdx.x;
        double2 acc[M2L_NB];
#pragma unroll
        for (int b = 0; b < M2L_NB; ++b) acc[b] = make_double2(0.0, 0.0);
        for (int j0 = 0; j0 < ku; j0 += M2L_J) {
            __syncthreads();
            for (int e = threadIdx.x; e < M2L_J * M2L_NB; e += blockDim.x) {
                const int jj = e % M2L_J, b = e / M2L_J;
                double2 v = make_double2(0.0, 0.0);
                if (b < nb && j0 + jj < ku) v = sr[(int64_t)pp_src[p0 + b] * ku + j0 + jj];
                S[jj][b] = v;
            }
            __syncthreads();
            if (r < kd) {
                const int jm = min(M2L_J, ku - j0);
                const double2 *Kc = Kp + r + (int64_t)j0 * kd;
                for (int jj = 0; jj < jm; ++jj) {
                    const double2 a = Kc[(int64_t)jj * kd];
#pragma unroll
                    for (int b = 0; b < M2L_NB; ++b) cfma(acc[b], a, S[jj][b]);
                }
            }
        }
        if (r < kd) {
            double2 *out = tmp + (int64_t)blockIdx.y * tstride + (int64_t)p0 * kd + r;
            for (int b = 0; b < nb; ++b) out[(int64_t)b * kd] = acc[b];
        }
    }
}

// c[target] += sum of the per-pair products of the target's interaction list
// (fixed order: deterministic).
__global__ void k_m2l_reduce(const int32_t *tg_state, const int32_t *tg_off, const int32_t *tg_pairs, int kd,
                             const double2 *tmp, double2 *c, int64_t tstride, int64_t cstride) {
    const int t = blockIdx.x;
    const double2 *tr = tmp + (int64_t)blockIdx.y * tstride;
    double2 *out = c + (int64_t)blockIdx.y * cstride + (int64_t)tg_state[t] * kd;
    for (int r = threadIdx.x; r < kd; r += blockDim.x) {
        double2 acc = out[r];
        for (int q = tg_off[t]; q < tg_off[t + 1]; ++q) {
            double2 v = tr[(int64_t)tg_pairs[q] * kd + r];
            acc.x += v.x;
            acc.y += v.y;
        }
        out[r] = acc;
    }
}

// Child incoming states += L2L of the parent's incoming states.
__global__ void k_l2l(int nslotC, int kdC, const int32_t *parent, const int32_t *octant, int nslotP, int kdP,
                      const int32_t *src_off, const int32_t *src, const double2 *Lo, const double2 *cP, double2 *cC,
                      int64_t strideP, int64_t strideC) {
    extern __shared__ double2 v[];
    const int g = blockIdx.x;
    const int C = g / nslotC, cs = g - C * nslotC;
    const int P = parent[C], o = octant[C];
    const double2 *cPr = cP + (int64_t)blockIdx.y * strideP;
    double2 acc[FDA_MAXR];
    for (int q = 0; q < FDA_MAXR; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int t = src_off[cs]; t < src_off[cs + 1]; ++t) {
        const int ps = src[t];
        __syncthreads();
        for (int j = threadIdx.x; j < kdP; j += blockDim.x) v[j] = cPr[((int64_t)P * nslotP + ps) * kdP + j];
        __syncthreads();
        const double2 *Lm = Lo + ((int64_t)o * nslotP + ps) * kdC * kdP;
        for (int q = 0; q < FDA_MAXR; ++q) {
            int r = threadIdx.x + q * blockDim.x;
            if (r >= kdC) break;
            for (int j = 0; j < kdP; ++j) cfma(acc[q], Lm[r + (int64_t)j * kdC], v[j]);
        }
    }
    double2 *out = cC + (int64_t)blockIdx.y * strideC + ((int64_t)C * nslotC + cs) * kdC;
    for (int q = 0; q < FDA_MAXR; ++q) {
        int r = threadIdx.x + q * blockDim.x;
        if (r < kdC) {
            double2 ov = out[r];
            out[r] = make_double2(ov.x + acc[q].x, ov.y + acc[q].y);
        }
    }
}

// y_leaf += T~ c_leaf
__global__ void k_l2t(const int64_t *leaf_off, const double2 *Tm, int kd, const double2 *c, double2 *y, int64_t N,
                      int64_t cstride) {
    extern __shared__ double2 v[];
    const int b = blockIdx.x;
    const double2 *cr = c + (int64_t)blockIdx.y * cstride + (int64_t)b * kd;
    for (int j = threadIdx.x; j < kd; j += blockDim.x) v[j] = cr[j];
    __syncthreads();
    const int64_t e0 = leaf_off[b];
    const int nl = (int)(leaf_off[b + 1] - e0);
    const double2 *Tb = Tm + (int64_t)kd * e0;
    double2 *yr = y + (int64_t)blockIdx.y * N;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < kd; ++r) cfma(acc, Tb[i + (int64_t)r * nl], v[r]);
        double2 o = yr[e0 + i];
        yr[e0 + i] = make_double2(o.x + acc.x, o.y + acc.y);
    }
}

__global__ void k_fill_zero(double2 *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

// tree-order xt[i + c N] = x[perm[i] + c ld]
__global__ void k_permute_in(const int32_t *perm, const double2 *x, int64_t ld, double2 *xt, int64_t N) {
    const int64_t c = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        xt[i + c * N] = x[perm[i] + c * ld];
}
__global__ void k_permute_out(const int32_t *perm, const double2 *yt, int64_t N, double2 *y, int64_t ld) {
    const int64_t c = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        y[perm[i] + c * ld] = yt[i + c * N];
}

// b_i = exp(ik d.c_i) (1 + alpha i k d.n_i), written in caller order.
__global__ void k_rhs_planewave(const int32_t *perm, const double *cen, const double *nrm, const double *dirs,
                                double k, double2 alpha, double2 *b, int64_t N, int64_t ld) {
    const int64_t c = blockIdx.y;
    const double *d = dirs + 3 * c;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double ph = k * (d[0] * cen[3 * i] + d[1] * cen[3 * i + 1] + d[2] * cen[3 * i + 2]);
        double dn = d[0] * nrm[3 * i] + d[1] * nrm[3 * i + 1] + d[2] * nrm[3 * i + 2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        // 1 + alpha * (i k dn)
        double2 f = make_double2(1.0 - alpha.y * k * dn, alpha.x * k * dn);
        b[perm[i] + c * ld] = cmul(make_double2(cs, sn), f);
    }
}

// ------------------------------------------------------------ GMRES helpers
// Vectors are tree ordered, one column of length N per right-hand side;
// Krylov basis V[i] holds nrhs columns: V + (i * nrhs + c) * N.

#define RED_BLOCKS 240
#define RED_THREADS 256

// partial[(c * m + i) * RED_BLOCKS + blk] = sum over this block's range of conj(V_i,c) w_c
__global__ void k_multidot_partial(const double2 *V, int m, int nrhs, const double2 *w, int64_t N,
                                   double2 *partial) {
    __shared__ double2 red[RED_THREADS];
    const int c = blockIdx.y;
    const double2 *wc = w + (int64_t)c * N;
    for (int i = 0; i < m; ++i) {
        const double2 *vc = V + ((int64_t)i * nrhs + c) * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
            double2 a = vc[n], b = wc[n];
            acc.x += a.x * b.x + a.y * b.y;
            acc.y += a.x * b.y - a.y * b.x;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                red[threadIdx.x].x += red[threadIdx.x + s].x;
                red[threadIdx.x].y += red[threadIdx.x + s].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[((int64_t)c * m + i) * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[c * m + i] = sum_blk partial[...]
__global__ void k_multidot_final(const double2 *partial, int nblk, int total, double2 *out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) {
        acc.x += partial[(int64_t)t * nblk + b].x;
        acc.y += partial[(int64_t)t * nblk + b].y;
    }
    out[t] = acc;
}

// w_c += sign * sum_{i < m} V_i,c h[c * m + i]   (active columns only)
__global__ void k_multi_axpy(const double2 *V, int m, int nrhs, const double2 *h, double sign, double2 *w, int64_t N,
                             const int32_t *active) {
    const int c = blockIdx.y;
    if (active && !active[c]) return;
    double2 *wc = w + (int64_t)c * N;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        double2 acc = wc[n];
        for (int i = 0; i < m; ++i) {
            double2 v = V[((int64_t)i * nrhs + c) * N + n];
            double2 hh = h[c * m + i];
            acc.x += sign * (v.x * hh.x - v.y * hh.y);
            acc.y += sign * (v.x * hh.y + v.y * hh.x);
        }
        wc[n] = acc;
    }
}

// out_c = in_c * scale[c]  (complex scale per column)
__global__ void k_scale_cols(const double2 *in, const double2 *scale, double2 *out, int64_t N) {
    const int c = blockIdx.y;
    const double2 s = scale[c];
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x)
        out[(int64_t)c * N + n] = cmul(in[(int64_t)c * N + n], s);
}

// r = b - y
__global__ void k_sub(const double2 *b, const double2 *y, double2 *r, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = make_double2(b[i].x - y[i].x, b[i].y - y[i].y);
}

// ------------------------------------------------------------ block Jacobi

// In-place Gauss-Jordan inversion (partial pivoting) of each leaf's diagonal
// near block, copied from the near-field values.  One block per leaf.
__global__ void k_bj_invert(const int64_t *leaf_off, const int64_t *blk_off, const int32_t *self_col,
                            const int32_t *ncol, const double2 *vals, const int64_t *inv_off, double2 *inv) {
    __shared__ int piv[256];
    __shared__ double2 fcol[256];
    __shared__ int pr;
    const int b = blockIdx.x;
    const int n = (int)(leaf_off[b + 1] - leaf_off[b]);
    const int nc = ncol[b], sc = self_col[b];
    double2 *A = inv + inv_off[b];  // column-major n x n
    const double2 *blk = vals + blk_off[b];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        int i = idx % n, j = idx / n;
        A[i + j * n] = blk[(int64_t)i * nc + sc + j];
    }
    __syncthreads();
    for (int kk = 0; kk < n; ++kk) {
        if (threadIdx.x == 0) {
            int best = kk;
            double bv = -1;
            for (int i = kk; i < n; ++i) {
                double v = A[i + kk * n].x * A[i + kk * n].x + A[i + kk * n].y * A[i + kk * n].y;
                if (v > bv) { bv = v; best = i; }
            }
            pr = best;
            piv[kk] = best;
        }
        __syncthreads();
        const int p = pr;
        if (p != kk)
            for (int j = threadIdx.x; j < n; j += blockDim.x) {
                double2 t = A[kk + j * n];
                A[kk + j * n] = A[p + j * n];
                A[p + j * n] = t;
            }
        __syncthreads();
        double2 pv = A[kk + kk * n];
        double den = pv.x * pv.x + pv.y * pv.y;
        double2 ip = make_double2(pv.x / den, -pv.y / den);
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double2 v = (j == kk) ? make_double2(1.0, 0.0) : A[kk + j * n];
            A[kk + j * n] = cmul(v, ip);
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) fcol[i] = A[i + kk * n];
        __syncthreads();
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
            int i = idx % n, j = idx / n;
            if (i == kk) continue;
            double2 f = fcol[i];
            double2 akj = A[kk + j * n];
            double2 v = (j == kk) ? make_double2(0.0, 0.0) : A[i + j * n];
            double2 pr2 = cmul(f, akj);
            // column kk of row i becomes -f * (1/pivot) (stored in akj for j == kk)
            A[i + j * n] = make_double2(v.x - pr2.x, v.y - pr2.y);
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int kk = n - 1; kk >= 0; --kk) {
        int p = piv[kk];
        if (p != kk)
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                double2 t = A[i + kk * n];
                A[i + kk * n] = A[i + p * n];
                A[i + p * n] = t;
            }
        __syncthreads();
    }
}

// z_leaf = inv_leaf r_leaf
__global__ void k_bj_apply(const int64_t *leaf_off, const int64_t *inv_off, const double2 *inv, const double2 *r,
                           double2 *z, int64_t N, const int32_t *active) {
    extern __shared__ double2 v[];
    const int b = blockIdx.x, c = blockIdx.y;
    if (active && !active[c]) return;
    const int64_t e0 = leaf_off[b];
    const int n = (int)(leaf_off[b + 1] - e0);
    const double2 *rc = r + (int64_t)c * N + e0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = rc[i];
    __syncthreads();
    const double2 *A = inv + inv_off[b];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < n; ++j) cfma(acc, A[i + j * n], v[j]);
        z[(int64_t)c * N + e0 + i] = acc;
    }
}

// ------------------------------------------------------------ launchers

#define CHECK_LAUNCH()                                   \
    do {                                                 \
        hipError_t e_ = hipGetLastError();               \
        if (e_ != hipSuccess) return e_;                 \
    } while (0)

hipError_t set_quadrature_constants(const double r7b[7][3], const double r7w[7], const double glx[32],
                                    const double glw[32]) {
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_r7b), r7b, sizeof(double) * 21)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_r7w), r7w, sizeof(double) * 7)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_glx), glx, sizeof(double) * 32)) != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_glw), glw, sizeof(double) * 32);
}

hipError_t launch_near_blocks(const DevPlan &d, hipStream_t st) {
    if (d.nleaf == 0) return hipSuccess;
    hipLaunchKernelGGL(k_near_blocks, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_col_off, d.nf_cols,
                       d.nf_blk_off, d.tri, d.cen, d.nrm, d.area, d.k, d.alpha, d.h_max, d.nf_vals);
    CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_bj_invert(const DevPlan &d, hipStream_t st) {
    hipLaunchKernelGGL(k_bj_invert, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_blk_off, d.nf_self_col,
                       d.nf_ncol, d.nf_vals, d.bj_off, d.bj_inv);
    CHECK_LAUNCH();
    return hipSuccess;
}

static int grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 4096);
}

// Stage timings are recorded when ev != nullptr (7 events: start, after
// near, after S2M, after M2M, after M2L, after L2L, end).
hipError_t launch_matvec_tree(const DevPlan &d, const double2 *xt, double2 *yt, int nrhs, hipStream_t st,
                              hipEvent_t *ev) {
    const int64_t N = d.n;
    if (ev) hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_p2p, dim3(d.nleaf, nrhs), dim3(256), sizeof(double2) * d.max_ncol, st, d.leaf_off,
                       d.nf_list_off, d.nf_list, d.nf_blk_off, d.nf_vals, xt, yt, N);
    CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[1], st);
    if (!d.has_far) {
        for (int q = 2; q < 7 && ev; ++q) hipEventRecord(ev[q], st);
        return hipSuccess;
    }
    const int L = d.depth, top = d.top;
    const DevLevel &lf = d.lv[L];
    hipLaunchKernelGGL(k_s2m, dim3(d.nleaf, nrhs), dim3(128), sizeof(double2) * d.max_leaf, st, d.leaf_off, d.S,
                       lf.ku, xt, lf.s, N, lf.sstride);
    CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[2], st);
    for (int l = L - 1; l >= top; --l) {
        const DevLevel &P = d.lv[l], &C = d.lv[l + 1];
        hipLaunchKernelGGL(k_m2m, dim3(P.nbox * P.nslot, nrhs), dim3(256), sizeof(double2) * C.ku, st, P.nslot, P.ku,
                           P.child_begin, C.octant, C.nslot, C.ku, P.cslot, P.M, C.s, P.s, C.sstride, P.sstride);
        CHECK_LAUNCH();
    }
    if (ev) hipEventRecord(ev[3], st);
    for (int l = top; l <= L; ++l) {
        const DevLevel &lv = d.lv[l];
        int64_t n = lv.cstride * nrhs;
        hipLaunchKernelGGL(k_fill_zero, dim3(grid1(n)), dim3(256), 0, st, lv.c, n);
        CHECK_LAUNCH();
        if (lv.nwork > 0) {
            const int bs = std::min(256, ((lv.kd + 63) / 64) * 64);
            // a multiple of 8 workgroups so every XCD gets the same share
            const int grid = (lv.nwork + 7) / 8 * 8;
            hipLaunchKernelGGL(k_m2l_gemm, dim3(grid, nrhs), dim3(bs), 0, st, lv.work, lv.pp_src, lv.K, lv.kd,
                               lv.ku, lv.s, lv.tmp, lv.sstride, lv.tstride, lv.nwork);
            CHECK_LAUNCH();
            hipLaunchKernelGGL(k_m2l_reduce, dim3(lv.ntgt, nrhs), dim3(std::min(256, ((lv.kd + 63) / 64) * 64)), 0,
                               st, lv.tg_state, lv.tg_off, lv.tg_pairs, lv.kd, lv.tmp, lv.c, lv.tstride, lv.cstride);
            CHECK_LAUNCH();
        }
    }
    if (ev) hipEventRecord(ev[4], st);
    for (int l = top; l < L; ++l) {
        const DevLevel &P = d.lv[l], &C = d.lv[l + 1];
        hipLaunchKernelGGL(k_l2l, dim3(C.nbox * C.nslot, nrhs), dim3(256), sizeof(double2) * P.kd, st, C.nslot, C.kd,
                           C.parent, C.octant, P.nslot, P.kd, P.l2l_off, P.l2l_src, P.Lo, P.c, C.c, P.cstride,
                           C.cstride);
        CHECK_LAUNCH();
    }
    if (ev) hipEventRecord(ev[5], st);
    hipLaunchKernelGGL(k_l2t, dim3(d.nleaf, nrhs), dim3(64), sizeof(double2) * lf.kd, st, d.leaf_off, d.T, lf.kd,
                       lf.c, yt, N, lf.cstride);
    CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[6], st);
    return hipSuccess;
}

hipError_t launch_permute_in(const DevPlan &d, const double2 *x, int64_t ld, double2 *xt, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_in, dim3(grid1(d.n), nrhs), dim3(256), 0, st, d.perm, x, ld, xt, d.n);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_permute_out(const DevPlan &d, const double2 *yt, double2 *y, int64_t ld, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_out, dim3(grid1(d.n), nrhs), dim3(256), 0, st, d.perm, yt, d.n, y, ld);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_rhs_planewave(const DevPlan &d, const double *dirs_dev, int nrhs, double2 *b, int64_t ld,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_rhs_planewave, dim3(grid1(d.n), nrhs), dim3(256), 0, st, d.perm, d.cen, d.nrm, dirs_dev, d.k,
                       d.alpha, b, d.n, ld);
    CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_multidot(const double2 *V, int m, int nrhs, const double2 *w, int64_t N, double2 *partial,
                           double2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_multidot_partial, dim3(RED_BLOCKS, nrhs), dim3(RED_THREADS), 0, st, V, m, nrhs, w, N,
                       partial);
    CHECK_LAUNCH();
    int total = m * nrhs;
    hipLaunchKernelGGL(k_multidot_final, dim3((total + 255) / 256), dim3(256), 0, st, partial, RED_BLOCKS, total, out);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_multi_axpy(const double2 *V, int m, int nrhs, const double2 *h, double sign, double2 *w, int64_t N,
                             const int32_t *active, hipStream_t st) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(grid1(N), nrhs), dim3(256), 0, st, V, m, nrhs, h, sign, w, N, active);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_scale_cols(const double2 *in, const double2 *scale, double2 *out, int64_t N, int nrhs,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols, dim3(grid1(N), nrhs), dim3(256), 0, st, in, scale, out, N);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_sub(const double2 *b, const double2 *y, double2 *r, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_sub, dim3(grid1(n)), dim3(256), 0, st, b, y, r, n);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_bj_apply(const DevPlan &d, const double2 *r, double2 *z, int nrhs, const int32_t *active,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_bj_apply, dim3(d.nleaf, nrhs), dim3(64), sizeof(double2) * d.max_leaf, st, d.leaf_off,
                       d.bj_off, d.bj_inv, r, z, d.n, active);
    CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_fill_zero(double2 *p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_zero, dim3(grid1(n)), dim3(256), 0, st, p, n);
    CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace fda
