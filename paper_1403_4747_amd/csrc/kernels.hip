// HIP kernels of the fast directional BEM matvec and of the GMRES solver
// (gfx950).  Complex values are interleaved double2 (re, im).
//
// Matvec pipeline (Algorithm, Steps 2-4), all in element tree order:
//   near field (S2T, eq. (eq_sum)) -> leaf S2M -> M2M up the tree ->
//   M2L per level -> L2L down the tree -> leaf L2T (eq. (eq_l2t)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

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

// [G + alpha dG/dn_x](x, y): the kernel of the right-hand operator B of
// eq. (eq_bm), which acts on Neumann data (paper normal convention).
__device__ __forceinline__ double2 rhs_kernel(const double *x, const double *y, const double *nx, double k,
                                              double2 alpha) {
    double r0 = x[0] - y[0], r1 = x[1] - y[1], r2 = x[2] - y[2];
    double R = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    double2 g, gp;
    green_pair(k, R, g, gp);
    double rnx = (r0 * nx[0] + r1 * nx[1] + r2 * nx[2]) / R;
    const double2 d = cmul(alpha, make_double2(gp.x * rnx, gp.y * rnx));
    return make_double2(g.x + d.x, g.y + d.y);
}

// Near-field entry A_ij (OP 0) or B_ij (OP 1), i != j: 7-point rule on
// 4^level midpoint sub-triangles of triangle j.
template <int OP>
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
            const double2 v = OP == 0 ? lhs_kernel(x, y, nx, ny, k, alpha) : rhs_kernel(x, y, nx, k, alpha);
            double w = c_r7w[p] * asub;
            acc.x += w * v.x;
            acc.y += w * v.y;
        }
    }
    return acc;
}

// Geometry of one edge (p, q) of a flat triangle seen from an interior point
// x: d = distance from x to the edge's line, and the angles phi1 < phi2 of
// the end points measured at x from the foot of the perpendicular, as sines
// and as angles.  Along the edge R(phi) = d / cos(phi).
struct EdgeView {
    double d, sin1, sin2, phi1, phi2;
};
__device__ __forceinline__ EdgeView edge_view(const double *p, const double *q, const double *x) {
    const double ev[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    const double L = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
    const double t = ((x[0] - p[0]) * ev[0] + (x[1] - p[1]) * ev[1] + (x[2] - p[2]) * ev[2]) / L;  // foot at p + t e
    const double xp2 = (x[0] - p[0]) * (x[0] - p[0]) + (x[1] - p[1]) * (x[1] - p[1]) + (x[2] - p[2]) * (x[2] - p[2]);
    const double xq2 = (x[0] - q[0]) * (x[0] - q[0]) + (x[1] - q[1]) * (x[1] - q[1]) + (x[2] - q[2]) * (x[2] - q[2]);
    EdgeView e;
    e.d = sqrt(fmax(xp2 - t * t, 0.0));
    e.sin1 = -t / sqrt(xp2);
    e.sin2 = (L - t) / sqrt(xq2);
    e.phi1 = atan2(-t, e.d);
    e.phi2 = atan2(L - t, e.d);
    return e;
}

// Diagonal entry of A: 1/2 + alpha * (finite part of the integral of
// d2G/dn_x dn_y over the element's own flat triangle at its centroid).  On a
// flat triangle r . n = 0 and the kernel is exp(ikR)(1 - ikR)/(4 pi R^3),
// whose radial antiderivative is -exp(ikR)/(4 pi R); dropping the 1/eps of a
// small disc about the centroid leaves
//   ik/2 - (1/4pi) oint exp(ikR(theta)) / R(theta) dtheta
// over the polar angle theta.  The contour integral is split as
// exp(ikR)/R = 1/R + (exp(ikR) - 1)/R: per edge the static part is exact,
// int cos(phi)/d dphi = (sin phi2 - sin phi1)/d, and the rest,
// (-2 sin^2(kR/2) + i sin(kR))/R, is bounded by k and smooth in phi, which a
// 32-point Gauss-Legendre rule integrates.
__device__ double2 self_entry(const double *tv, const double *x, double k, double2 alpha) {
    double2 s = make_double2(0.0, 0.0);
    for (int e = 0; e < 3; ++e) {
        const EdgeView ed = edge_view(tv + 3 * e, tv + 3 * ((e + 1) % 3), x);
        s.x += (ed.sin2 - ed.sin1) / ed.d;
        const double half = 0.5 * (ed.phi2 - ed.phi1), mid = 0.5 * (ed.phi2 + ed.phi1);
        for (int g = 0; g < 32; ++g) {
            const double R = ed.d / cos(mid + half * c_glx[g]);
            const double h = sin(0.5 * k * R);
            const double w = half * c_glw[g] / R;
            s.x -= w * 2.0 * h * h;
            s.y += w * sin(k * R);
        }
    }
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
    double2 hyp = make_double2(-s.x * inv4pi, 0.5 * k - s.y * inv4pi);
    double2 ah = cmul(alpha, hyp);
    return make_double2(0.5 + ah.x, ah.y);
}

// Diagonal entry of B: -alpha/2 + int G over the element's own flat
// triangle at its centroid (the alpha dG/dn_x part vanishes there, r . n_x
// = 0).  In polar coordinates about the centroid the radial integral of
// exp(ikR)/(4 pi R) R dR is exact, so
//   int G = (i / (4 pi k)) oint (1 - exp(ik R(theta))) dtheta,
// with 1 - exp(ikR) = 2 sin^2(kR/2) - i sin(kR), integrated edge by edge with
// 32-point Gauss-Legendre in phi.
__device__ double2 self_entry_rhs(const double *tv, const double *x, double k, double2 alpha) {
    double2 s = make_double2(0.0, 0.0);
    for (int e = 0; e < 3; ++e) {
        const EdgeView ed = edge_view(tv + 3 * e, tv + 3 * ((e + 1) % 3), x);
        const double half = 0.5 * (ed.phi2 - ed.phi1), mid = 0.5 * (ed.phi2 + ed.phi1);
        for (int g = 0; g < 32; ++g) {
            const double R = ed.d / cos(mid + half * c_glx[g]);
            const double h = sin(0.5 * k * R);
            const double w = half * c_glw[g];
            s.x += w * 2.0 * h * h;
            s.y -= w * sin(k * R);
        }
    }
    const double c = 1.0 / (4.0 * 3.14159265358979323846 * k);  // i c s = (-c s.y, c s.x)
    return make_double2(-c * s.y - 0.5 * alpha.x, c * s.x - 0.5 * alpha.y);
}

template <int OP>
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
            v = OP == 0 ? self_entry(tri + 9 * tj, x, k, alpha) : self_entry_rhs(tri + 9 * tj, x, k, alpha);
        } else {
            const double *cj = cen + 3 * tj;
            double dd = sqrt((x[0] - cj[0]) * (x[0] - cj[0]) + (x[1] - cj[1]) * (x[1] - cj[1]) +
                             (x[2] - cj[2]) * (x[2] - cj[2]));
            int level = (dd < h) ? 3 : (dd < 1.75 * h) ? 2 : (dd < 2.5 * h) ? 1 : 0;
            v = near_entry<OP>(tri + 9 * tj, area[tj], x, nrm + 3 * ti, nrm + 3 * tj, k, alpha, level);
        }
        blk[idx] = v;
    }
}

// ------------------------------------------------------------ matvec
//
// The matvec kernels are templates over the storage type of the operators
// and states: double2 (FP64 plan) or float2 (FP32 plan: M2L, M2M, L2L, S2M,
// L2T and the off-diagonal near field stored in FP32 with FP32 accumulation;
// the element self terms and every vector the caller sees stay FP64).  The
// dense contractions (M2M, M2L, L2L) run on the matrix cores (FP64 or FP32
// MFMA); the near field, S2M and L2T stream their precomputed operators from
// HBM once per product and are scalar FMA loops.

template <class C>
struct CT;
template <>
struct CT<double2> {
    using R = double;
    typedef double v2 __attribute__((ext_vector_type(2)));
    typedef double v4 __attribute__((ext_vector_type(4)));
    // v_mfma_f64_16x16x4f64; result row of lane group lk, element v
    static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct CT<float2> {
    using R = float;
    typedef float v2 __attribute__((ext_vector_type(2)));
    typedef float v4 __attribute__((ext_vector_type(4)));
    // v_mfma_f32_16x16x4f32
    static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// Load of one complex value from global memory.  A pointer read out of a
// device-side table is generic to the compiler, which then emits flat loads;
// those count against the LDS wait counter as well, so every wait for an LDS
// read would also wait for all loads in flight.  Reading through a
// global-space pointer keeps the two counters apart.
template <class C>
__device__ __forceinline__ C gload(const C *p) {
    using v2 = typename CT<C>::v2;
    const v2 v = *(const __attribute__((address_space(1))) v2 *)p;
    C c;
    c.x = v.x;
    c.y = v.y;
    return c;
}

template <class C>
__device__ __forceinline__ C czero() {
    C z;
    z.x = 0;
    z.y = 0;
    return z;
}
template <class C>
__device__ __forceinline__ C cfrom(double2 v) {
    C z;
    z.x = (typename CT<C>::R)v.x;
    z.y = (typename CT<C>::R)v.y;
    return z;
}
template <class C>
__device__ __forceinline__ void cmac(C &acc, C a, C b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// Block order of a product over nrhs right-hand sides (a 1-D grid of
// rhs_grid(n, nrhs) workgroups for n work items): workgroup b runs on XCD
// b % 8 (round-robin dispatch), and the blocks of one work item for every
// right-hand side follow each other on that XCD, so the item's operator is
// read from HBM once and from the XCD's L2 for the other columns.  Items
// t * 8 + x go to XCD x; with one right-hand side block b takes item b.
struct RhsBlock {
    int item, rhs;
};
__device__ __forceinline__ RhsBlock rhs_block(int nrhs) {
    const int b = blockIdx.x, x = b & 7, j = b >> 3;
    const int t = j / nrhs;
    return {t * 8 + x, j - t * nrhs};
}
// The same order for work lists cut into one contiguous chunk of `per`
// items per XCD (item x * per + t on XCD x).
__device__ __forceinline__ RhsBlock rhs_block_chunked(int nrhs, int per) {
    const int b = blockIdx.x, x = b & 7, j = b >> 3;
    const int t = j / nrhs;
    return {x * per + t, j - t * nrhs};
}
// The same grid taken in groups of G right-hand sides: every item of the
// XCD's queue (nq items) for the group's columns, then the next group, so
// that the states gathered for one group's columns stay in the caches
// while the group runs (G >= nrhs: the order of rhs_block).
__device__ __forceinline__ RhsBlock rhs_block_grouped(int nrhs, int nq, int G) {
    const int b = blockIdx.x, x = b & 7, j = b >> 3;
    const int g = j / (nq * G), rem = j - g * nq * G;
    const int gg = min(G, nrhs - g * G);
    const int t = rem / gg;
    return {t * 8 + x, g * G + (rem - t * gg)};
}
// rhs_block_chunked taken in groups of G right-hand sides (every item of the
// XCD's chunk for the group's columns, then the next group).
__device__ __forceinline__ RhsBlock rhs_block_chunked_grouped(int nrhs, int per, int G) {
    const int b = blockIdx.x, x = b & 7, j = b >> 3;
    const int g = j / (per * G), rem = j - g * per * G;
    const int gg = min(G, nrhs - g * G);
    const int t = rem / gg;
    return {x * per + t, g * G + (rem - t * gg)};
}
static inline dim3 rhs_grid(int64_t n, int nrhs) { return dim3((unsigned)(((n + 7) / 8) * 8 * nrhs)); }

// Near field, S2M and L2T take R right-hand sides per workgroup (the
// columns r0 .. r0 + R - 1 of group g = r0 / R): every operator entry is
// read once and applied to the group's columns, which are staged in LDS as
// R rows (no bank conflicts between lanes of one column index).  Each
// column is summed in the same order whatever R, so a product of several
// columns equals the single-column products bit for bit.

// Row sum of a wave's partial products (lane 0 ends with the total).
template <class C>
__device__ __forceinline__ C wave_sum(C acc) {
    for (int o = 32; o > 0; o >>= 1) {
        acc.x += __shfl_down(acc.x, o, 64);
        acc.y += __shfl_down(acc.y, o, 64);
    }
    return acc;
}

// Sum over the kP2PGroup lanes of a row group (the group's first lane ends
// with the total); every lane of the wave takes part.
template <class C>
__device__ __forceinline__ C group_sum(C acc) {
    for (int o = kP2PGroup / 2; o > 0; o >>= 1) {
        acc.x += __shfl_down(acc.x, o, kP2PGroup);
        acc.y += __shfl_down(acc.y, o, kP2PGroup);
    }
    return acc;
}

// y_tree[i] = sum over the near leaves of the block entries times x
// (+ the FP64 self term diag[i] x[i] when the blocks are FP32).  x of the
// block's columns (listed in cols from col_off[leaf], the near leaves'
// elements in order) is gathered into LDS in one parallel pass.  A row is
// taken by a group of kP2PGroup lanes (four rows per wave, sixteen per
// workgroup), each lane summing the columns lane, lane + kP2PGroup, ... in
// order, with kP2PUnroll row loads in flight: rows are a few hundred
// columns long, so full-wave rows would leave lanes idle in their last
// chunk and wait on one load at a time.
template <class C, int R>
__global__ void __launch_bounds__(256) k_p2p(const int4 *items, const int64_t *leaf_off, const int64_t *col_off,
                                             const int32_t *cols, const int64_t *blk_off, const C *vals,
                                             const double2 *diag, const double2 *x, double2 *y, int64_t N,
                                             int nitems, int ngroups, int nrhs) {
    constexpr int G = kP2PGroup;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *xs = (C *)smem_raw;  // R x nc
    const RhsBlock rb = rhs_block(ngroups);
    if (rb.item >= nitems) return;
    const int r0 = rb.rhs * R, nr = min(R, nrhs - r0);
    const int4 it = items[rb.item];  // (leaf, first row, end row, -)
    const int b = it.x;
    const int64_t c0 = col_off[b];
    const int nc = (int)(col_off[b + 1] - c0);
    const int32_t *cl = cols + c0;
    for (int e = threadIdx.x; e < R * nc; e += blockDim.x) {
        const int r = e / nc, c = e - r * nc;
        xs[e] = r < nr ? cfrom<C>(x[(int64_t)(r0 + r) * N + cl[c]]) : czero<C>();
    }
    __syncthreads();
    const int64_t t0 = leaf_off[b];
    const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G, ngrp = blockDim.x / G;
    const C *blk = vals + blk_off[b];
    for (int i0 = it.y; i0 < it.z; i0 += ngrp) {  // the same trip count for every lane
        const int i = i0 + grp;
        C acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = czero<C>();
        if (i < it.z) {
            const C *row = blk + (int64_t)i * nc;
            int c = lane;
            constexpr int U = kP2PUnroll;
            for (; c + (U - 1) * G < nc; c += U * G) {
                C v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = row[c + u * G];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const C *xr = xs + r * nc + c;
#pragma unroll
                    for (int u = 0; u < U; ++u) cmac(acc[r], v[u], xr[u * G]);
                }
            }
            for (; c < nc; c += G) {
                const C v = row[c];
#pragma unroll
                for (int r = 0; r < R; ++r) cmac(acc[r], v, xs[r * nc + c]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] = group_sum(acc[r]);
            if (i < it.z && lane == 0 && r < nr) {
                double2 out = make_double2((double)acc[r].x, (double)acc[r].y);
                if (diag) {
                    const double2 d = diag[t0 + i], v = x[(int64_t)(r0 + r) * N + t0 + i];
                    out.x += d.x * v.x - d.y * v.y;
                    out.y += d.x * v.y + d.y * v.x;
                }
                y[(int64_t)(r0 + r) * N + t0 + i] = out;
            }
        }
    }
}

// The same product for long rows (more than kP2PShortCols columns): x is
// read through the row's column list instead of being staged in LDS, so
// these workgroups need no LDS and keep full occupancy (x is small enough
// to stay in L2); a full wave per row.
template <class C, int R>
__global__ void __launch_bounds__(256) k_p2p_direct(const int4 *items, const int64_t *leaf_off,
                                                    const int64_t *col_off, const int32_t *cols,
                                                    const int64_t *blk_off, const C *vals, const double2 *diag,
                                                    const double2 *x, double2 *y, int64_t N, int nitems,
                                                    int ngroups, int nrhs) {
    const RhsBlock rb = rhs_block(ngroups);
    if (rb.item >= nitems) return;
    const int r0 = rb.rhs * R, nr = min(R, nrhs - r0);
    const int4 it = items[rb.item];  // (leaf, first row, end row, -)
    const int b = it.x;
    const int64_t c0 = col_off[b];
    const int nc = (int)(col_off[b + 1] - c0);
    const int32_t *cl = cols + c0;
    const int64_t t0 = leaf_off[b];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const C *blk = vals + blk_off[b];
    for (int i = it.y + wv; i < it.z; i += nw) {
        C acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = czero<C>();
        const C *row = blk + (int64_t)i * nc;
        for (int c = lane; c < nc; c += 64) {
            const C v = row[c];
            const int64_t j = cl[c];
#pragma unroll
            for (int r = 0; r < R; ++r)
                cmac(acc[r], v, r < nr ? cfrom<C>(x[(int64_t)(r0 + r) * N + j]) : czero<C>());
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] = wave_sum(acc[r]);
            if (lane == 0 && r < nr) {
                double2 out = make_double2((double)acc[r].x, (double)acc[r].y);
                if (diag) {
                    const double2 d = diag[t0 + i], v = x[(int64_t)(r0 + r) * N + t0 + i];
                    out.x += d.x * v.x - d.y * v.y;
                    out.y += d.x * v.y + d.y * v.x;
                }
                y[(int64_t)(r0 + r) * N + t0 + i] = out;
            }
        }
    }
}

// s_leaf = S~ x_leaf, for the leaves of one level (ids: global leaf ids,
// box: their boxes on the level, sop: offset of each leaf's S~), R
// right-hand sides per workgroup.
template <class C, int R>
__global__ void k_s2m(const int64_t *leaf_off, const int32_t *ids, const int32_t *box, const int64_t *sop,
                      const C *S, int ku, const double2 *x, C *s, int64_t N, int64_t sstride, int nleaves,
                      int ngroups, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *xs = (C *)smem_raw;  // R x nl
    const RhsBlock rb = rhs_block(ngroups);
    if (rb.item >= nleaves) return;
    const int r0 = rb.rhs * R, nr = min(R, nrhs - r0);
    const int b = ids[rb.item];
    const int64_t e0 = leaf_off[b];
    const int nl = (int)(leaf_off[b + 1] - e0);
    for (int e = threadIdx.x; e < R * nl; e += blockDim.x) {
        const int r = e / nl, j = e - r * nl;
        xs[e] = r < nr ? cfrom<C>(x[(int64_t)(r0 + r) * N + e0 + j]) : czero<C>();
    }
    __syncthreads();
    const C *Sb = S + sop[b];
    const int64_t so = (int64_t)box[rb.item] * ku;
    for (int row = threadIdx.x; row < ku; row += blockDim.x) {
        C acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = czero<C>();
        for (int j = 0; j < nl; ++j) {
            const C v = Sb[row + (int64_t)j * ku];
#pragma unroll
            for (int r = 0; r < R; ++r) cmac(acc[r], v, xs[r * nl + j]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < nr) s[(int64_t)(r0 + r) * sstride + so + row] = acc[r];
    }
}

// Gathered batched GEMM shared by M2M, M2L and L2L, on the matrix cores.  A
// work item multiplies one translation matrix (m x kin, column-major) by up
// to GG_NB gathered input states and writes the m-vectors to consecutive
// columns of a scratch buffer:
//   T[:, tcol + b] = A[mat] X[src[b]]   (src = -1: zero column).
//   M2L: one matrix per distinct translation (eq. (eq_m2l) compressed by
//        eq. (eq_cmpm2l)), columns = the interaction pairs sharing it.
//   M2M: one matrix per (child octant, direction) (Section 4.3), columns =
//        the parents with a child in that octant.
//   L2L: one matrix per (child octant, parent direction), columns = the
//        children in that octant.
// A second kernel sums the scratch columns of every destination state in a
// fixed order (deterministic results).  Where every destination receives a
// single product (L2L between non-directional levels: one parent each), the
// product is added to it in place and the scratch and the second kernel
// are skipped.
// MFMA operand layout per wave (16x16x4, FP64 and FP32): A (16 x 4) lane l
// holds row l % 16, column l / 16; B (4 x 16) lane l holds row l / 16, column
// l % 16; the 16 x 16 result of lane l is column l % 16, rows CT<C>::row.  A
// complex product is taken as three real products (CAcc).  The 4 waves of a
// block take row tiles w, w + 4, ... of a band of 64 or 128 rows
// (GemmShape).  Work items of consecutive index are mapped to the same XCD
// so that the shared translation matrices stay in that XCD's L2.
#define GG_NB 32
#define GG_LD (GG_NB + 1)  // padded LDS row: spreads the 4 k-rows of an MFMA operand over the banks
#define MF_RT 4
#define LR_MAX 72
#define LR_LD (LR_MAX + 1)
#ifndef LRJ
#define LRJ 16  // k-chunk of the low-rank M2L phase 1
#endif
#define LR_P2 1  // row tiles per wave and pass in phase 2
#ifndef FDA_M2L_WAVES64
#define FDA_M2L_WAVES64 4  // k_m2l_lowrank<double2> waves per SIMD
#endif
// Variants of the low-rank M2L kernel (chosen per plan, fda_autotune):
// k-steps in flight in the register rings of phase 1 (direct form; waves
// with two / one row tiles) and of phase 2.  Every variant runs at 4 FP64
// waves per SIMD without spills and gives bit-identical results.
template <int VAR>
struct M2LVariant;
template <>
struct M2LVariant<0> {
    static constexpr int p1d = 4, p1d1 = 4, pd = 5;
};
template <>
struct M2LVariant<1> {
    static constexpr int p1d = 2, p1d1 = 4, pd = 2;
};
template <>
struct M2LVariant<2> {
    static constexpr int p1d = 4, p1d1 = 6, pd = 6;
};
template <>
struct M2LVariant<3> {
    static constexpr int p1d = 3, p1d1 = 4, pd = 3;
};
static_assert(kM2LVariants == 4, "one M2LVariant per variant index");

// Complex accumulator of one 16 x 16 output tile on the matrix cores, in the
// three-product form (Gauss): P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
// then Re = P1 - P2 and Im = P3 - P1 - P2 (three MFMAs per complex k-step
// instead of four).  Independent accumulators keep consecutive MFMAs from
// waiting on each other.
template <class C>
struct CAcc {
    using v4 = typename CT<C>::v4;
    using R = typename CT<C>::R;
    v4 p1, p2, p3;
    __device__ __forceinline__ void zero() {
        p1 = (v4){0, 0, 0, 0};
        p2 = (v4){0, 0, 0, 0};
        p3 = (v4){0, 0, 0, 0};
    }
    __device__ __forceinline__ void mac(C a, C b) {
        p1 = CT<C>::mfma(a.x, b.x, p1);
        p2 = CT<C>::mfma(a.y, b.y, p2);
        p3 = CT<C>::mfma(a.x + a.y, b.x + b.y, p3);
    }
    __device__ __forceinline__ R re(int v) const { return p1[v] - p2[v]; }
    __device__ __forceinline__ R im(int v) const { return p3[v] - p1[v] - p2[v]; }
};

// Gathered GEMM body: every GG_SJ-deep k-chunk of a band of 64 RT rows of A
// is staged in LDS beside the chunk of the NB gathered states, and the next
// chunk of both is fetched into registers while the current one is
// multiplied (the MFMA loop reads only LDS).  NCT column tiles of 16 are
// live (the item's column count rounded up).  Column col of the product
// goes to scratch column col (Tr, m rows per column) or, when the item
// lists destination states (sdst), is written (accumulate: added) to state
// sdst[col] of Yr, the only contribution that state receives.
#ifndef GG_SJ
#define GG_SJ 8  // k-chunk of the staged form
#endif
template <class C, int NCT, int RT>
__device__ __forceinline__ void ggemm_body_staged(const int4 h, const int32_t *sidx, const int32_t *sdst,
                                                  const C *At, int m, int kin, const C *Xr, C *Tr, C *Yr,
                                                  int accumulate, int band0, int band1, C (*S)[GG_LD],
                                                  C (*As)[64 * RT + 1]) {
    constexpr int SB = 64 * RT;  // rows per band
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    constexpr int SPT = GG_SJ * GG_NB / 256;
    constexpr int APT = SB * GG_SJ / 256;
    for (int band = band0; band < band1; band += SB) {
        const int ntile = min(RT * 4, (m - band + 15) >> 4);
        const int nrow = min(SB, m - band);
        CAcc<C> acc[RT][NCT];
#pragma unroll
        for (int q = 0; q < RT; ++q)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[q][c].zero();
        C sreg[SPT], areg[APT];
        auto fetch = [&](int j0) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                const int jj = e % GG_SJ, b = e / GG_SJ;
                const int sb = sidx[b];
                sreg[i] = czero<C>();
                if (sb >= 0 && j0 + jj < kin) sreg[i] = Xr[(int64_t)sb * kin + j0 + jj];
            }
#pragma unroll
            for (int i = 0; i < APT; ++i) {
                const int e = threadIdx.x + 256 * i;
                const int row = e % SB, kc = e / SB;
                areg[i] = czero<C>();
                if (row < nrow && j0 + kc < kin) areg[i] = At[band + row + (int64_t)(j0 + kc) * m];
            }
        };
        __syncthreads();  // sidx, and the previous band's last chunk is consumed
        fetch(0);
        for (int j0 = 0; j0 < kin; j0 += GG_SJ) {
            __syncthreads();  // the previous chunk is consumed
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                S[e % GG_SJ][e / GG_SJ] = sreg[i];
            }
#pragma unroll
            for (int i = 0; i < APT; ++i) {
                const int e = threadIdx.x + 256 * i;
                As[e / SB][e % SB] = areg[i];
            }
            __syncthreads();
            if (j0 + GG_SJ < kin) fetch(j0 + GG_SJ);
            const int jm = min(GG_SJ, kin - j0);
            for (int kk = 0; kk < jm; kk += 4) {
                C bv[NCT];
#pragma unroll
                for (int c = 0; c < NCT; ++c) bv[c] = S[kk + lk][c * 16 + li];
#pragma unroll
                for (int q = 0; q < RT; ++q) {
                    const int rt = wave + 4 * q;
                    if (rt >= ntile) break;
                    const C av = As[kk + lk][rt * 16 + li];
#pragma unroll
                    for (int c = 0; c < NCT; ++c) acc[q][c].mac(av, bv[c]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const int rt = wave + 4 * q;
            if (rt >= ntile) break;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const int col = c * 16 + li;
                if (col >= h.z) continue;
                C *o = sdst ? Yr + (int64_t)sdst[col] * m : Tr + (int64_t)col * m;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = band + rt * 16 + CT<C>::row(lk, v);
                    if (row < m) {
                        C r;
                        r.x = acc[q][c].re(v);
                        r.y = acc[q][c].im(v);
                        if (sdst && accumulate) {
                            const C old = o[row];
                            r.x = old.x + r.x;
                            r.y = old.y + r.y;
                        }
                        o[row] = r;
                    }
                }
            }
        }
    }
}


#ifndef FDA_GEMM_ZGROUP
#define FDA_GEMM_ZGROUP 16  // right-hand sides per group of the gathered GEMM's block order
#endif
// Waves per SIMD the GEMM kernels are compiled for: FP64 needs more
// registers per complex accumulator than FP32.
#ifndef FDA_GEMM_WAVES64
#define FDA_GEMM_WAVES64 3
#endif
template <class C>
struct GemmOcc {
    static constexpr int waves = FDA_GEMM_WAVES64;
};
template <class C>
struct M2LOcc {
    static constexpr int waves = FDA_M2L_WAVES64;
    static constexpr bool direct = true;  // phase 1: operands straight into registers (no LDS staging)
};
template <>
struct M2LOcc<float2> {
    static constexpr int waves = 4;
    static constexpr bool direct = false;  // phase 1 staged through LDS (the direct form is slower in FP32)
};
#ifndef FDA_GEMM_WAVES32
#define FDA_GEMM_WAVES32 3
#endif
template <>
struct GemmOcc<float2> {
    static constexpr int waves = FDA_GEMM_WAVES32;
};

// Shape of the gathered GEMM per storage type.  FP64 accumulators take
// twice the registers of FP32 ones, so an FP64 wave keeps one 16-row tile
// (64-row bands) and every band of an item is a workgroup of its own (more
// workgroups for the few, tall items of the upper levels; measured at
// N = 81,920, kD = 100: M2M 0.242 -> 0.225 ms, L2L 0.272 -> 0.252 ms); an
// FP32 wave keeps two tiles (128-row bands) and a workgroup loops over the
// bands of its item (splitting was slower there: L2L 0.181 -> 0.213 ms).
template <class C>
struct GemmShape {
    static constexpr int rt = 1;
    static constexpr bool band_split = true;
};
template <>
struct GemmShape<float2> {
    static constexpr int rt = 2;
    static constexpr bool band_split = false;
};

// One work item per workgroup (or one band of 64 RT rows of an item):
// matrix hdr.x times the item's gathered states, into scratch columns
// hdr.y .. or, with dst, straight into the listed destination states of Y.
template <class C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GemmOcc<C>::waves)))
k_ggemm(const int4 *hdr, const int32_t *src, const int32_t *dst, const C *A, int m, int kin, const C *X,
        int64_t xstride, C *T, int64_t tstride, C *Y, int64_t ystride, int accumulate, int nwork, int nband,
        int nrhs) {
    constexpr int RT = GemmShape<C>::rt;
    constexpr int SB = 64 * RT;
    __shared__ C S[GG_SJ][GG_LD];
    __shared__ C As[GG_SJ][SB + 1];
    __shared__ int32_t sidx[GG_NB], sdst[GG_NB];
    // one contiguous chunk of the work list per XCD (consecutive items
    // share their translation matrix; the bands of an item are consecutive)
    const int nunit = nwork * nband;
    const RhsBlock rb = rhs_block_chunked_grouped(nrhs, (nunit + 7) / 8, FDA_GEMM_ZGROUP);
    if (rb.item >= nunit) return;
    const int w = rb.item / nband, bnd = rb.item - w * nband;
    const int band0 = nband == 1 ? 0 : bnd * SB, band1 = nband == 1 ? m : min(m, band0 + SB);
    const int4 h = hdr[w];  // (matrix, first scratch column, column count, 0)
    if (threadIdx.x < GG_NB) {
        sidx[threadIdx.x] = src[(int64_t)w * GG_NB + threadIdx.x];
        if (dst) sdst[threadIdx.x] = dst[(int64_t)w * GG_NB + threadIdx.x];
    }
    const C *Xr = X + (int64_t)rb.rhs * xstride;
    C *Tr = dst ? nullptr : T + (int64_t)rb.rhs * tstride + (int64_t)h.y * m;
    C *Yr = dst ? Y + (int64_t)rb.rhs * ystride : nullptr;
    const int32_t *sd = dst ? sdst : nullptr;
    const C *At = A + (int64_t)h.x * m * kin;
    if (h.z > 16)
        ggemm_body_staged<C, 2, RT>(h, sidx, sd, At, m, kin, Xr, Tr, Yr, accumulate, band0, band1, S, As);
    else
        ggemm_body_staged<C, 1, RT>(h, sidx, sd, At, m, kin, Xr, Tr, Yr, accumulate, band0, band1, S, As);
}

// The destination-major kernels (k_ggemm_dest, k_m2l_dest): k-steps in
// flight in the register ring, largest column-tile count per wave, and
// waves per SIMD (FP64 keeps 96 accumulator registers at 64 columns).
#ifndef FDA_M2L_DEST_PD
#define FDA_M2L_DEST_PD 4
#endif
#ifndef FDA_M2L_DEST_NCT
#define FDA_M2L_DEST_NCT 4
#endif
template <class C>
struct M2LDestOcc {
    static constexpr int waves = 2;
};
template <>
struct M2LDestOcc<float2> {
    static constexpr int waves = 4;
};

// The gathered GEMM of a list with a reduction, destination-major, for many
// right-hand sides: y_t (+)= sum over the entries (matrix a, source s) of
// destination t of A_a x_s, accumulated on the matrix cores across the
// entries in list order and written once (no scratch columns, no
// reduction launch).  Wave w of workgroup b owns unit 4 b + w, one
// (destination, 16-row tile), and columns 16 NCT blockIdx.y ..; its k loop
// runs over the entries, kin / 4 steps each (rounded up: the lanes past kin
// load a clamped element and multiply it by a zero A fragment), with the A
// and x fragments loaded PD steps ahead as in k_m2l_dest.
template <class C, int NCT, int PD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M2LDestOcc<C>::waves)))
k_ggemm_dest(const int2 *units, int nunits, const int2 *ent, const int32_t *off, const int32_t *dstl, const C *A,
             int m, int kin, const C *X, int64_t xstride, C *Y, int64_t ystride, int accumulate, int nrhs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int u = (int)blockIdx.x * 4 + wave;
    if (u >= nunits) return;
    const int2 un = units[u];  // (destination entry, row tile)
    const int t = un.x, rt = un.y;
    const int c0 = (int)blockIdx.y * 16 * NCT;
    const int64_t mk = (int64_t)m * kin;
    const int arow = min(rt * 16 + li, m - 1);
    int64_t bo[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) bo[c] = (int64_t)min(c0 + c * 16 + li, nrhs - 1) * xstride;
    CAcc<C> acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c].zero();
    const int ks = (kin + 3) >> 2;  // k-steps per entry
    const int e0 = off[t], last = off[t + 1] - 1;
    const int ns = (last - e0 + 1) * ks;
    if (ns > 0) {
        int fe = e0, fk = 0;
        int2 en = ent[fe];  // (matrix, source state)
        int2 nx = ent[min(fe + 1, last)];
        const C *fa = A + en.x * mk + arow;
        const C *fb = X + (int64_t)en.y * kin;
        auto fetch = [&](C &a, C (&b)[NCT], bool &live) {
            const int k = 4 * fk + lk;
            live = k < kin;
            const int kc = min(k, kin - 1);
            a = gload(fa + (int64_t)kc * m);
#pragma unroll
            for (int c = 0; c < NCT; ++c) b[c] = gload(fb + bo[c] + kc);
            if (++fk == ks) {
                if (fe < last) {
                    ++fe;
                    en = nx;
                    nx = ent[min(fe + 1, last)];
                    fk = 0;
                    fa = A + en.x * mk + arow;
                    fb = X + (int64_t)en.y * kin;
                } else {
                    fk = ks - 1;
                }
            }
        };
        auto use = [&](const C &a, const C (&b)[NCT], bool live) {
            const C av = live ? a : czero<C>();
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[c].mac(av, b[c]);
        };
        C ar[PD], br[PD][NCT];
        bool lv[PD];
#pragma unroll
        for (int d = 0; d < PD; ++d) fetch(ar[d], br[d], lv[d]);
        int s = 0;
        for (; s + PD <= ns; s += PD) {
#pragma unroll
            for (int d = 0; d < PD; ++d) {
                use(ar[d], br[d], lv[d]);
                fetch(ar[d], br[d], lv[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < PD; ++d)
            if (s + d < ns) use(ar[d], br[d], lv[d]);
    }
    C *yt = Y + (int64_t)dstl[t] * m;
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
        const int col = c0 + c * 16 + li;
        if (col >= nrhs) continue;
        C *o = yt + (int64_t)col * ystride;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = rt * 16 + CT<C>::row(lk, v);
            if (row < m) {
                C y;
                y.x = acc[c].re(v);
                y.y = acc[c].im(v);
                if (accumulate) {
                    const C old = o[row];
                    y.x = old.x + y.x;
                    y.y = old.y + y.y;
                }
                o[row] = y;
            }
        }
    }
}

// Phase 1 of the low-rank M2L in the direct form: NQ row tiles of V^ (rows
// vrow[q]) times one column tile of gathered states (column xcol), k-steps
// kb0, kb0 + kstep, ... below ku.  Operands are loaded PD steps ahead into a
// ring of registers; the main loop issues exactly PD loads per trip and the
// tail none, so the waits count loads instead of draining them.
template <class C, int NQ, int PD>
__device__ __forceinline__ void m2l_p1_direct(CAcc<C> *zacc, const C *xcol, const C *const *vrow, int rmax,
                                              int ku, int kb0, int kstep, int lk) {
    const int ku4 = (ku + 3) & ~3;
    auto fetch = [&](C (&av)[NQ], C &bv, int kc) {
        bv = gload(xcol + min(kc, ku - 1));
        const int64_t vc = (int64_t)min(kc, ku4 - 1) * rmax;
#pragma unroll
        for (int q = 0; q < NQ; ++q) av[q] = gload(vrow[q] + vc);
    };
    C ar[PD][NQ], br[PD];
#pragma unroll
    for (int d = 0; d < PD; ++d) fetch(ar[d], br[d], kb0 + d * kstep + lk);
    const int nsteps = kb0 < ku ? (ku - kb0 + kstep - 1) / kstep : 0;
    int s = 0;
    for (; s + PD <= nsteps; s += PD) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) zacc[q].mac(ar[d][q], br[d]);
            fetch(ar[d], br[d], kb0 + (s + d + PD) * kstep + lk);  // slot d now holds step s + d + PD
        }
    }
#pragma unroll
    for (int d = 0; d < PD; ++d)
        if (s + d < nsteps) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) zacc[q].mac(ar[d][q], br[d]);
        }
}

// Low-rank reduced M2L (Section 4.2, eq. (eq_epsk)): K~ = U^ V^ with rank r
// per translation, so each work item first forms Z = V^ S (r x ncols) and
// then U^ Z (kd x ncols), both on the matrix cores; Z stays in LDS.  Same
// work list, scratch layout and reduction as k_ggemm.  Phase 1 spreads its
// (row tile, column tile) outputs over the 4 waves round-robin so that the
// usual ranks (r <= 32, two column tiles: four tiles) keep every wave busy.
//
// ZOUT (the many-column form): the item stores rows 0 .. r - 1 of Z, column
// col at Tr + col * ldt, and skips phase 2.
template <class C, int NCT, int P1D, int P1D1, int PD, bool ZOUT>
__device__ __forceinline__ void m2l_body(const int4 h, const int32_t *sidx, const C *Ut, const C *Vt, int r, int kd,
                                         int ku, int rmax, const C *Xr, C *Tr, int ldt, C (*S)[GG_LD],
                                         C (*Vs)[LR_LD], C (*Z)[GG_LD]) {
    using v4 = typename CT<C>::v4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // phase 1: Z = V^[0:r, :] S; tile ti = wave + 4 q is (row tile ti / NCT,
    // column tile ti % NCT).  Each k-chunk of V^ is staged in LDS next to the
    // chunk of gathered states, so the MFMA loop reads only LDS.
    const int ztiles = (r + 15) >> 4;
    const int ntz = ztiles * NCT;
    constexpr int ZQ = 2;  // tiles per wave: ntz <= 8 (the host gives ranks above 64 16-column items)
    // With fewer than 4 output tiles the waves also split the k-steps
    // (kg_n groups; wave = kg * ntz + tile) and the partial products are
    // summed in LDS afterwards.
    const int kg_n = ntz == 1 ? 4 : (ntz == 2 ? 2 : 1);
    const int kg = kg_n > 1 ? wave / ntz : 0;
    const int tbase = kg_n > 1 ? wave % ntz : wave;
    const int tstep = kg_n > 1 ? 64 : 4;  // kg_n > 1: one tile per wave
    CAcc<C> zacc[ZQ];
#pragma unroll
    for (int q = 0; q < ZQ; ++q) zacc[q].zero();
    if constexpr (M2LOcc<C>::direct) {
        // Every wave multiplies its own tiles with operands loaded straight from
        // memory into MFMA registers, P1D (P1D1) k-steps ahead of their use: the
        // V^ rows of its row tiles and the gathered state columns of its column
        // tile (all tiles of a wave share one column tile: the tile stride is 4
        // and NCT divides 4).  No LDS staging and no barriers in the k loop.
        __syncthreads();  // sidx
        if (tbase < ntz) {
            // Every load is unconditional (a skipped load would make the
            // compiler wait for all loads in flight): addresses are clamped
            // into the operands instead.  A padding column (no source) reads
            // state 0, and its products are never stored; rows of V^ from r
            // on are zero up to rmax and the Z rows they give are never read;
            // the columns of V^ from ku to ku4 are zero, so the clamped state
            // element they meet adds nothing.
            const int sb = sidx[(tbase % NCT) * 16 + li];
            const C *xcol = Xr + (int64_t)(sb >= 0 ? sb : 0) * ku;
            const C *vrow[ZQ];
#pragma unroll
            for (int q = 0; q < ZQ; ++q) vrow[q] = Vt + min(((tbase + tstep * q) / NCT) * 16 + li, rmax - 1);
            if (tbase + tstep < ntz)
                m2l_p1_direct<C, 2, P1D>(zacc, xcol, vrow, rmax, ku, 4 * kg, 4 * kg_n, lk);
            else
                m2l_p1_direct<C, 1, P1D1>(zacc, xcol, vrow, rmax, ku, 4 * kg, 4 * kg_n, lk);
        }
    } else {
        // the next chunk is fetched into registers while the current one is
        // multiplied out of LDS (the MFMA loop issues no global loads, so these
        // loads are waited for only when they are committed to LDS)
        constexpr int SPT = LRJ * GG_NB / 256;
        constexpr int VPT = 64 * LRJ / 256;  // ranks up to 64 prefetched; rows 64.. read at commit
        C sreg[SPT], vreg[VPT];
        auto fetch = [&](int j0) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                const int jj = e % LRJ, b = e / LRJ;
                const int sb = sidx[b];
                sreg[i] = czero<C>();
                if (sb >= 0 && j0 + jj < ku) sreg[i] = gload(Xr + (int64_t)sb * ku + j0 + jj);
            }
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                vreg[i] = czero<C>();
                if (e < r * LRJ) {
                    const int row = e % r, kc = e / r;
                    if (j0 + kc < ku) vreg[i] = gload(Vt + row + (int64_t)(j0 + kc) * rmax);
                }
            }
        };
        __syncthreads();  // sidx
        fetch(0);
        for (int j0 = 0; j0 < ku; j0 += LRJ) {
            __syncthreads();  // the previous chunk is consumed
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                S[e % LRJ][e / LRJ] = sreg[i];
            }
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = threadIdx.x + 256 * i;
                if (e < r * LRJ) Vs[e / r][e % r] = vreg[i];
            }
            for (int e = threadIdx.x + 256 * VPT; e < r * LRJ; e += 256) {
                const int row = e % r, kc = e / r;
                C v = czero<C>();
                if (j0 + kc < ku) v = gload(Vt + row + (int64_t)(j0 + kc) * rmax);
                Vs[kc][row] = v;
            }
            __syncthreads();
            if (j0 + LRJ < ku) fetch(j0 + LRJ);
            const int jm = min(LRJ, ku - j0);
            for (int kk = 4 * kg; kk < jm; kk += 4 * kg_n) {
#pragma unroll
                for (int q = 0; q < ZQ; ++q) {
                    const int ti = tbase + tstep * q;
                    if (ti >= ntz) break;
                    const int row = (ti / NCT) * 16 + li;
                    C a = czero<C>();
                    if (row < r) a = Vs[kk + lk][row];
                    const C b = S[kk + lk][(ti % NCT) * 16 + li];
                    zacc[q].mac(a, b);
                }
            }
        }
        __syncthreads();
    }
    const int zoff = kg * 16 * ztiles;  // partial sums of k group kg (<= 64 rows in all)
#pragma unroll
    for (int q = 0; q < ZQ; ++q) {
        const int ti = tbase + tstep * q;
        if (ti >= ntz) break;
        const int zt = ti / NCT, c = ti % NCT;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            C z;
            z.x = zacc[q].re(v);
            z.y = zacc[q].im(v);
            // rows from r on are never read; for r > 64 the fifth row tile
            // would run past the LR_MAX rows of Z
            const int zr = zoff + zt * 16 + CT<C>::row(lk, v);
            if (zr < LR_MAX) Z[zr][c * 16 + li] = z;
        }
    }
    __syncthreads();
    if (kg_n > 1) {
        const int zr = 16 * ztiles, zc = 16 * NCT;
        for (int e = threadIdx.x; e < zr * zc; e += blockDim.x) {
            const int row = e / zc, col = e % zc;
            C s = Z[row][col];
            for (int g = 1; g < kg_n; ++g) {
                const C t = Z[g * zr + row][col];
                s.x += t.x;
                s.y += t.y;
            }
            Z[row][col] = s;
        }
        __syncthreads();
    }
    if constexpr (ZOUT) {
        for (int e = threadIdx.x; e < h.z * r; e += blockDim.x) {
            const int col = e / r, row = e - col * r;
            Tr[(int64_t)col * ldt + row] = Z[row][col];
        }
        return;
    }
    // phase 2: Y = U^[:, 0:r] Z (kd <= 256: 16 row tiles, 4 per wave, taken
    // two at a time to keep the accumulators small)
    const int ntile = (kd + 15) >> 4;
    constexpr int P2 = LR_P2;
    for (int pass = 0; pass < MF_RT / P2; ++pass) {
        const int rt0 = wave + 4 * P2 * pass;  // this pass: row tiles rt0, rt0 + 4
        if (rt0 >= ntile) break;
        CAcc<C> acc[P2][NCT];
#pragma unroll
        for (int q = 0; q < P2; ++q)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[q][c].zero();
        // U^ fragments PD k-steps ahead of their use (a phase-2 step is only
        // a few MFMAs); slot d is refilled right after it is consumed, so no
        // register moves tie a step to the load just issued.  Loads are
        // unconditional: rows from kd on are clamped (they feed output rows
        // that are never stored) and so are columns from r on (prefetches
        // past the last step, never used).
        C af[PD][P2];
        const C *urow[P2];
#pragma unroll
        for (int q = 0; q < P2; ++q) urow[q] = Ut + min((rt0 + 4 * q) * 16 + li, kd - 1);
        auto uload = [&](C (&av)[P2], int kc) {
            const int64_t o = (int64_t)min(kc, r - 1) * kd;
#pragma unroll
            for (int q = 0; q < P2; ++q) av[q] = gload(urow[q] + o);
        };
#pragma unroll
        for (int d = 0; d < PD; ++d) uload(af[d], 4 * d + lk);
        auto step = [&](const C (&av)[P2], int kk) {
            const C b0 = Z[kk + lk][li];
            const C b1 = NCT == 2 ? Z[kk + lk][16 + li] : czero<C>();
#pragma unroll
            for (int q = 0; q < P2; ++q) {
                acc[q][0].mac(av[q], b0);
                if (NCT == 2) acc[q][NCT - 1].mac(av[q], b1);
            }
        };
        const int nsteps = r >> 2;  // r is a multiple of 4
        int s = 0;
        for (; s + PD <= nsteps; s += PD) {
#pragma unroll
            for (int d = 0; d < PD; ++d) {
                step(af[d], 4 * (s + d));
                uload(af[d], 4 * (s + d + PD) + lk);
            }
        }
#pragma unroll
        for (int d = 0; d < PD; ++d)
            if (s + d < nsteps) step(af[d], 4 * (s + d));
#pragma unroll
        for (int q = 0; q < P2; ++q) {
            const int rt = rt0 + 4 * q;
            if (rt >= ntile) break;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const int col = c * 16 + li;
                if (col >= h.z) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rt * 16 + CT<C>::row(lk, v);
                    if (row < kd) {
                        C o;
                        o.x = acc[q][c].re(v);
                        o.y = acc[q][c].im(v);
                        Tr[(int64_t)col * ldt + row] = o;
                    }
                }
            }
        }
    }
}

#ifndef FDA_M2L_ZGROUP
// right-hand sides per group of the many-column phase 1 (rhs_block_grouped);
// 64 columns at N = 81,920, kD = 100 (FP64 phase 1): groups of 64 (item
// after item, every column) 11.7 ms, 16: 10.4, 4: 8.7, 1: 9.2
#define FDA_M2L_ZGROUP 4
#endif
// One launch for the low-rank M2L of every level: the item's level slot
// (h.w) selects its factors, states and scratch region.  ZOUT: phase 1
// only, Z of pair column c (level-local) and right-hand side j stored at
// T + zbase nrhs + (c nrhs + j) rmax.
template <class C, int VAR, bool ZOUT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M2LOcc<C>::waves)))
k_m2l_lowrank(const int4 *hdr, const int32_t *src, const M2LLevelArgs *args, C *T, int64_t tstride, int nwork,
              int nrhs) {
    // LDS: phase 1 stages S (LRJ x GG_LD) and V^ (LRJ x LR_LD); phase 2
    // reuses the same bytes for Z (LR_MAX x GG_LD) once phase 1 is done
    constexpr int kStage = M2LOcc<C>::direct ? 0 : LRJ * GG_LD + LRJ * LR_LD;
    constexpr int kZ = LR_MAX * GG_LD;
    __shared__ C smem[kStage > kZ ? kStage : kZ];
    __shared__ int32_t sidx[GG_NB];
    C(*S)[GG_LD] = (C(*)[GG_LD])smem;
    C(*Vs)[LR_LD] = (C(*)[LR_LD])(smem + LRJ * GG_LD);
    C(*Z)[GG_LD] = (C(*)[GG_LD])smem;
    // the host ordered the items for round-robin XCD dispatch (item t * 8 + x
    // on XCD x); empty items pad the queues
    const RhsBlock rb = ZOUT ? rhs_block_grouped(nrhs, (nwork + 7) >> 3, FDA_M2L_ZGROUP) : rhs_block(nrhs);
    const int w = rb.item;
    if (w >= nwork) return;
    const int4 h = hdr[w];
    if (h.z == 0) return;
    const M2LLevelArgs &la = args[h.w];
    const int kd = la.kd, ku = la.ku, rmax = la.rmax;
    const int op = h.x;
    const int r = la.rank[op];
    if (threadIdx.x < GG_NB) sidx[threadIdx.x] = src[(int64_t)w * GG_NB + threadIdx.x];
    const C *Xr = (const C *)la.X + (int64_t)rb.rhs * la.xstride;
    C *Tr = ZOUT ? T + la.zbase * nrhs + ((int64_t)h.y * nrhs + rb.rhs) * rmax
                 : T + (int64_t)rb.rhs * tstride + la.tbase + (int64_t)h.y * la.ldt;
    const int ldt = ZOUT ? nrhs * rmax : la.ldt;
    const C *Vt = (const C *)la.V + (int64_t)op * rmax * ((ku + 3) & ~3);
    const C *Ut = (const C *)la.U + (int64_t)op * kd * rmax;
    using V = M2LVariant<VAR>;
    if (h.z > 16)
        m2l_body<C, 2, V::p1d, V::p1d1, V::pd, ZOUT>(h, sidx, Ut, Vt, r, kd, ku, rmax, Xr, Tr, ldt, S, Vs, Z);
    else
        m2l_body<C, 1, V::p1d, V::p1d1, V::pd, ZOUT>(h, sidx, Ut, Vt, r, kd, ku, rmax, Xr, Tr, ldt, S, Vs, Z);
}

// The many-column form's second phase: c_t = sum over the interaction list
// of state t of U^_p Z_p (U^_p: kd x r_p, Z_p: the pair's phase-1 product,
// r_p x nrhs), accumulated on the matrix cores across the list and written
// once; with many columns every U^ fragment meets 16 NCT of them, so the
// destination-major order is dense.  Wave w of workgroup b owns unit
// 4 b + w, one (state, row tile) of the list (consecutive units share their
// state, so the waves of a workgroup mostly read the same Z), and columns
// 16 NCT blockIdx.y ..; its k loop runs over the list's pairs in list
// order, rank by rank, with the U^ and Z fragments loaded PD k-steps ahead
// (a fetch cursor walks the entries, the next entry's scalar load issued one
// pair ahead; past the last step it re-reads that step, never used).  No
// LDS, no barriers.
template <class C, int NCT, int PD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M2LDestOcc<C>::waves)))
k_m2l_dest(const int4 *units, int nunits, const int4 *ent, const int32_t *off, const int32_t *nst, const int32_t *dst,
           const M2LLevelArgs *args, const C *Zs, int nrhs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int u = (int)blockIdx.x * 4 + wave;
    if (u >= nunits) return;
    const int4 un = units[u];  // (state, row tile, level slot, 0)
    const M2LLevelArgs &la = args[un.z];
    const int kd = la.kd, rmax = la.rmax;
    const int rt = un.y;
    const int t = un.x;
    const int c0 = (int)blockIdx.y * 16 * NCT;
    const int64_t zp = (int64_t)nrhs * rmax;  // Z elements per pair
    const C *Zl = Zs + la.zbase * nrhs;
    const C *U = (const C *)la.U;
    const int64_t ukd = (int64_t)kd * rmax;  // U^ elements per translation
    const int arow = min(rt * 16 + li, kd - 1);
    int64_t bo[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) bo[c] = (int64_t)min(c0 + c * 16 + li, nrhs - 1) * rmax + lk;
    CAcc<C> acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c].zero();
    const int ns = nst[t];
    if (ns > 0) {
        int fe = off[t];
        const int last = off[t + 1] - 1;
        int4 en = ent[fe];  // (pair, translation, rank / 4, 0)
        int4 nx = ent[min(fe + 1, last)];
        int fk = 0;
        const C *fa = U + en.y * ukd + arow + (int64_t)lk * kd;
        const C *fb = Zl + en.x * zp;
        auto fetch = [&](C &a, C (&b)[NCT]) {
            a = gload(fa + (int64_t)(4 * fk) * kd);
#pragma unroll
            for (int c = 0; c < NCT; ++c) b[c] = gload(fb + bo[c] + 4 * fk);
            if (++fk == en.z) {
                if (fe < last) {
                    ++fe;
                    en = nx;
                    nx = ent[min(fe + 1, last)];
                    fk = 0;
                    fa = U + en.y * ukd + arow + (int64_t)lk * kd;
                    fb = Zl + en.x * zp;
                } else {
                    fk = en.z - 1;
                }
            }
        };
        C ar[PD], br[PD][NCT];
#pragma unroll
        for (int d = 0; d < PD; ++d) fetch(ar[d], br[d]);
        int s = 0;
        for (; s + PD <= ns; s += PD) {
#pragma unroll
            for (int d = 0; d < PD; ++d) {
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[c].mac(ar[d], br[d][c]);
                fetch(ar[d], br[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < PD; ++d)
            if (s + d < ns) {
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[c].mac(ar[d], br[d][c]);
            }
    }
    C *Y = (C *)la.Y + (int64_t)dst[t] * kd;
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
        const int col = c0 + c * 16 + li;
        if (col >= nrhs) continue;
        C *o = Y + (int64_t)col * la.ystride;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = rt * 16 + CT<C>::row(lk, v);
            if (row < kd) {
                C y;
                y.x = acc[c].re(v);
                y.y = acc[c].im(v);
                o[row] = y;
            }
        }
    }
}

// c[dst] = sum of the M2L scratch columns listed for dst (every state of the
// merged levels has an entry; an empty list writes zero), in list order.
// The (state, row) entries of a level are spread over the threads, kRedRows
// per block, so that every lane has a row whatever the rank.
template <class C>
__global__ void __launch_bounds__(kRedRows) k_gather_reduce_m2l(const int32_t *dst, const int32_t *off,
                                                                const int32_t *list, const int32_t *rd_block,
                                                                const int32_t *rd_state, int nlev,
                                                                const M2LLevelArgs *args, const C *T,
                                                                int64_t tstride) {
    // blocks run from the last level slot to the first: the finest levels'
    // states have the longest lists (about 45 scratch columns each against
    // 10 at the directional levels), and starting them first keeps them from
    // forming the launch's tail (0.158 -> 0.128 ms at N = 81,920, kD = 100)
    const int bx = (int)(gridDim.x - 1 - blockIdx.x);
    int q = 0;
    while (q + 1 < nlev && bx >= rd_block[q + 1]) ++q;
    const M2LLevelArgs &la = args[q];
    const int m = la.kd;
    const int64_t ld = la.ldt;  // scratch column stride
    const int64_t e = (int64_t)(bx - rd_block[q]) * kRedRows + threadIdx.x;
    const int64_t sl = e / m;
    const int r = (int)(e - sl * m);
    const int64_t t = rd_state[q] + sl;
    if (t >= rd_state[q + 1]) return;
    const C *Tr = T + (int64_t)blockIdx.y * tstride + la.tbase;
    C *out = (C *)la.Y + (int64_t)blockIdx.y * la.ystride + (int64_t)dst[t] * m;
    // four independent loads in flight per step; the sum keeps list order
    C acc = czero<C>();
    const int q0 = off[t], q1 = off[t + 1];
    int k = q0;
    for (; k + 4 <= q1; k += 4) {
        const C v0 = Tr[(int64_t)list[k] * ld + r], v1 = Tr[(int64_t)list[k + 1] * ld + r];
        const C v2 = Tr[(int64_t)list[k + 2] * ld + r], v3 = Tr[(int64_t)list[k + 3] * ld + r];
        acc.x += v0.x;
        acc.y += v0.y;
        acc.x += v1.x;
        acc.y += v1.y;
        acc.x += v2.x;
        acc.y += v2.y;
        acc.x += v3.x;
        acc.y += v3.y;
    }
    for (; k < q1; ++k) {
        const C v = Tr[(int64_t)list[k] * ld + r];
        acc.x += v.x;
        acc.y += v.y;
    }
    out[r] = acc;
}

// Y[dst] (+)= sum of the scratch columns listed for dst, in list order.
template <class C>
__global__ void k_gather_reduce(const int32_t *dst, const int32_t *off, const int32_t *list, int m, const C *T,
                                int64_t tstride, C *Y, int64_t ystride, int accumulate) {
    const int t = blockIdx.x;
    const C *Tr = T + (int64_t)blockIdx.y * tstride;
    C *out = Y + (int64_t)blockIdx.y * ystride + (int64_t)dst[t] * m;
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        C acc = accumulate ? out[r] : czero<C>();
        for (int q = off[t]; q < off[t + 1]; ++q) {
            C v = Tr[(int64_t)list[q] * m + r];
            acc.x += v.x;
            acc.y += v.y;
        }
        out[r] = acc;
    }
}

// y_leaf += T~ c_leaf (T~: n_L x kd, column-major per leaf; on a
// directional level kd counts every slot's columns, c_leaf being the box's
// [slot][rank] states), R right-hand sides per workgroup.  256 threads per
// leaf: rows are padded to a power of two npad <= 256 and the kd columns
// are split over 256 / npad thread groups, whose partial sums are added in
// a fixed order (the product is bound by reading T~ from HBM).  c_leaf is
// staged in LDS in chunks of kL2TChunk / R entries per column; a chunk is a
// multiple of the group count, so every thread meets its columns in
// increasing order whatever the chunking.
template <class C, int R>
__global__ void __launch_bounds__(256) k_l2t(const int64_t *leaf_off, const int32_t *ids, const int32_t *box,
                                             const int64_t *top, const C *Tm, int kd, const C *c, double2 *y,
                                             int64_t N, int64_t cstride, int nleaves, int ngroups, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int kc = min(kd, kL2TChunk / R);
    C *v = (C *)smem_raw;     // R x kc
    C *part = v + R * kc;     // R x 256
    const RhsBlock rb = rhs_block(ngroups);
    if (rb.item >= nleaves) return;
    const int r0 = rb.rhs * R, nr = min(R, nrhs - r0);
    const int b = ids[rb.item], t = threadIdx.x;
    const int64_t co = (int64_t)box[rb.item] * kd;
    const int64_t e0 = leaf_off[b];
    const int nl = (int)(leaf_off[b + 1] - e0);  // <= 256
    int npad = 1;
    while (npad < nl && npad < 256) npad <<= 1;
    const int G = 256 / npad;
    const int g = t / npad;
    const int i = t % npad;
    const C *Tb = Tm + top[b];
    C acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = czero<C>();
    for (int q0 = 0; q0 < kd; q0 += kc) {
        const int q1 = min(kd, q0 + kc), nq = q1 - q0;
        __syncthreads();  // the previous chunk is consumed
        for (int e = t; e < R * nq; e += blockDim.x) {
            const int r = e / nq, j = e - r * nq;
            v[r * kc + j] = r < nr ? c[(int64_t)(r0 + r) * cstride + co + q0 + j] : czero<C>();
        }
        __syncthreads();
        if (i < nl) {
            // four operator loads in flight (a group's column loop is only
            // about ten steps long; one load at a time left it waiting:
            // 0.034 -> 0.028 ms FP64 at N = 81,920); columns summed in
            // increasing order
            int q = q0 + g;
            for (; q + 3 * G < q1; q += 4 * G) {
                C m[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) m[u] = Tb[i + (int64_t)(q + u * G) * nl];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) cmac(acc[r], m[u], v[r * kc + q + u * G - q0]);
            }
            for (; q < q1; q += G) {
                const C m = Tb[i + (int64_t)q * nl];
#pragma unroll
                for (int r = 0; r < R; ++r) cmac(acc[r], m, v[r * kc + q - q0]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) part[r * 256 + t] = acc[r];
    __syncthreads();
    if (t < npad && i < nl) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            C s = part[r * 256 + t];
            for (int q = 1; q < G; ++q) {
                const C u = part[r * 256 + t + q * npad];
                s.x += u.x;
                s.y += u.y;
            }
            double2 *yr = y + (int64_t)(r0 + r) * N;
            double2 o = yr[e0 + i];
            yr[e0 + i] = make_double2(o.x + (double)s.x, o.y + (double)s.y);
        }
    }
}

template <class C>
__global__ void k_fill_zero(C *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = czero<C>();
}

// FP64 -> FP32 copy of an operator array.
__global__ void k_to_f32(const double2 *in, float2 *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// FP32 near-field blocks: the off-diagonal entries in FP32, the self terms
// kept in FP64 in diag (tree order).
__global__ void k_near_split(const int64_t *leaf_off, const int64_t *blk_off, const int32_t *self_col,
                             const int32_t *ncol, const double2 *vals, float2 *out, double2 *diag) {
    const int b = blockIdx.x;
    const int64_t t0 = leaf_off[b];
    const int nt = (int)(leaf_off[b + 1] - t0), nc = ncol[b], sc = self_col[b];
    const int64_t o = blk_off[b];
    for (int idx = threadIdx.x; idx < nt * nc; idx += blockDim.x) {
        const int i = idx / nc, c = idx - i * nc;
        const double2 v = vals[o + idx];
        if (c == sc + i) {
            diag[t0 + i] = v;
            out[o + idx] = make_float2(0.0f, 0.0f);
        } else {
            out[o + idx] = make_float2((float)v.x, (float)v.y);
        }
    }
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
// scale[c] = 1 / sqrt(Re d[c]) (0 for a zero column): reciprocal column
// norms from the columns' inner products with themselves, on the device.
__global__ void k_inv_norm(const double2 *d, double2 *scale, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) {
        const double r = d[c].x;
        scale[c] = make_double2(r > 0 ? 1.0 / sqrt(r) : 0.0, 0.0);
    }
}

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

hipError_t launch_near_blocks(const DevPlan &d, double2 *vals64, hipStream_t st, int op) {
    if (d.nleaf == 0) return hipSuccess;
    if (op == 1)
        hipLaunchKernelGGL(k_near_blocks<1>, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_col_off, d.nf_cols,
                           d.nf_blk_off, d.tri, d.cen, d.nrm, d.area, d.k, d.alpha, d.h_max, vals64);
    else
        hipLaunchKernelGGL(k_near_blocks<0>, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_col_off, d.nf_cols,
                           d.nf_blk_off, d.tri, d.cen, d.nrm, d.area, d.k, d.alpha, d.h_max, vals64);
    CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_bj_invert(const DevPlan &d, const double2 *vals64, hipStream_t st) {
    hipLaunchKernelGGL(k_bj_invert, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_blk_off, d.nf_self_col,
                       d.nf_ncol, vals64, d.bj_off, d.bj_inv);
    CHECK_LAUNCH();
    return hipSuccess;
}

static int grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 4096);
}

hipError_t launch_near_split(const DevPlan &d, const double2 *vals64, void *out32, double2 *diag, hipStream_t st) {
    hipLaunchKernelGGL(k_near_split, dim3(d.nleaf), dim3(256), 0, st, d.leaf_off, d.nf_blk_off, d.nf_self_col,
                       d.nf_ncol, vals64, (float2 *)out32, diag);
    CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_to_f32(const double2 *in, void *out, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3(grid1(n)), dim3(256), 0, st, in, (float2 *)out, n);
    CHECK_LAUNCH();
    return hipSuccess;
}

template <class C>
static hipError_t ggemm_t(const GWork &g, const void *A, int m, int kin, const void *X, int64_t xstride, void *Y,
                          int64_t ystride, int accumulate, int nrhs, hipStream_t st, hipEvent_t *ev) {
    if (g.nwork == 0) return hipSuccess;
    if constexpr (std::is_same<C, double2>::value) {
        if (!g.dst && g.dm_nunits > 0 && nrhs >= kGemmDestCols64) {
            // many columns (FP64): destination-major, no scratch and no reduction
            if (ev) hipEventRecord(ev[0], st);
            constexpr int PD = FDA_M2L_DEST_PD;
            auto go = [&](auto nc) -> hipError_t {
                constexpr int NCT = decltype(nc)::value;
                const dim3 gr((unsigned)((g.dm_nunits + 3) / 4), (unsigned)((nrhs + 16 * NCT - 1) / (16 * NCT)));
                hipLaunchKernelGGL((k_ggemm_dest<C, NCT, PD>), gr, dim3(256), 0, st, g.dm_units, g.dm_nunits, g.dm_ent,
                                   g.rd_off, g.rd_dst, (const C *)A, m, kin, (const C *)X, xstride, (C *)Y, ystride,
                                   accumulate, nrhs);
                CHECK_LAUNCH();
                if (ev) hipEventRecord(ev[1], st);
                return hipSuccess;
            };
            if (nrhs >= 64 && FDA_M2L_DEST_NCT >= 4) return go(std::integral_constant<int, 4>{});
            if (nrhs >= 32) return go(std::integral_constant<int, 2>{});
            return go(std::integral_constant<int, 1>{});
        }
    }
    constexpr int SB = 64 * GemmShape<C>::rt;
    const int nband = GemmShape<C>::band_split ? (m + SB - 1) / SB : 1;
    // a multiple of 8 workgroups so every XCD runs the same share
    const int grid = (g.nwork * nband + 7) / 8 * 8;
    const int64_t tstride = g.ncol * m;
    if (ev) hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_ggemm<C>, rhs_grid(grid, nrhs), dim3(256), 0, st, g.hdr, g.src, g.dst, (const C *)A, m,
                       kin, (const C *)X, xstride, (C *)g.tmp, tstride, (C *)Y, ystride, accumulate, g.nwork, nband,
                       nrhs);
    CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[1], st);
    if (g.dst) return hipSuccess;  // every destination had one product, written in place
    hipLaunchKernelGGL(k_gather_reduce<C>, dim3(g.nred, nrhs), dim3(std::min(256, ((m + 63) / 64) * 64)), 0, st,
                       g.rd_dst, g.rd_off, g.rd_list, m, (const C *)g.tmp, tstride, (C *)Y, ystride, accumulate);
    CHECK_LAUNCH();
    return hipSuccess;
}

// The merged low-rank M2L of all levels: the product kernel (variant
// mm.variant; ev[0], ev[1] around it when given) and the reduction of its
// scratch columns into the incoming states.
template <class C>
static hipError_t m2l_merged_t(const M2LMerged &mm, int nrhs, hipStream_t st, hipEvent_t *ev) {
    const dim3 g2 = rhs_grid(mm.nwork, nrhs);  // items ordered for XCD dispatch (or in translation order)
    if (ev) hipEventRecord(ev[0], st);
    if (nrhs >= (std::is_same<C, double2>::value ? kM2LManyCols64 : kM2LManyCols32) && mm.nzunits > 0) {
        // many-column form: Z per pair, then the destination-major U^ Z
        hipLaunchKernelGGL((k_m2l_lowrank<C, 0, true>), g2, dim3(256), 0, st, mm.hdr, mm.src, mm.args, (C *)mm.tmp,
                           mm.nscratch, mm.nwork, nrhs);
        CHECK_LAUNCH();
        if (ev) hipEventRecord(ev[1], st);
        constexpr int PD = FDA_M2L_DEST_PD;
        auto go = [&](auto nc) -> hipError_t {
            constexpr int NCT = decltype(nc)::value;
            const dim3 g((unsigned)((mm.nzunits + 3) / 4), (unsigned)((nrhs + 16 * NCT - 1) / (16 * NCT)));
            hipLaunchKernelGGL((k_m2l_dest<C, NCT, PD>), g, dim3(256), 0, st, mm.zunits, mm.nzunits, mm.rd_ent, mm.rd_off,
                               mm.rd_nst, mm.rd_dst, mm.args, (const C *)mm.tmp, nrhs);
            CHECK_LAUNCH();
            return hipSuccess;
        };
        if (nrhs >= 64 && FDA_M2L_DEST_NCT >= 4) return go(std::integral_constant<int, 4>{});
        if (nrhs >= 32) return go(std::integral_constant<int, 2>{});
        return go(std::integral_constant<int, 1>{});
    }
    switch (mm.variant) {
    case 1:
        hipLaunchKernelGGL((k_m2l_lowrank<C, 1>), g2, dim3(256), 0, st, mm.hdr, mm.src, mm.args, (C *)mm.tmp,
                           mm.nscratch, mm.nwork, nrhs);
        break;
    case 2:
        hipLaunchKernelGGL((k_m2l_lowrank<C, 2>), g2, dim3(256), 0, st, mm.hdr, mm.src, mm.args, (C *)mm.tmp,
                           mm.nscratch, mm.nwork, nrhs);
        break;
    case 3:
        hipLaunchKernelGGL((k_m2l_lowrank<C, 3>), g2, dim3(256), 0, st, mm.hdr, mm.src, mm.args, (C *)mm.tmp,
                           mm.nscratch, mm.nwork, nrhs);
        break;
    default:
        hipLaunchKernelGGL((k_m2l_lowrank<C, 0>), g2, dim3(256), 0, st, mm.hdr, mm.src, mm.args, (C *)mm.tmp,
                           mm.nscratch, mm.nwork, nrhs);
    }
    CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_gather_reduce_m2l<C>, dim3(mm.nredblocks, nrhs), dim3(kRedRows), 0, st, mm.rd_dst,
                       mm.rd_off, mm.rd_list, mm.rd_block, mm.rd_state, mm.nlev, mm.args, (const C *)mm.tmp,
                       mm.nscratch);
    CHECK_LAUNCH();
    return hipSuccess;
}

// The near field: work items of at most about 24k block entries (rows of
// one leaf), those with rows of <= kP2PShortCols columns first (x staged in
// LDS sized for their longest row), then the long rows (x read through the
// column list, no LDS), so that a few long rows neither serialise at the
// tail nor limit the occupancy of all.
template <class C>
static hipError_t launch_p2p_t(const DevPlan &d, const NearFar &op, const double2 *xt, double2 *yt, int nrhs,
                               hipStream_t st) {
    const int ns = d.p2p_nshort, nl = d.p2p_nitems - d.p2p_nshort;
    // right-hand sides per workgroup: up to 8, with x of the short rows'
    // columns for all of them in at most 64 KiB of LDS
    int R = 1;
    while (R < 8 && 2 * R <= nrhs && (size_t)2 * R * d.p2p_cols_short * sizeof(C) <= 65536) R *= 2;
    const int ng = (nrhs + R - 1) / R;
    auto go = [&](auto rc) -> hipError_t {
        constexpr int RR = decltype(rc)::value;
        if (ns > 0) {
            hipLaunchKernelGGL((k_p2p<C, RR>), rhs_grid(ns, ng), dim3(256), sizeof(C) * RR * d.p2p_cols_short, st,
                               d.p2p_items, d.leaf_off, d.nf_col_off, d.nf_cols, d.nf_blk_off, (const C *)op.nf_vals,
                               (const double2 *)op.nf_diag, xt, yt, d.n, ns, ng, nrhs);
            CHECK_LAUNCH();
        }
        if (nl > 0) {
            hipLaunchKernelGGL((k_p2p_direct<C, RR>), rhs_grid(nl, ng), dim3(256), 0, st, d.p2p_items + ns,
                               d.leaf_off, d.nf_col_off, d.nf_cols, d.nf_blk_off, (const C *)op.nf_vals,
                               (const double2 *)op.nf_diag, xt, yt, d.n, nl, ng, nrhs);
            CHECK_LAUNCH();
        }
        return hipSuccess;
    };
    switch (R) {
    case 8: return go(std::integral_constant<int, 8>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 2: return go(std::integral_constant<int, 2>{});
    default: return go(std::integral_constant<int, 1>{});
    }
}

// Leaf S2M and L2T of one level for nrhs columns, up to 8 per workgroup.
template <class C>
static hipError_t launch_s2m_t(const DevPlan &d, const DevLevel &lf, const void *S, const double2 *xt, int nrhs,
                               hipStream_t st) {
    const int R = nrhs >= 8 ? 8 : nrhs >= 4 ? 4 : nrhs >= 2 ? 2 : 1;
    const int ng = (nrhs + R - 1) / R;
    const int ku = lf.nslot * lf.ku;  // a leaf's states are [slot][rank]: one vector of nslot ku entries
    auto go = [&](auto rc) -> hipError_t {
        constexpr int RR = decltype(rc)::value;
        hipLaunchKernelGGL((k_s2m<C, RR>), rhs_grid(lf.nleaves, ng), dim3(128), sizeof(C) * RR * d.max_leaf, st,
                           d.leaf_off, lf.leaf_ids, lf.leaf_box, d.leaf_sop, (const C *)S, ku, xt, (C *)lf.s, d.n,
                           lf.sstride, lf.nleaves, ng, nrhs);
        CHECK_LAUNCH();
        return hipSuccess;
    };
    switch (R) {
    case 8: return go(std::integral_constant<int, 8>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 2: return go(std::integral_constant<int, 2>{});
    default: return go(std::integral_constant<int, 1>{});
    }
}

template <class C>
static hipError_t launch_l2t_t(const DevPlan &d, const DevLevel &lf, const double2 *dummy, double2 *yt, int nrhs,
                               hipStream_t st) {
    (void)dummy;
    const int R = nrhs >= 8 ? 8 : nrhs >= 4 ? 4 : nrhs >= 2 ? 2 : 1;
    const int ng = (nrhs + R - 1) / R;
    const int kd = lf.nslot * lf.kd;
    auto go = [&](auto rc) -> hipError_t {
        constexpr int RR = decltype(rc)::value;
        const size_t lds = sizeof(C) * RR * (std::min(kd, kL2TChunk / RR) + 256);
        hipLaunchKernelGGL((k_l2t<C, RR>), rhs_grid(lf.nleaves, ng), dim3(256), lds, st, d.leaf_off, lf.leaf_ids,
                           lf.leaf_box, d.leaf_top, (const C *)d.T, kd, (const C *)lf.c, yt, d.n, lf.cstride,
                           lf.nleaves, ng, nrhs);
        CHECK_LAUNCH();
        return hipSuccess;
    };
    switch (R) {
    case 8: return go(std::integral_constant<int, 8>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 2: return go(std::integral_constant<int, 2>{});
    default: return go(std::integral_constant<int, 1>{});
    }
}

// Stage timings are recorded when ev != nullptr (7 events: start, after
// near, after S2M, after M2M, after M2L, after L2L, end).
template <class C>
static hipError_t matvec_t(const DevPlan &d, const double2 *xt, double2 *yt, int nrhs, hipStream_t st,
                           hipEvent_t *ev, hipEvent_t *lev, const NearFar &op) {
    const int64_t N = d.n;
    // The near field (HBM-bound) overlaps the far-field chain (matrix cores)
    // on the plan's side stream, unless stage timings are taken or the
    // caller's stream is being captured into a graph (a fork onto the side
    // stream inside a capture has crashed the runtime; captured branches
    // run concurrently anyway).
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (d.side) {
        const hipError_t e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return e;
    }
    const bool overlap = !ev && d.side && d.has_far && cs == hipStreamCaptureStatusNone;
    // near field on the side stream, forked from st at this point
    auto near_side = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(d.fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(d.side, d.fork, 0);
        if (e != hipSuccess) return e;
        e = launch_p2p_t<C>(d, op, xt, yt, nrhs, d.side);
        if (e == hipSuccess) e = hipEventRecord(d.join, d.side);
        return e;
    };
    if (ev) hipEventRecord(ev[0], st);
    if (!overlap) {
        const hipError_t e = launch_p2p_t<C>(d, op, xt, yt, nrhs, st);
        if (e != hipSuccess) return e;
    } else {  // the side stream starts with the matvec (beside S2M, M2M and M2L)
        const hipError_t e = near_side();
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[1], st);
    if (!d.has_far) {
        for (int q = 2; q < 7 && ev; ++q) hipEventRecord(ev[q], st);
        return hipSuccess;
    }
    const int L = d.depth, top = d.top;
    // S2M at the leaves of every level (a leaf's state is never written by
    // M2M: only boxes with children are)
    for (int l = L; l >= top; --l) {
        const DevLevel &lf = d.lv[l];
        if (lf.nleaves == 0) continue;
        const hipError_t e = launch_s2m_t<C>(d, lf, op.S, xt, nrhs, st);
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[2], st);
    for (int l = L - 1; l >= top; --l) {
        const DevLevel &P = d.lv[l], &Cl = d.lv[l + 1];
        hipError_t e = ggemm_t<C>(P.m2m, P.M, P.ku, Cl.ku, Cl.s, Cl.sstride, P.s, P.sstride, 0, nrhs, st, nullptr);
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[3], st);
    if (d.m2l_all.nwork > 0) {
        const hipError_t e = m2l_merged_t<C>(d.m2l_all, nrhs, st, lev ? lev + 48 : nullptr);
        if (e != hipSuccess) return e;
    }
    for (int l = top; l <= L; ++l) {
        const DevLevel &lv = d.lv[l];
        if (lv.merged) continue;
        int64_t n = lv.cstride * nrhs;
        hipLaunchKernelGGL(k_fill_zero<C>, dim3(grid1(n)), dim3(256), 0, st, (C *)lv.c, n);
        CHECK_LAUNCH();
        hipError_t e = ggemm_t<C>(lv.m2l, lv.K, lv.kd, lv.ku, lv.s, lv.sstride, lv.c, lv.cstride, 1, nrhs, st,
                                  lev ? lev + 2 * l : nullptr);
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[4], st);
    for (int l = top; l < L; ++l) {
        const DevLevel &P = d.lv[l], &Cl = d.lv[l + 1];
        hipError_t e = ggemm_t<C>(P.l2l, P.Lo, Cl.kd, P.kd, P.c, P.cstride, Cl.c, Cl.cstride, 1, nrhs, st, nullptr);
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[5], st);
    if (overlap) {
        hipError_t e = hipStreamWaitEvent(st, d.join, 0);  // L2T adds to the near-field result
        if (e != hipSuccess) return e;
    }
    for (int l = top; l <= L; ++l) {
        const DevLevel &lf = d.lv[l];
        if (lf.nleaves == 0) continue;
        const hipError_t e = launch_l2t_t<C>(d, lf, xt, yt, nrhs, st);
        if (e != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[6], st);
    return hipSuccess;
}

hipError_t launch_matvec_tree(const DevPlan &d, const double2 *xt, double2 *yt, int nrhs, hipStream_t st,
                              hipEvent_t *ev, hipEvent_t *lev, const NearFar *ops) {
    NearFar a;
    a.nf_vals = d.nf_vals;
    a.nf_diag = d.nf_diag;
    a.S = d.S;
    const NearFar &op = ops ? *ops : a;
    if (d.prec == 1) return matvec_t<float2>(d, xt, yt, nrhs, st, ev, lev, op);
    return matvec_t<double2>(d, xt, yt, nrhs, st, ev, lev, op);
}

hipError_t launch_m2l_merged(const DevPlan &d, int nrhs, hipStream_t st) {
    if (d.m2l_all.nwork == 0) return hipSuccess;
    if (d.prec == 1) return m2l_merged_t<float2>(d.m2l_all, nrhs, st, nullptr);
    return m2l_merged_t<double2>(d.m2l_all, nrhs, st, nullptr);
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
hipError_t launch_inv_norm(const double2 *d, double2 *scale, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_inv_norm, dim3((n + 63) / 64), dim3(64), 0, st, d, scale, n);
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
    hipLaunchKernelGGL(k_fill_zero<double2>, dim3(grid1(n)), dim3(256), 0, st, p, n);
    CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace fda
