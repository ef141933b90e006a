/*
 * FP64 CPU oracle for the collocation Burton-Miller boundary element
 * operator with piecewise-constant flat triangles.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, dense definition
 * of what the fast directional algorithm approximates.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * What is computed (paper, Section 2, eqs. (cbie), (eq_bm), (eq_sum); and
 * Section 5 for the collocation / piecewise-constant choice):
 *
 *   A_ij = 1/2 delta_ij + int_{D_j} [ dG/dn_y + alpha d2G/dn_x dn_y ](c_i, y) dy
 *   B_ij = -alpha/2 delta_ij + int_{D_j} [ G + alpha dG/dn_x ](c_i, y) dy
 *
 * with G = exp(ikR) / (4 pi R), c_i the centroid of triangle i, collocation
 * weight delta(c_i) and basis chi_j = 1 on triangle j.  The free term c = 1/2
 * holds at the centroid of a flat triangle.  The normal n used by the
 * paper's equations points out of the fluid, into the scatterer: it is the
 * opposite of the right-hand normal of a triangle wound counter-clockwise as
 * seen from the fluid.  A is the left-hand operator acting on the surface
 * potential u; B is the right-hand operator acting on Neumann data du/dn.
 *
 * Element integration (the paper leaves the rule open):
 *   - regular pairs: Radon's 7-point degree-5 rule on the triangle;
 *   - near pairs, graded by d = |c_i - c_j| against the largest edge h of
 *     the mesh:  d/h < 1      -> the 7-point rule on 64 sub-triangles,
 *                1 <= d/h < 1.75 -> on 16 sub-triangles,
 *                1.75 <= d/h < 2.5 -> on 4 sub-triangles,
 *                d/h >= 2.5   -> the plain 7-point rule;
 *     sub-triangles come from repeated midpoint subdivision;
 *   - the element's own integral at its centroid (flat triangle, so
 *     r . n = 0 and the double-layer parts vanish):
 *       f.p. int d2G/dn_x dn_y = ik/2 - (1/4pi) int_0^{2pi} exp(ikR(t))/R(t) dt
 *       int G                  = (i/(4 pi k)) int_0^{2pi} (1 - exp(ikR(t))) dt
 *     where R(t) is the distance from the centroid to the boundary along
 *     the polar angle t; each edge's angular range is integrated with a
 *     32-point Gauss-Legendre rule in the angle measured from the foot of
 *     the perpendicular.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- rules */

/* Radon 7-point rule: barycentric coordinates (3 per point) and weights as a
 * fraction of the triangle area. */
static double r7_bary[7][3];
static double r7_w[7];
/* Gauss-Legendre nodes and weights on [-1, 1]. */
#define GL_N 32
static double gl_x[GL_N], gl_w[GL_N];
static int rules_ready = 0;

static void legendre_rule(int n, double *x, double *w)
{
    /* Newton iteration on P_n from the Chebyshev guesses, three-term
     * recurrence for P_n and its derivative. */
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void init_rules(void)
{
    if (rules_ready) return;
    const double s15 = sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
    r7_bary[0][0] = r7_bary[0][1] = r7_bary[0][2] = 1.0 / 3.0;
    r7_w[0] = 9.0 / 40.0;
    for (int p = 0; p < 3; ++p) {
        for (int q = 0; q < 3; ++q) {
            r7_bary[1 + p][q] = (q == p) ? 1.0 - 2.0 * a : a;
            r7_bary[4 + p][q] = (q == p) ? 1.0 - 2.0 * b : b;
        }
        r7_w[1 + p] = wa;
        r7_w[4 + p] = wb;
    }
    legendre_rule(GL_N, gl_x, gl_w);
    rules_ready = 1;
}

/* --------------------------------------------------------------- vectors */

static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* -------------------------------------------------------------- geometry */

/* Centroid, paper normal (into the body), area of every triangle and the
 * largest edge of the mesh.  Returns 0, or -1 for a bad index or a
 * degenerate triangle. */
int or_geometry(const double *V, int64_t nv, const int32_t *T, int64_t nt,
                double *cen, double *nrm, double *area, double *hmax)
{
    double h = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *f = T + 3 * t;
        for (int q = 0; q < 3; ++q)
            if (f[q] < 0 || f[q] >= nv) return -1;
        const double *p0 = V + 3 * f[0], *p1 = V + 3 * f[1], *p2 = V + 3 * f[2];
        double e1[3], e2[3], e3[3], c[3];
        for (int q = 0; q < 3; ++q) {
            e1[q] = p1[q] - p0[q];
            e2[q] = p2[q] - p0[q];
            e3[q] = p2[q] - p1[q];
        }
        cross3(e1, e2, c);
        double len = sqrt(dot3(c, c));
        if (!(len > 0.0)) return -1;
        for (int q = 0; q < 3; ++q) {
            cen[3 * t + q] = (p0[q] + p1[q] + p2[q]) / 3.0;
            nrm[3 * t + q] = -c[q] / len; /* right-hand normal points into the fluid */
        }
        area[t] = 0.5 * len;
        double l1 = sqrt(dot3(e1, e1)), l2 = sqrt(dot3(e2, e2)), l3 = sqrt(dot3(e3, e3));
        if (l1 > h) h = l1;
        if (l2 > h) h = l2;
        if (l3 > h) h = l3;
    }
    *hmax = h;
    return 0;
}

/* --------------------------------------------------------------- kernels */

/* Kernel values at x (normal nx) due to y (normal ny):
 *   out[0] = G, out[1] = dG/dn_y, out[2] = dG/dn_x, out[3] = d2G/dn_x dn_y.
 * With r = x - y, R = |r| and G'(R) = exp(ikR)(ikR - 1)/(4 pi R^2):
 *   dG/dn_y = -G'(R) (r.n_y)/R,   dG/dn_x = G'(R) (r.n_x)/R,
 *   d2G     = exp(ikR)/(4 pi R^3) [ (1 - ikR) n_x.n_y
 *                                  - (3 - 3ikR - k^2R^2)(r^.n_x)(r^.n_y) ]. */
static inline void kernel4(const double *x, const double *y, const double *nx, const double *ny,
                           double k, cplx out[4])
{
    double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double R = sqrt(dot3(r, r));
    cplx ikR = I * k * R;
    cplx g = cexp(ikR) / (4.0 * OR_PI * R);
    cplx gp = g * (ikR - 1.0) / R;
    double rnx = dot3(r, nx) / R, rny = dot3(r, ny) / R;
    out[0] = g;
    out[1] = -gp * rny;
    out[2] = gp * rnx;
    out[3] = g / (R * R) * ((1.0 - ikR) * dot3(nx, ny) - (3.0 - 3.0 * ikR - k * k * R * R) * rnx * rny);
}

void or_kernels(int64_t n, const double *x, const double *y, const double *nx, const double *ny,
                double k, double *out /* n x 4 complex, interleaved */)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx v[4];
        kernel4(x + 3 * i, y + 3 * i, nx + 3 * i, ny + 3 * i, k, v);
        for (int q = 0; q < 4; ++q) {
            out[8 * i + 2 * q] = creal(v[q]);
            out[8 * i + 2 * q + 1] = cimag(v[q]);
        }
    }
}

/* ------------------------------------------------------ element integrals */

/* Integrate the four kernels over a triangle (vertices a, b, c, area A) with
 * the 7-point rule, accumulating into acc[4]. */
static void r7_triangle(const double *a, const double *b, const double *c, double A,
                        const double *x, const double *nx, const double *ny, double k, cplx acc[4])
{
    for (int p = 0; p < 7; ++p) {
        double y[3];
        for (int q = 0; q < 3; ++q)
            y[q] = r7_bary[p][0] * a[q] + r7_bary[p][1] * b[q] + r7_bary[p][2] * c[q];
        cplx v[4];
        kernel4(x, y, nx, ny, k, v);
        for (int q = 0; q < 4; ++q) acc[q] += r7_w[p] * A * v[q];
    }
}

/* Midpoint-subdivide a triangle `level` times and apply the 7-point rule on
 * every piece. */
static void r7_subdivided(const double *a, const double *b, const double *c, double A, int level,
                          const double *x, const double *nx, const double *ny, double k, cplx acc[4])
{
    if (level == 0) {
        r7_triangle(a, b, c, A, x, nx, ny, k, acc);
        return;
    }
    double ab[3], bc[3], ca[3];
    for (int q = 0; q < 3; ++q) {
        ab[q] = 0.5 * (a[q] + b[q]);
        bc[q] = 0.5 * (b[q] + c[q]);
        ca[q] = 0.5 * (c[q] + a[q]);
    }
    double A4 = 0.25 * A;
    r7_subdivided(a, ab, ca, A4, level - 1, x, nx, ny, k, acc);
    r7_subdivided(b, bc, ab, A4, level - 1, x, nx, ny, k, acc);
    r7_subdivided(c, ca, bc, A4, level - 1, x, nx, ny, k, acc);
    r7_subdivided(ab, bc, ca, A4, level - 1, x, nx, ny, k, acc);
}

/* Subdivision level chosen from the centroid distance d and the mesh's
 * largest edge h. */
static int grade_level(double d, double h)
{
    if (d < 1.0 * h) return 3;
    if (d < 1.75 * h) return 2;
    if (d < 2.5 * h) return 1;
    return 0;
}

/* Self integrals over the element's own triangle at its centroid:
 *   s[0] = int G,  s[3] = f.p. int d2G/dn_x dn_y;  s[1] = s[2] = 0. */
static void self_integrals(const double *a, const double *b, const double *c, const double *x,
                           double k, cplx s[4])
{
    const double *P[3] = {a, b, c};
    cplx int_e_over_R = 0.0, int_e = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *p = P[e], *q = P[(e + 1) % 3];
        double ev[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        double L = sqrt(dot3(ev, ev));
        double eh[3] = {ev[0] / L, ev[1] / L, ev[2] / L};
        double xp[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        double t = dot3(xp, eh); /* foot of the perpendicular at p + t eh */
        double f[3] = {p[0] + t * eh[0] - x[0], p[1] + t * eh[1] - x[1], p[2] + t * eh[2] - x[2]};
        double d = sqrt(dot3(f, f));
        double phi1 = atan2(-t, d), phi2 = atan2(L - t, d);
        double half = 0.5 * (phi2 - phi1), mid = 0.5 * (phi2 + phi1);
        for (int g = 0; g < GL_N; ++g) {
            double phi = mid + half * gl_x[g];
            double R = d / cos(phi);
            cplx eR = cexp(I * k * R);
            int_e_over_R += half * gl_w[g] * eR / R;
            int_e += half * gl_w[g] * eR;
        }
    }
    s[0] = (I / (4.0 * OR_PI * k)) * (2.0 * OR_PI - int_e);
    s[1] = 0.0;
    s[2] = 0.0;
    s[3] = I * k / 2.0 - int_e_over_R / (4.0 * OR_PI);
}

typedef struct {
    const double *V;
    const int32_t *T;
    int64_t nt;
    const double *cen, *nrm, *area;
    double h;
} geo_t;

/* The four element integrals of row i, column j:
 *   v[0] = int G, v[1] = int dG/dn_y, v[2] = int dG/dn_x, v[3] = int d2G. */
static void element_integrals(const geo_t *g, int64_t i, int64_t j, double k, cplx v[4])
{
    const int32_t *f = g->T + 3 * j;
    const double *a = g->V + 3 * f[0], *b = g->V + 3 * f[1], *c = g->V + 3 * f[2];
    const double *x = g->cen + 3 * i;
    v[0] = v[1] = v[2] = v[3] = 0.0;
    if (i == j) {
        self_integrals(a, b, c, x, k, v);
        return;
    }
    double dv[3] = {x[0] - g->cen[3 * j], x[1] - g->cen[3 * j + 1], x[2] - g->cen[3 * j + 2]};
    double d = sqrt(dot3(dv, dv));
    r7_subdivided(a, b, c, g->area[j], grade_level(d, g->h), x, g->nrm + 3 * i, g->nrm + 3 * j, k, v);
}

/* Operator selector. */
enum { OP_S = 0, OP_K = 1, OP_KP = 2, OP_T = 3, OP_A = 4, OP_B = 5 };

static cplx op_entry(const geo_t *g, int64_t i, int64_t j, double k, cplx alpha, int op)
{
    cplx v[4];
    element_integrals(g, i, j, k, v);
    switch (op) {
    case OP_S: return v[0];
    case OP_K: return v[1];
    case OP_KP: return v[2];
    case OP_T: return v[3];
    case OP_A: return (i == j ? 0.5 : 0.0) + v[1] + alpha * v[3];
    case OP_B: return (i == j ? -0.5 * alpha : 0.0) + v[0] + alpha * v[2];
    }
    return 0.0;
}

static int build_geo(const double *V, int64_t nv, const int32_t *T, int64_t nt, geo_t *g)
{
    init_rules();
    double *buf = (double *)malloc(sizeof(double) * 7 * (size_t)nt);
    if (!buf) return -2;
    g->V = V;
    g->T = T;
    g->nt = nt;
    g->cen = buf;
    g->nrm = buf + 3 * nt;
    g->area = buf + 6 * nt;
    if (or_geometry(V, nv, T, nt, buf, buf + 3 * nt, buf + 6 * nt, &g->h) != 0) {
        free(buf);
        return -1;
    }
    return 0;
}

/* Dense rows: out[r * nt + j] = M(rows[r], j) for the selected operator,
 * complex interleaved, row-major. */
int or_rows(const double *V, int64_t nv, const int32_t *T, int64_t nt, double k,
            double alpha_re, double alpha_im, int op, const int64_t *rows, int64_t nrows,
            double *out)
{
    geo_t g;
    int rc = build_geo(V, nv, T, nt, &g);
    if (rc) return rc;
    cplx alpha = alpha_re + I * alpha_im;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        for (int64_t j = 0; j < nt; ++j) {
            cplx e = op_entry(&g, rows[r], j, k, alpha, op);
            out[2 * (r * nt + j)] = creal(e);
            out[2 * (r * nt + j) + 1] = cimag(e);
        }
    }
    free((void *)g.cen);
    return 0;
}

/* Matrix-free product over selected rows:
 *   y[r, c] = sum_j M(rows[r], j) x[j, c],  c < nrhs,
 * x is nt x nrhs and y is nrows x nrhs, both complex interleaved, row-major
 * (the nrhs values of one element are adjacent). */
int or_apply(const double *V, int64_t nv, const int32_t *T, int64_t nt, double k,
             double alpha_re, double alpha_im, int op, const int64_t *rows, int64_t nrows,
             const double *x, int64_t nrhs, double *y)
{
    geo_t g;
    int rc = build_geo(V, nv, T, nt, &g);
    if (rc) return rc;
    cplx alpha = alpha_re + I * alpha_im;
#pragma omp parallel
    {
        cplx *acc = (cplx *)malloc(sizeof(cplx) * (size_t)nrhs);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            for (int64_t c = 0; c < nrhs; ++c) acc[c] = 0.0;
            for (int64_t j = 0; j < nt; ++j) {
                cplx e = op_entry(&g, rows[r], j, k, alpha, op);
                for (int64_t c = 0; c < nrhs; ++c)
                    acc[c] += e * (x[2 * (j * nrhs + c)] + I * x[2 * (j * nrhs + c) + 1]);
            }
            for (int64_t c = 0; c < nrhs; ++c) {
                y[2 * (r * nrhs + c)] = creal(acc[c]);
                y[2 * (r * nrhs + c) + 1] = cimag(acc[c]);
            }
        }
        free(acc);
    }
    free((void *)g.cen);
    return 0;
}

/* The 7-point rule itself (barycentric coordinates and area fractions), for
 * the exactness check. */
void or_r7_rule(double *bary /* 7 x 3 */, double *w /* 7 */)
{
    init_rules();
    for (int p = 0; p < 7; ++p) {
        for (int q = 0; q < 3; ++q) bary[3 * p + q] = r7_bary[p][q];
        w[p] = r7_w[p];
    }
}

/* The Gauss-Legendre rule used by the self integrals. */
void or_gl_rule(double *x, double *w)
{
    init_rules();
    memcpy(x, gl_x, sizeof(gl_x));
    memcpy(w, gl_w, sizeof(gl_w));
}

/* Self integrals of one triangle at a given collocation point (for pins):
 * out = [int G, 0, 0, f.p. int d2G] as complex interleaved. */
void or_self(const double *a, const double *b, const double *c, const double *x, double k, double *out)
{
    init_rules();
    cplx s[4];
    self_integrals(a, b, c, x, k, s);
    for (int q = 0; q < 4; ++q) {
        out[2 * q] = creal(s[q]);
        out[2 * q + 1] = cimag(s[q]);
    }
}

/* Element integrals of an arbitrary triangle against an arbitrary target
 * point and normal, with an explicit subdivision level (for pins). */
void or_element(const double *a, const double *b, const double *c, const double *x, const double *nx,
                double k, int level, double *out)
{
    init_rules();
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double cr[3];
    cross3(e1, e2, cr);
    double len = sqrt(dot3(cr, cr));
    double ny[3] = {-cr[0] / len, -cr[1] / len, -cr[2] / len};
    cplx v[4] = {0, 0, 0, 0};
    r7_subdivided(a, b, c, 0.5 * len, level, x, nx, ny, k, v);
    for (int q = 0; q < 4; ++q) {
        out[2 * q] = creal(v[q]);
        out[2 * q + 1] = cimag(v[q]);
    }
}
