// Leaf operators of the fast directional algorithm formed on the host from
// the SVD factors: compressed S2M and L2T matrices per leaf (Section 4.3),
// which fold the 7-point element quadrature (S2M, eq. (eq_s2m)) and the
// target operator [1 + alpha d/dn_x] (L2T, eq. (eq_l2t)).  The left-hand
// operator A has the source kernel dG/dn_y; the right-hand operator B of
// eq. (eq_bm) (Neumann data) the source kernel G and the same target
// operator, so only its S2M differs.
#include <cmath>
#include <cstring>

#include "operators.hpp"

namespace fda {

static const double kPi = 3.14159265358979323846;

// Radon's 7-point degree-5 rule on a triangle (barycentric coordinates and
// area fractions).
static void r7_rule(double bary[7][3], double w[7]) {
    const double s15 = std::sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    for (int p = 0; p < 3; ++p) {
        for (int q = 0; q < 3; ++q) {
            bary[1 + p][q] = (q == p) ? 1.0 - 2.0 * a : a;
            bary[4 + p][q] = (q == p) ? 1.0 - 2.0 * b : b;
        }
        w[1 + p] = (155.0 - s15) / 1200.0;
        w[4 + p] = (155.0 + s15) / 1200.0;
    }
}

static void scale_rows(Mat &M, const std::vector<double> &s) {
    for (int j = 0; j < M.n; ++j)
        for (int i = 0; i < M.m; ++i) M(i, j) /= s[i];
}
static void scale_cols(Mat &M, const std::vector<double> &s) {
    for (int j = 0; j < M.n; ++j)
        for (int i = 0; i < M.m; ++i) M(i, j) /= s[j];
}

void form_operators(const HostPlan &hp, HostOps &ops) {
    const int L = hp.depth;
    const double k = hp.k;
    const cplx alpha = hp.alpha;
    bool any = false;
    for (int l = hp.top; l <= L; ++l)
        if (!hp.lv[l].offsets.empty()) any = true;
    if (!any) return;  // everything is near field

    // leaf S2M and L2T per leaf (Section 4.3): S~ = S^-1 U^H E_up, T~ = E_dn V S^-1,
    // with the point sets and factors of the leaf's own level; a leaf on a
    // directional level has one S~ and one T~ per direction slot of the
    // level (outgoing check set and incoming equivalent set of that slot's
    // cone), stacked so that its states [slot][rank] are one vector
    double bary[7][3], w7[7];
    r7_rule(bary, w7);
    const int64_t nleaf = hp.nleaf;
    const bool rhsB = hp.opt.neumann_rhs != 0;
    auto has_far = [&](int64_t t) { return hp.leaf_level[t] >= hp.top; };
    auto nslot = [&](const Level &lf) { return lf.hf ? lf.nslot : 1; };
    ops.sop.assign(nleaf + 1, 0);
    ops.top.assign(nleaf + 1, 0);
    for (int64_t t = 0; t < nleaf; ++t) {
        const Level &lf = hp.lv[hp.leaf_level[t]];
        const int64_t nl = hp.leaf_off[t + 1] - hp.leaf_off[t];
        ops.sop[t + 1] = ops.sop[t] + (has_far(t) ? (int64_t)nslot(lf) * lf.ku * nl : 0);
        ops.top[t + 1] = ops.top[t] + (has_far(t) ? (int64_t)nslot(lf) * lf.kd * nl : 0);
    }
    ops.S.assign((size_t)ops.sop[nleaf], cplx(0));
    ops.T.assign((size_t)ops.top[nleaf], cplx(0));
    if (rhsB) ops.SB.assign((size_t)ops.sop[nleaf], cplx(0));
    parallel_for(nleaf, [&](int64_t t) {
        if (!has_far(t)) return;
        const Level &lf = hp.lv[hp.leaf_level[t]];
        const int64_t b = hp.leaf_box[t];
        const int ns = nslot(lf);
        int64_t e0 = hp.leaf_off[t], e1 = hp.leaf_off[t + 1];
        int nl = (int)(e1 - e0);
        double c[3];
        for (int q = 0; q < 3; ++q) c[q] = hp.origin[q] + (lf.key[3 * b + q] + 0.5) * lf.w;
        const int64_t srows = (int64_t)ns * lf.ku;
        for (int sl = 0; sl < ns; ++sl) {
            const std::vector<double> uc = out_check(lf, sl), de = in_equiv(lf, sl);
            const int nc = (int)uc.size() / 3, nd = (int)de.size() / 3;
            Mat E(nc, nl), Ed(nl, nd), EB(rhsB ? nc : 0, rhsB ? nl : 0);
            for (int j = 0; j < nl; ++j) {
                int64_t e = e0 + j;
                const double *tv = &hp.tri[9 * e];
                const double *ny = &hp.nrm[3 * e];
                for (int i = 0; i < nc; ++i) {
                    double x[3] = {uc[3 * i] + c[0], uc[3 * i + 1] + c[1], uc[3 * i + 2] + c[2]};
                    cplx acc = 0, accB = 0;
                    for (int q = 0; q < 7; ++q) {
                        double y[3];
                        for (int a = 0; a < 3; ++a)
                            y[a] = bary[q][0] * tv[a] + bary[q][1] * tv[3 + a] + bary[q][2] * tv[6 + a];
                        double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
                        double R = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                        cplx g = std::exp(cplx(0, k * R)) / (4 * kPi * R);
                        cplx gp = g * cplx(-1.0, k * R) / R;
                        double rny = (r[0] * ny[0] + r[1] * ny[1] + r[2] * ny[2]) / R;
                        acc += w7[q] * hp.area[e] * (-gp * rny);
                        accB += w7[q] * hp.area[e] * g;
                    }
                    E(i, j) = acc;
                    if (rhsB) EB(i, j) = accB;
                }
                // target side: [G + alpha dG/dn_x](c_j, incoming equivalent point)
                const double *x = &hp.cen[3 * e];
                const double *nx = &hp.nrm[3 * e];
                for (int i = 0; i < nd; ++i) {
                    double y[3] = {de[3 * i] + c[0], de[3 * i + 1] + c[1], de[3 * i + 2] + c[2]};
                    double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
                    double R = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                    cplx g = std::exp(cplx(0, k * R)) / (4 * kPi * R);
                    cplx gp = g * cplx(-1.0, k * R) / R;
                    double rnx = (r[0] * nx[0] + r[1] * nx[1] + r[2] * nx[2]) / R;
                    Ed(j, i) = g + alpha * gp * rnx;
                }
            }
            Mat St = matmul(lf.Uu[sl], 'C', E, 'N');
            scale_rows(St, lf.su[sl]);
            Mat Tt = matmul(Ed, 'N', lf.Vd[sl], 'N');
            scale_cols(Tt, lf.sd[sl]);
            // slot sl: rows sl ku .. of S~ ((ns ku) x nl, column-major at
            // sop[t]) and columns sl kd .. of T~ (nl x (ns kd) at top[t])
            const size_t so = (size_t)ops.sop[t] + (size_t)sl * lf.ku;
            const size_t to = (size_t)ops.top[t] + (size_t)sl * lf.kd * nl;
            for (int j = 0; j < nl; ++j)
                for (int i = 0; i < lf.ku; ++i)
                    ops.S[so + i + (size_t)j * srows] = (i < St.m) ? St(i, j) : cplx(0);
            for (int j = 0; j < lf.kd; ++j)
                for (int i = 0; i < nl; ++i)
                    ops.T[to + i + (size_t)j * nl] = (j < Tt.n) ? Tt(i, j) : cplx(0);
            if (rhsB) {
                Mat SBt = matmul(lf.Uu[sl], 'C', EB, 'N');
                scale_rows(SBt, lf.su[sl]);
                for (int j = 0; j < nl; ++j)
                    for (int i = 0; i < lf.ku; ++i)
                        ops.SB[so + i + (size_t)j * srows] = (i < SBt.m) ? SBt(i, j) : cplx(0);
            }
        }
    });
}

}  // namespace fda
