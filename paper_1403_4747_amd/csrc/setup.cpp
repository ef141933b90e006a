// Host phase of fda_build (Algorithm, Step 1): geometry, octree, near and
// interaction lists, low/high-frequency regimes, directional cones, the
// equivalent and check point sets, and the truncated SVDs of G_up / G_dn
// (Section 4.1.2, eqs. (eq_svdg)-(eq_invg)).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <numeric>
#include <stdexcept>

#include "plan.hpp"

namespace fda {

static const double kPi = 3.14159265358979323846;

// Radial scale factor of the outgoing equivalent / incoming check cube
// relative to the box half width: the cube just encloses the box (the far
// point sets of directional levels start beyond it).
static const double kRin = 1.05;
static const int kShells = 6, kRings = 8;

cplx green(const double *x, const double *y, double k) {
    double a = x[0] - y[0], b = x[1] - y[1], c = x[2] - y[2];
    double R = std::sqrt(a * a + b * b + c * c);
    return std::exp(cplx(0.0, k * R)) / (4.0 * kPi * R);
}

// ------------------------------------------------------------- helpers

static uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}
static uint64_t morton(int x, int y, int z) { return spread3(x) << 2 | spread3(y) << 1 | spread3(z); }

// Cube-face cell of a direction vector with n x n cells per face.
static int dir_index(const double *d, int n) {
    int a = 0;
    double m = std::fabs(d[0]);
    if (std::fabs(d[1]) > m) { a = 1; m = std::fabs(d[1]); }
    if (std::fabs(d[2]) > m) { a = 2; m = std::fabs(d[2]); }
    int s = d[a] > 0 ? 1 : 0;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double u = d[b] / m, v = d[c] / m;
    int i = std::min(n - 1, std::max(0, (int)std::floor((u + 1) * 0.5 * n)));
    int j = std::min(n - 1, std::max(0, (int)std::floor((v + 1) * 0.5 * n)));
    return ((a * 2 + s) * n + i) * n + j;
}

static void dir_vector(int id, int n, double *out) {
    int j = id % n, i = (id / n) % n, as = id / (n * n);
    int a = as / 2, s = as % 2;
    double d[3];
    d[a] = s ? 1.0 : -1.0;
    d[(a + 1) % 3] = -1.0 + (2.0 * i + 1.0) / n;
    d[(a + 2) % 3] = -1.0 + (2.0 * j + 1.0) / n;
    double l = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int q = 0; q < 3; ++q) out[q] = d[q] / l;
}

// Well-separation test at a level for an integer offset (target - source):
// not adjacent, and on a directional level at least rho apart.
static bool well_separated(const Level &L, const int *d) {
    int m = std::max(std::abs(d[0]), std::max(std::abs(d[1]), std::abs(d[2])));
    if (m < 2) return false;
    if (!L.hf) return true;
    double dist = std::sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]) * L.w;
    return dist >= L.rho * (1.0 - 1e-12);
}

static int64_t floordiv2(int64_t a) { return (a >= 0) ? a / 2 : -((-a + 1) / 2); }

// ------------------------------------------------------------- main

void host_setup(const double *V, int64_t nv, const int32_t *T, int64_t nt, double k, double eps,
                const fda_options &opt, HostPlan &hp) {
    if (!(k > 0) || !std::isfinite(k)) throw BuildError{FDA_EINVAL, "k must be finite and > 0"};
    if (!(eps > 0 && eps < 1)) throw BuildError{FDA_EINVAL, "eps must be in (0, 1)"};
    if (nt <= 0 || nv <= 0 || !V || !T) throw BuildError{FDA_EINVAL, "empty mesh"};
    if (opt.max_leaf < 1 || opt.max_leaf > 256) throw BuildError{FDA_EINVAL, "max_leaf must be in [1, 256]"};
    if (opt.adaptive != 0 && opt.adaptive != 1) throw BuildError{FDA_EINVAL, "adaptive must be 0 or 1"};
    if (!(opt.svd_eps >= 0 && opt.svd_eps < 1) || !(opt.m2l_svd_eps >= 0 && opt.m2l_svd_eps < 1))
        throw BuildError{FDA_EINVAL, "svd_eps and m2l_svd_eps must be in [0, 1)"};
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(V[i])) throw BuildError{FDA_EINVAL, "non-finite vertex coordinate"};
    hp.n = nt;
    hp.k = k;
    hp.eps = eps;
    hp.opt = opt;
    hp.svd_eps = opt.svd_eps > 0 ? opt.svd_eps : eps / 10.0;
    hp.m2l_svd_eps = opt.m2l_svd_eps > 0 ? opt.m2l_svd_eps : hp.svd_eps;
    // i/k for the fluid-side normal, i.e. -i/k for the body-pointing normal n
    hp.alpha = (opt.alpha_re == 0 && opt.alpha_im == 0) ? cplx(0.0, -1.0 / k) : cplx(opt.alpha_re, opt.alpha_im);
    const double lambda = 2.0 * kPi / k;

    // geometry (caller order)
    std::vector<double> cen(3 * nt), nrm(3 * nt), area(nt), emax(nt);
    double h = 0;
    for (int64_t t = 0; t < nt; ++t) {
        for (int q = 0; q < 3; ++q)
            if (T[3 * t + q] < 0 || T[3 * t + q] >= nv) throw BuildError{FDA_EMESH, "vertex index out of range"};
        const double *a = V + 3 * T[3 * t], *b = V + 3 * T[3 * t + 1], *c = V + 3 * T[3 * t + 2];
        double e1[3], e2[3], e3[3];
        for (int q = 0; q < 3; ++q) {
            e1[q] = b[q] - a[q];
            e2[q] = c[q] - a[q];
            e3[q] = c[q] - b[q];
        }
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double ln = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(ln > 0)) throw BuildError{FDA_EMESH, "zero-area triangle " + std::to_string(t)};
        for (int q = 0; q < 3; ++q) {
            cen[3 * t + q] = (a[q] + b[q] + c[q]) / 3.0;
            nrm[3 * t + q] = -cr[q] / ln;
        }
        area[t] = 0.5 * ln;
        emax[t] = std::max(std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]),
                           std::max(std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]),
                                    std::sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2])));
        h = std::max(h, emax[t]);
    }
    hp.h_max = h;

    // root cube: bounding cube of the vertices, expanded slightly
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < nv; ++i)
        for (int q = 0; q < 3; ++q) {
            lo[q] = std::min(lo[q], V[3 * i + q]);
            hi[q] = std::max(hi[q], V[3 * i + q]);
        }
    double side = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2])) * (1.0 + 1e-9);
    if (!(side > 0)) throw BuildError{FDA_EMESH, "degenerate bounding box"};
    for (int q = 0; q < 3; ++q) hp.origin[q] = 0.5 * (lo[q] + hi[q]) - 0.5 * side;
    hp.side = side;

    auto keys_at = [&](int l, int64_t e, int32_t *kk) {
        double w = side / std::ldexp(1.0, l);
        int lim = (1 << l) - 1;
        for (int q = 0; q < 3; ++q) {
            int v = (int)std::floor((cen[3 * e + q] - hp.origin[q]) / w);
            kk[q] = std::min(lim, std::max(0, v));
        }
    };

    // Tree (Algorithm, Step 1.1).  A box is a leaf when it holds at most
    // max_leaf elements or when its children would be narrower than
    // leaf_min_h times the largest edge (near-singular pairs must stay in the
    // near field).  Uniform trees put every leaf on one level: the first on
    // which every box qualifies, with the largest edge of the mesh.  Adaptive
    // trees (Section 3.2) stop subdividing each box as soon as it qualifies,
    // with the largest edge among the box's own elements, so leaves sit on
    // many levels and every box is still at least leaf_min_h of its own
    // largest edges wide.  A leaf may sit on a directional level (Section
    // 3.2, completely adaptive trees): its outgoing and incoming states are
    // then kept per direction slot like those of any box of that level.  A
    // directional box that can still be subdivided is subdivided, even when
    // it holds few elements, since a directional leaf carries one S2M and
    // one L2T operator per slot; it becomes a leaf when its children would
    // be too narrow (coarse meshes at high frequency), and on a uniform tree
    // whose leaf level is directional.
    const double tau = opt.leaf_min_h * h;
    auto width = [&](int l) { return side / std::ldexp(1.0, l); };
    auto hf_width = [&](int l) { return l > 0 && width(l) >= opt.hf_wavelengths * lambda * (1.0 - 1e-9); };
    const bool adaptive = opt.adaptive != 0;
    // boxes per level, Morton ordered: the occupied octants of the boxes of
    // the level above that are subdivided, parent by parent (a child's
    // Morton code is its parent's followed by the octant bits)
    std::vector<int32_t> elev(nt, -1);  // leaf level of each element
    std::vector<int32_t> ebox(nt, 0);   // its box on the current level
    std::vector<uint8_t> eoct(nt, 0);
    hp.lv.clear();
    for (int l = 0;; ++l) {
        hp.lv.emplace_back();
        Level &lv = hp.lv[l];
        lv.w = width(l);
        lv.r = 0.5 * lv.w;
        if (l == 0) {
            lv.nbox = 1;
            lv.key.assign(3, 0);
        } else {
            Level &pv = hp.lv[l - 1];
            std::vector<int32_t> slot(8 * (size_t)pv.nbox, -1);
            for (int64_t e = 0; e < nt; ++e) {
                if (elev[e] >= 0) continue;
                int32_t kk[3];
                keys_at(l, e, kk);
                for (int q = 0; q < 3; ++q)
                    if ((kk[q] >> 1) != pv.key[3 * (size_t)ebox[e] + q])
                        throw BuildError{FDA_EINVAL, "internal: element box is not inside its parent box"};
                eoct[e] = (uint8_t)(((kk[0] & 1) << 2) | ((kk[1] & 1) << 1) | (kk[2] & 1));
                slot[8 * (size_t)ebox[e] + eoct[e]] = 0;
            }
            lv.nbox = 0;
            pv.child_begin.assign(pv.nbox + 1, 0);
            for (int64_t pb = 0; pb < pv.nbox; ++pb) {
                for (int o = 0; o < 8; ++o) {
                    int32_t &s = slot[8 * (size_t)pb + o];
                    if (s < 0) continue;
                    s = (int32_t)lv.nbox++;
                    lv.parent.push_back((int32_t)pb);
                    lv.octant.push_back(o);
                    lv.key.push_back(2 * pv.key[3 * pb] + ((o >> 2) & 1));
                    lv.key.push_back(2 * pv.key[3 * pb + 1] + ((o >> 1) & 1));
                    lv.key.push_back(2 * pv.key[3 * pb + 2] + (o & 1));
                }
                pv.child_begin[pb + 1] = (int32_t)lv.nbox;
            }
            for (int64_t e = 0; e < nt; ++e)
                if (elev[e] < 0) ebox[e] = slot[8 * (size_t)ebox[e] + eoct[e]];
        }
        std::vector<double> hbox(lv.nbox, 0.0);
        lv.nelem.assign(lv.nbox, 0);
        int64_t most = 0;
        for (int64_t e = 0; e < nt; ++e) {
            if (elev[e] >= 0) continue;
            most = std::max(most, ++lv.nelem[ebox[e]]);
            hbox[ebox[e]] = std::max(hbox[ebox[e]], emax[e]);
        }
        // uniform: this is the leaf level when every box qualifies
        const bool uniform_leaves = l >= 20 || lv.w * 0.5 < tau || most <= opt.max_leaf;
        lv.leaf.assign(lv.nbox, -1);
        bool split = false;
        for (int64_t b = 0; b < lv.nbox; ++b) {
            bool leaf;
            if (!adaptive) {
                leaf = uniform_leaves;
            } else {
                // children would be too narrow
                const bool cannot = lv.w * 0.5 < opt.leaf_min_h * hbox[b] || l >= 20;
                leaf = cannot || (lv.nelem[b] <= opt.max_leaf && !hf_width(l));
            }
            if (leaf) lv.leaf[b] = 0;  // marked; numbered below
            else split = true;
        }
        for (int64_t e = 0; e < nt; ++e)
            if (elev[e] < 0 && lv.leaf[ebox[e]] >= 0) elev[e] = l;
        if (!split) break;
    }
    const int L = (int)hp.lv.size() - 1;
    hp.depth = L;
    hp.lv[L].child_begin.assign(hp.lv[L].nbox + 1, 0);

    // leaves in depth-first Morton order: a box's code shifted to the finest
    // level orders boxes of different levels, and the leaves below any box
    // are a contiguous range
    auto dfs_key = [&](int l, int64_t b) {
        const int32_t *kk = &hp.lv[l].key[3 * b];
        return morton(kk[0], kk[1], kk[2]) << (3 * (L - l));
    };
    std::vector<std::pair<uint64_t, std::pair<int32_t, int32_t>>> lk;
    for (int l = 0; l <= L; ++l)
        for (int64_t b = 0; b < hp.lv[l].nbox; ++b)
            if (hp.lv[l].leaf[b] >= 0) lk.push_back({dfs_key(l, b), {l, (int32_t)b}});
    std::sort(lk.begin(), lk.end());
    hp.nleaf = (int64_t)lk.size();
    hp.leaf_level.resize(hp.nleaf);
    hp.leaf_box.resize(hp.nleaf);
    std::vector<uint64_t> leaf_dfs(hp.nleaf);
    for (int64_t t = 0; t < hp.nleaf; ++t) {
        const int l = lk[t].second.first, b = lk[t].second.second;
        hp.leaf_level[t] = l;
        hp.leaf_box[t] = b;
        hp.lv[l].leaf[b] = (int32_t)t;
        hp.lv[l].leaves.push_back((int32_t)t);
        leaf_dfs[t] = lk[t].first;
    }
    // leaves below box b of level l: [first, last)
    auto subtree_leaves = [&](int l, int64_t b) {
        const uint64_t lo = dfs_key(l, b), hi = lo + (1ULL << (3 * (L - l)));
        return std::make_pair(std::lower_bound(leaf_dfs.begin(), leaf_dfs.end(), lo) - leaf_dfs.begin(),
                              std::lower_bound(leaf_dfs.begin(), leaf_dfs.end(), hi) - leaf_dfs.begin());
    };

    // element permutation: by leaf, then caller index
    std::vector<uint64_t> leafcode(nt);
    for (int64_t e = 0; e < nt; ++e) {
        int32_t kk[3];
        keys_at(elev[e], e, kk);
        leafcode[e] = morton(kk[0], kk[1], kk[2]) << (3 * (L - elev[e]));
    }
    std::vector<int32_t> perm(nt);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return leafcode[a] < leafcode[b]; });
    hp.perm = perm;
    {
        hp.leaf_off.assign(hp.nleaf + 1, 0);
        int64_t b = 0;
        for (int64_t i = 0; i < nt; ++i) {
            uint64_t c = leafcode[perm[i]];
            while (leaf_dfs[b] != c) hp.leaf_off[++b] = i;
        }
        while (b < hp.nleaf) hp.leaf_off[++b] = nt;
        hp.max_leaf_count = 0;
        for (int64_t q = 0; q < hp.nleaf; ++q)
            hp.max_leaf_count = std::max<int>(hp.max_leaf_count, (int)(hp.leaf_off[q + 1] - hp.leaf_off[q]));
        // leaves wider than leaf_min_h * h_max may hold more elements than
        // max_leaf on strongly graded meshes; the leaf kernels (block-Jacobi
        // inversion, near-field rows) hold one leaf in a workgroup
        if (hp.max_leaf_count > 256)
            throw BuildError{FDA_EMESH, "a leaf holds " + std::to_string(hp.max_leaf_count) +
                                            " elements (> 256): the mesh is too strongly graded for leaves at least "
                                            "leaf_min_h largest edges wide; lower leaf_min_h or refine the large "
                                            "triangles"};
    }
    hp.tri.resize(9 * nt);
    hp.cen.resize(3 * nt);
    hp.nrm.resize(3 * nt);
    hp.area.resize(nt);
    for (int64_t i = 0; i < nt; ++i) {
        int64_t e = perm[i];
        for (int v = 0; v < 3; ++v)
            for (int q = 0; q < 3; ++q) hp.tri[9 * i + 3 * v + q] = V[3 * T[3 * e + v] + q];
        for (int q = 0; q < 3; ++q) {
            hp.cen[3 * i + q] = cen[3 * e + q];
            hp.nrm[3 * i + q] = nrm[3 * e + q];
        }
        hp.area[i] = area[e];
    }

    // regimes and directions: a level is directional when its boxes are at
    // least hf_wavelengths wide; directional cells per face edge double per
    // level upwards, starting from round(w / lambda) at the finest such level
    int finest_hf = -1;
    for (int l = 0; l <= L; ++l) {
        Level &lv = hp.lv[l];
        lv.hf = lv.w >= opt.hf_wavelengths * lambda * (1.0 - 1e-9) && l > 0;
        if (lv.hf) finest_hf = l;
    }
    if (finest_hf >= 0) {
        int n0 = std::max(1, (int)std::lround(hp.lv[finest_hf].w / lambda));
        for (int l = 0; l <= finest_hf; ++l) {
            Level &lv = hp.lv[l];
            if (!lv.hf) continue;
            lv.nface = n0 << (finest_hf - l);
            lv.ndir = 6 * lv.nface * lv.nface;
            lv.rho = std::max(2.0 * lv.w, opt.rho_c * lv.w * lv.w / lambda);
            lv.dirvec.resize(3 * lv.ndir);
            for (int d = 0; d < lv.ndir; ++d) dir_vector(d, lv.nface, &lv.dirvec[3 * d]);
        }
    }

    // near and interaction lists, top-down (Algorithm, Step 1.2-1.5).  On an
    // adaptive tree a leaf in the near list of a box's parent is coarser than
    // the box's children: it stays in their near lists (near_up) while it
    // touches them, and otherwise its elements act on every leaf below the
    // child directly (the X list of the child, evaluated in the near field).
    // closed boxes b1 (level l1) and b2 (level l2 >= l1) meet
    auto touches = [&](int l1, int64_t b1, int l2, int64_t b2) {
        const int s = l2 - l1;
        for (int q = 0; q < 3; ++q) {
            const int64_t k1 = hp.lv[l1].key[3 * b1 + q], k2 = hp.lv[l2].key[3 * b2 + q];
            if (k2 + 1 < (k1 << s) || k2 > ((k1 + 1) << s)) return false;
        }
        return true;
    };
    struct XEntry {
        int l;
        int32_t b, src;  // box of level l, source leaf
    };
    std::vector<XEntry> xlist;
    hp.lv[0].near.assign(1, std::vector<int32_t>{0});
    hp.lv[0].il.assign(1, {});
    hp.lv[0].il_ops.assign(1, {});
    hp.lv[0].near_up.assign(1, {});
    for (int l = 1; l <= L; ++l) {
        Level &lv = hp.lv[l], &pv = hp.lv[l - 1];
        lv.near.assign(lv.nbox, {});
        lv.il.assign(lv.nbox, {});
        lv.il_ops.assign(lv.nbox, {});
        lv.near_up.assign(lv.nbox, {});
        std::map<std::array<int32_t, 3>, int32_t> opidx;
        for (int64_t b = 0; b < lv.nbox; ++b) {
            int32_t P = lv.parent[b];
            for (int32_t pn : pv.near[P]) {
                if (pv.leaf[pn] >= 0) {
                    if (touches(l - 1, pn, l, b)) lv.near_up[b].push_back(pv.leaf[pn]);
                    else xlist.push_back({l, (int32_t)b, pv.leaf[pn]});
                    continue;
                }
                for (int32_t a = pv.child_begin[pn]; a < pv.child_begin[pn + 1]; ++a) {
                    int d[3] = {lv.key[3 * b] - lv.key[3 * a], lv.key[3 * b + 1] - lv.key[3 * a + 1],
                                lv.key[3 * b + 2] - lv.key[3 * a + 2]};
                    if (well_separated(lv, d)) {
                        std::array<int32_t, 3> key = {d[0], d[1], d[2]};
                        auto it = opidx.find(key);
                        int32_t op;
                        if (it == opidx.end()) {
                            op = (int32_t)lv.offsets.size();
                            opidx[key] = op;
                            lv.offsets.push_back(key);
                            if (lv.hf) {
                                double dv[3] = {(double)d[0], (double)d[1], (double)d[2]};
                                lv.offset_dir.push_back(dir_index(dv, lv.nface));
                            } else {
                                lv.offset_dir.push_back(-1);
                            }
                        } else {
                            op = it->second;
                        }
                        lv.il[b].push_back(a);
                        lv.il_ops[b].push_back(op);
                    } else {
                        lv.near[b].push_back(a);
                    }
                }
            }
            for (int32_t c : pv.near_up[P]) {
                if (touches(hp.leaf_level[c], hp.leaf_box[c], l, b)) lv.near_up[b].push_back(c);
                else xlist.push_back({l, (int32_t)b, c});
            }
        }
    }
    hp.top = L;
    for (int l = 0; l <= L; ++l) {
        bool any = false;
        for (auto &x : hp.lv[l].il)
            if (!x.empty()) { any = true; break; }
        if (any) { hp.top = l; break; }
    }
    hp.far_elem_pairs = 0;
    for (int l = 0; l <= L; ++l) {
        const Level &lv = hp.lv[l];
        for (int64_t b = 0; b < lv.nbox; ++b)
            for (int32_t a : lv.il[b]) hp.far_elem_pairs += lv.nelem[b] * lv.nelem[a];
    }

    // the source leaves each leaf evaluates directly: its U list (touching
    // leaves of any level), its W list (boxes below a same-level neighbour
    // that do not touch it but whose parents do: every leaf below them) and
    // the X entries of its ancestors and itself
    int64_t wbox = 0, wbox_elems = 0, xbox_elems = 0;  // W entries and the elements below them
    {
        std::vector<std::vector<int32_t>> nsrc(hp.nleaf);
        hp.u_pairs = hp.w_pairs = hp.x_pairs = hp.wx_elem_pairs = 0;
        for (int64_t t = 0; t < hp.nleaf; ++t) {
            const int l = hp.leaf_level[t];
            const int32_t b = hp.leaf_box[t];
            const Level &lv = hp.lv[l];
            auto &out = nsrc[t];
            for (int32_t c : lv.near_up[b]) out.push_back(c);
            hp.u_pairs += (int64_t)lv.near_up[b].size();
            std::vector<std::pair<int, int32_t>> stack;
            for (int32_t a : lv.near[b]) {
                if (lv.leaf[a] >= 0) {
                    out.push_back(lv.leaf[a]);
                    ++hp.u_pairs;
                    continue;
                }
                stack.push_back({l, a});
                while (!stack.empty()) {
                    const auto [m, x] = stack.back();
                    stack.pop_back();
                    const Level &mv = hp.lv[m];
                    for (int32_t y = mv.child_begin[x]; y < mv.child_begin[x + 1]; ++y) {
                        if (!touches(l, b, m + 1, y)) {
                            const auto r = subtree_leaves(m + 1, y);
                            for (int64_t s = r.first; s < r.second; ++s) out.push_back((int32_t)s);
                            hp.w_pairs += r.second - r.first;
                            hp.wx_elem_pairs += (hp.leaf_off[t + 1] - hp.leaf_off[t]) *
                                                (hp.leaf_off[r.second] - hp.leaf_off[r.first]);
                            ++wbox;
                            wbox_elems += hp.leaf_off[r.second] - hp.leaf_off[r.first];
                        } else if (hp.lv[m + 1].leaf[y] >= 0) {
                            out.push_back(hp.lv[m + 1].leaf[y]);
                            ++hp.u_pairs;
                        } else {
                            stack.push_back({m + 1, y});
                        }
                    }
                }
            }
        }
        for (const XEntry &x : xlist) {
            const auto r = subtree_leaves(x.l, x.b);
            for (int64_t t = r.first; t < r.second; ++t) nsrc[t].push_back(x.src);
            hp.x_pairs += r.second - r.first;
            hp.wx_elem_pairs += (hp.leaf_off[r.second] - hp.leaf_off[r.first]) *
                                (hp.leaf_off[x.src + 1] - hp.leaf_off[x.src]);
            xbox_elems += hp.leaf_off[r.second] - hp.leaf_off[r.first];
        }
        hp.nf_list_off.assign(hp.nleaf + 1, 0);
        hp.nf_blk_off.assign(hp.nleaf + 1, 0);
        hp.nf_ncol.assign(hp.nleaf, 0);
        hp.nf_list.clear();
        for (int64_t t = 0; t < hp.nleaf; ++t) {
            auto &nl = nsrc[t];
            std::sort(nl.begin(), nl.end());
            if (std::adjacent_find(nl.begin(), nl.end()) != nl.end())
                throw BuildError{FDA_EINVAL, "internal: a leaf pair is listed twice"};
            int64_t ncol = 0;
            for (int32_t s : nl) {
                hp.nf_list.push_back(s);
                ncol += hp.leaf_off[s + 1] - hp.leaf_off[s];
            }
            hp.nf_list_off[t + 1] = (int64_t)hp.nf_list.size();
            hp.nf_ncol[t] = (int32_t)ncol;
            hp.nf_blk_off[t + 1] = hp.nf_blk_off[t] + ncol * (hp.leaf_off[t + 1] - hp.leaf_off[t]);
            std::vector<int32_t>().swap(nl);
        }
        hp.near_nnz = hp.nf_blk_off[hp.nleaf];
    }

    // active directions, top-down: those used by interaction lists, plus the
    // child cells of the parent's active directions (needed by M2M / L2L)
    for (int l = 0; l <= L; ++l) {
        Level &lv = hp.lv[l];
        if (!lv.hf) {
            lv.active = {0};
            lv.slot_of_dir = {0};
            lv.nslot = 1;
            continue;
        }
        std::vector<char> used(lv.ndir, 0);
        for (int32_t op = 0; op < (int32_t)lv.offsets.size(); ++op) used[lv.offset_dir[op]] = 1;
        if (l > 0 && hp.lv[l - 1].hf && l - 1 >= hp.top) {
            Level &pv = hp.lv[l - 1];
            for (int32_t d : pv.active) used[dir_index(&pv.dirvec[3 * d], lv.nface)] = 1;
        }
        lv.active.clear();
        lv.slot_of_dir.assign(lv.ndir, -1);
        for (int d = 0; d < lv.ndir; ++d)
            if (used[d]) {
                lv.slot_of_dir[d] = (int32_t)lv.active.size();
                lv.active.push_back(d);
            }
        lv.nslot = std::max<int>(1, (int)lv.active.size());
        if (lv.active.empty()) lv.active = {0}, lv.slot_of_dir[0] = 0;
    }

    // orbits of the active directions under the cube's symmetries (Section
    // 3.1: the directional point sets and translations are rotations of one
    // another).  The directions are the cell centres of an n x n grid on
    // each cube face, a set the 48 symmetries permute; each orbit's
    // representative is its first active direction, and every slot keeps
    // the symmetry that carries the representative's direction onto its own.
    for (int l = 0; l <= L; ++l) {
        Level &lv = hp.lv[l];
        lv.rep_slot.assign(lv.nslot, 0);
        lv.sym.assign(lv.nslot, 0);
        if (!lv.hf) continue;
        for (int s = 0; s < lv.nslot; ++s) {
            lv.rep_slot[s] = s;
            const double *u = &lv.dirvec[3 * lv.active[s]];
            for (int g = 0; g < kCubeSyms && lv.rep_slot[s] == s; ++g) {
                double w[3];
                cube_sym_apply_inv(g, u, w);  // a direction that g carries onto u
                const int r = lv.slot_of_dir[dir_index(w, lv.nface)];
                if (r >= 0 && r < s && lv.rep_slot[r] == r) {
                    lv.rep_slot[s] = r;
                    lv.sym[s] = g;
                }
            }
        }
    }

    // far point sets of the directional levels (top-down), Section 3.1:
    // a circular cone around +z whose half angle covers every possible
    // interaction-list target box and the parent's cone, from the nearest
    // such point to beyond the size of the whole mesh; points are spread on
    // geometrically spaced shells (denser at the near end).
    const double tmax = std::sqrt(3.0) * side * 1.05;
    for (int l = std::max(hp.top, 1); l <= L; ++l) {
        Level &lv = hp.lv[l];
        if (!lv.hf) continue;
        const Level &pv = hp.lv[l - 1];
        int R = std::min((1 << l) - 1, 24);
        double th = 0, tm = 1e300;
        double corner = kRin * lv.r;
        for (int x = -R; x <= R; ++x)
            for (int y = -R; y <= R; ++y)
                for (int z = -R; z <= R; ++z) {
                    int d[3] = {x, y, z};
                    if (!well_separated(lv, d)) continue;
                    bool possible = false;
                    for (int s = 0; s < 8 && !possible; ++s) {
                        int sb[3] = {(s >> 2) & 1, (s >> 1) & 1, s & 1};
                        int dp[3];
                        for (int q = 0; q < 3; ++q) dp[q] = (int)floordiv2(sb[q] + d[q]);
                        if (!well_separated(pv, dp)) possible = true;
                    }
                    if (!possible) continue;
                    double dv[3] = {(double)x, (double)y, (double)z};
                    int di = dir_index(dv, lv.nface);
                    const double *u = &lv.dirvec[3 * di];
                    for (int c = 0; c < 8; ++c) {
                        double P[3] = {x * lv.w + ((c & 4) ? corner : -corner), y * lv.w + ((c & 2) ? corner : -corner),
                                       z * lv.w + ((c & 1) ? corner : -corner)};
                        double pn = std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
                        double ca = (P[0] * u[0] + P[1] * u[1] + P[2] * u[2]) / pn;
                        th = std::max(th, std::acos(std::max(-1.0, std::min(1.0, ca))));
                        tm = std::min(tm, pn);
                    }
                }
        if (pv.hf && l - 1 >= hp.top && pv.theta > 0) {
            double off = std::sqrt(3.0) * lv.r;
            for (int32_t dp : pv.active) {
                const double *up = &pv.dirvec[3 * dp];
                const double *uc = &lv.dirvec[3 * dir_index(up, lv.nface)];
                double ca = up[0] * uc[0] + up[1] * uc[1] + up[2] * uc[2];
                double a = std::acos(std::max(-1.0, std::min(1.0, ca))) + pv.theta +
                           std::asin(std::min(1.0, off / pv.tmin));
                th = std::max(th, a);
            }
            tm = std::min(tm, pv.tmin - off);
        }
        if (tm == 1e300) { th = 0.5; tm = lv.rho; }
        if (!(th < 0.95 * kPi) || !(tm > 1.5 * kRin * lv.r * std::sqrt(3.0)))
            throw BuildError{FDA_EINVAL, "directional cone of level " + std::to_string(l) +
                                             " is too wide; raise hf_wavelengths or rho_c"};
        lv.theta = th;
        lv.tmin = tm;
        lv.far.clear();
        for (int si = 0; si < kShells; ++si) {
            double ts = tm * std::pow(tmax / tm, (double)si / (kShells - 1));
            for (int a = 0; a < kRings; ++a) {
                double ta = th * a / (kRings - 1);
                int m = (a == 0) ? 1 : std::max(1, (int)std::lround(2 * kPi * std::sin(ta) / (th / (kRings - 1))));
                for (int b = 0; b < m; ++b) {
                    double ph = 2 * kPi * b / m;
                    lv.far.push_back(ts * std::sin(ta) * std::cos(ph));
                    lv.far.push_back(ts * std::sin(ta) * std::sin(ph));
                    lv.far.push_back(ts * std::cos(ta));
                }
            }
        }
    }

    // number the distinct offsets of each level slot by slot, so that the
    // reduced M2L matrices of one direction are contiguous
    for (int l = 0; l <= L; ++l) {
        Level &lv = hp.lv[l];
        const size_t no = lv.offsets.size();
        if (no == 0) continue;
        std::vector<int32_t> ord(no);
        std::iota(ord.begin(), ord.end(), 0);
        auto slot = [&](int32_t o) { return lv.hf ? lv.slot_of_dir[lv.offset_dir[o]] : 0; };
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return slot(a) < slot(b); });
        std::vector<int32_t> newidx(no);
        std::vector<std::array<int32_t, 3>> offs(no);
        std::vector<int32_t> odir(no);
        for (size_t q = 0; q < no; ++q) {
            newidx[ord[q]] = (int32_t)q;
            offs[q] = lv.offsets[ord[q]];
            odir[q] = lv.offset_dir[ord[q]];
        }
        lv.offsets.swap(offs);
        lv.offset_dir.swap(odir);
        for (auto &ops : lv.il_ops)
            for (auto &o : ops) o = newidx[o];
    }

    // translations shared by symmetry: on a directional level the reduced
    // M2L matrix of offset t in slot s equals that of offset g^-1 t in the
    // representative slot (g = sym[s]), since both the point sets and the
    // SVD factors of slot s are the representative's carried over by g; the
    // level keeps one translation per distinct (g^-1 t, representative),
    // numbered representative by representative
    for (int l = 0; l <= L; ++l) {
        Level &lv = hp.lv[l];
        lv.il_slots.assign(lv.nbox, {});
        for (int64_t b = 0; b < lv.nbox; ++b)
            for (int32_t op : lv.il_ops[b]) lv.il_slots[b].push_back(lv.hf ? lv.slot_of_dir[lv.offset_dir[op]] : 0);
        if (!lv.hf || lv.offsets.empty()) continue;
        const size_t no = lv.offsets.size();
        std::map<std::pair<int32_t, std::array<int32_t, 3>>, int32_t> canon;
        std::vector<std::pair<int32_t, std::array<int32_t, 3>>> keys;
        std::vector<int32_t> cidx(no);
        for (size_t o = 0; o < no; ++o) {
            const int s = lv.slot_of_dir[lv.offset_dir[o]];
            const double t[3] = {(double)lv.offsets[o][0], (double)lv.offsets[o][1], (double)lv.offsets[o][2]};
            double tc[3];
            cube_sym_apply_inv(lv.sym[s], t, tc);
            const std::pair<int32_t, std::array<int32_t, 3>> key = {
                lv.rep_slot[s], {(int32_t)std::lround(tc[0]), (int32_t)std::lround(tc[1]), (int32_t)std::lround(tc[2])}};
            auto it = canon.find(key);
            if (it == canon.end()) {
                it = canon.emplace(key, (int32_t)keys.size()).first;
                keys.push_back(key);
            }
            cidx[o] = it->second;
        }
        // number the distinct translations by representative slot
        std::vector<int32_t> ord(keys.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return keys[a].first < keys[b].first; });
        std::vector<int32_t> pos(keys.size());
        std::vector<std::array<int32_t, 3>> offs(keys.size());
        std::vector<int32_t> odir(keys.size());
        for (size_t q = 0; q < ord.size(); ++q) {
            pos[ord[q]] = (int32_t)q;
            offs[q] = keys[ord[q]].second;
            odir[q] = lv.active[keys[ord[q]].first];
        }
        lv.offsets.swap(offs);
        lv.offset_dir.swap(odir);
        for (auto &ops : lv.il_ops)
            for (auto &o : ops) o = pos[cidx[o]];
    }

    // child slot of every slot (M2M source, L2L target) and its inverse
    for (int l = std::max(hp.top, 0); l < L; ++l) {
        Level &P = hp.lv[l];
        const Level &C = hp.lv[l + 1];
        P.cslot.assign(P.nslot, 0);
        if (C.hf)
            for (int s = 0; s < P.nslot; ++s) {
                int d = dir_index(&P.dirvec[3 * P.active[s]], C.nface);
                P.cslot[s] = C.slot_of_dir[d];
                if (P.cslot[s] < 0) throw BuildError{FDA_EINVAL, "internal: inactive child direction"};
            }
        P.l2l_off.assign(C.nslot + 1, 0);
        P.l2l_src.clear();
        for (int cs = 0; cs < C.nslot; ++cs) {
            for (int s = 0; s < P.nslot; ++s)
                if (P.cslot[s] == cs) P.l2l_src.push_back(s);
            P.l2l_off[cs + 1] = (int32_t)P.l2l_src.size();
        }
    }

    if (opt.verbose) {
        for (int l = 0; l <= L; ++l) {
            const Level &lv = hp.lv[l];
            int64_t pairs = 0;
            for (auto &x : lv.il) pairs += (int64_t)x.size();
            fprintf(stderr, "[fda] level %d w=%.4g (%.2f lambda) %s boxes=%lld pairs=%lld offsets=%zu dirs=%d/%d p=%d ku=%d theta=%.3f tmin/w=%.3f nfar=%zu\n",
                    l, lv.w, lv.w / lambda, lv.hf ? "HF" : "LF", (long long)lv.nbox, (long long)pairs, lv.offsets.size(),
                    lv.hf ? (int)lv.active.size() : 0, lv.ndir, lv.p, lv.ku, lv.theta, lv.tmin / lv.w, lv.far.size() / 3);
        }
        fprintf(stderr, "[fda] depth=%d top=%d leaves=%lld max_leaf=%d near_nnz=%lld h_max=%.4g\n", hp.depth, hp.top,
                (long long)hp.nleaf, hp.max_leaf_count, (long long)hp.near_nnz, hp.h_max);
        if (adaptive)
            fprintf(stderr,
                    "[fda] adaptive: U leaf pairs=%lld, W boxes=%lld (%.1f elements each, %lld leaf pairs), "
                    "X entries=%zu (%.1f elements below each box, %lld leaf pairs)\n",
                    (long long)hp.u_pairs, (long long)wbox, wbox ? (double)wbox_elems / wbox : 0.0,
                    (long long)hp.w_pairs, xlist.size(), xlist.empty() ? 0.0 : (double)xbox_elems / xlist.size(),
                    (long long)hp.x_pairs);
    }
}

void fill_stats(const HostPlan &hp, fda_stats *st) {
    std::memset(st, 0, sizeof(*st));
    st->n = hp.n;
    st->depth = hp.depth;
    st->top_level = hp.top;
    st->nleaf = hp.nleaf;
    st->u_pairs = hp.u_pairs;
    st->w_pairs = hp.w_pairs;
    st->x_pairs = hp.x_pairs;
    st->far_elem_pairs = hp.far_elem_pairs;
    st->wx_elem_pairs = hp.wx_elem_pairs;
    for (int32_t c : hp.nf_ncol) st->max_near_cols = std::max<int64_t>(st->max_near_cols, c);
    st->max_leaf_count = hp.max_leaf_count;
    st->near_nnz = hp.near_nnz;
    st->h_max = hp.h_max;
    st->root_width = hp.side;
    int64_t flops = 0, bytes = 0;
    for (int l = 0; l <= hp.depth && l < 24; ++l) {
        const Level &lv = hp.lv[l];
        st->boxes[l] = lv.nbox;
        st->leaves[l] = (int64_t)lv.leaves.size();
        int64_t pairs = 0;
        for (auto &x : lv.il) pairs += (int64_t)x.size();
        st->m2l_pairs[l] = pairs;
        st->m2l_offsets[l] = (int64_t)lv.offsets.size();
        st->hf[l] = lv.hf ? 1 : 0;
        st->ndir[l] = lv.ndir;
        st->active_dirs[l] = lv.hf ? (int)lv.active.size() : 0;
        st->p[l] = lv.p;
        st->rank_up[l] = lv.ku;
        st->rank_dn[l] = lv.kd;
        flops += pairs * 8LL * lv.ku * lv.kd;
        bytes += (int64_t)lv.offsets.size() * 16LL * lv.ku * lv.kd;
    }
    st->m2l_flops = flops;
    st->m2l_bytes = bytes;
}

}  // namespace fda
