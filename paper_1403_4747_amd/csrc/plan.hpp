// Internal plan of the fast directional BEM: host-side tree, lists and
// operators (built once by fda_build), plus the device buffers the matvec
// kernels read.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fda.h"
#include "linalg.hpp"

namespace fda {

// Per-level host data (Algorithm, Step 1).
struct Level {
    double w = 0, r = 0;        // box width and half width
    bool hf = false;            // directional (high-frequency) level
    int nface = 0;              // directional cells per cube-face edge
    int ndir = 0;               // 6 * nface^2 directions (0 for a non-directional level)
    double rho = 0;             // far distance of a directional level
    int64_t nbox = 0;
    std::vector<int32_t> key;   // 3 per box, integer box coordinates
    std::vector<int32_t> parent, octant;  // parent box index and child octant (bit 2: x, 1: y, 0: z)
    std::vector<int32_t> child_begin;     // children of box b are [child_begin[b], child_begin[b+1]) at level+1
    std::vector<int32_t> leaf;            // global leaf id of each box, -1 for a box that is subdivided
    std::vector<int64_t> nelem;           // elements in each box
    std::vector<int32_t> leaves;          // global ids of the leaves at this level, ascending
    std::vector<std::vector<int32_t>> near, il;  // near list and interaction list (sources) per box
    std::vector<std::vector<int32_t>> near_up;   // coarser leaves adjacent to the box (global leaf ids)
    std::vector<int32_t> il_op;           // per (box, il entry) flattened: distinct-offset index
    std::vector<std::vector<int32_t>> il_ops;  // per (box, il entry): translation index
    std::vector<std::vector<int32_t>> il_slots;  // per (box, il entry): direction slot of the pair
    std::vector<std::array<int32_t, 3>> offsets;  // distinct offsets (target - source) of this level
    std::vector<int32_t> offset_dir;      // direction of each distinct offset (-1 when non-directional)
    // directional bookkeeping
    std::vector<int32_t> active;          // active direction ids (slot -> dir)
    std::vector<int32_t> slot_of_dir;     // dir -> slot or -1
    std::vector<double> dirvec;           // 3 per direction
    int nslot = 1;
    // compressed representation
    int p = 0;                  // points per cube edge
    int ku = 0, kd = 0;         // padded compressed ranks (outgoing / incoming)
    std::vector<double> cube;   // unit cube-surface points (3 each)
    double theta = 0, tmin = 0; // directional check cone half-angle and near end
    std::vector<double> far;    // canonical (+z) far point set (3 each)
    // per slot (one slot on non-directional levels)
    std::vector<Mat> Uu, Vu, Ud, Vd;
    std::vector<std::vector<double>> su, sd;
    std::vector<int> ku_s, kd_s;
    // towards level + 1: child slot of each slot, and the slots feeding each child slot
    std::vector<int32_t> cslot, l2l_off, l2l_src;
    // directional levels: the slots fall into orbits of the cube's symmetry
    // group; each slot's check set, SVD factors and translations are those
    // of its orbit's representative slot carried over by one symmetry
    // (Section 3.1, rotational invariance): rep_slot[s] and sym[s] with
    // cube_sym(sym[s]) mapping the representative's direction to slot s's
    std::vector<int32_t> rep_slot, sym;
};

// The 48 symmetries of the cube (signed permutations of the axes): symmetry
// g = 8 q + b takes v to w with w[a] = (bit a of b ? -1 : 1) v[perm_q[a]].
constexpr int kCubeSyms = 48;
inline void cube_sym_apply(int g, const double *v, double *w) {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int *pq = perm[g / 8];
    for (int a = 0; a < 3; ++a) w[a] = ((g >> a) & 1 ? -1.0 : 1.0) * v[pq[a]];
}
// the inverse (transpose) of cube_sym_apply(g)
inline void cube_sym_apply_inv(int g, const double *w, double *v) {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int *pq = perm[g / 8];
    for (int a = 0; a < 3; ++a) v[pq[a]] = ((g >> a) & 1 ? -1.0 : 1.0) * w[a];
}

struct HostPlan {
    int64_t n = 0;
    double k = 0, eps = 0, svd_eps = 0, m2l_svd_eps = 0;
    cplx alpha;
    fda_options opt{};
    double h_max = 0;
    double origin[3] = {0, 0, 0};
    double side = 0;
    int depth = 0, top = 0;      // finest level, coarsest level with interactions
    std::vector<Level> lv;
    // geometry in tree order
    std::vector<int32_t> perm;   // tree index -> caller index
    std::vector<double> tri;     // 9 doubles per element (vertices), tree order
    std::vector<double> cen, nrm, area;  // tree order
    std::vector<int64_t> leaf_off;       // element range of each leaf
    int64_t nleaf = 0;                   // leaves at every level, in depth-first Morton order
    std::vector<int32_t> leaf_level, leaf_box;  // level and box index of each leaf
    int max_leaf_count = 0;
    // adaptive trees: leaf pairs evaluated directly because one box of the
    // pair is a leaf coarser than the other (U list across levels, W and X
    // lists), and element pairs covered by interaction lists (all levels)
    int64_t u_pairs = 0, w_pairs = 0, x_pairs = 0;
    int64_t far_elem_pairs = 0;
    int64_t wx_elem_pairs = 0;  // near-field entries that come from W and X pairs
    // near field: per target leaf, the source leaves evaluated directly
    std::vector<int64_t> nf_list_off;    // nleaf + 1
    std::vector<int32_t> nf_list;        // near source leaves
    std::vector<int64_t> nf_blk_off;     // nleaf + 1: value offset of each target block
    std::vector<int32_t> nf_ncol;        // columns of each target block
    int64_t near_nnz = 0;
    int cslot_of(int l, int s) const { return lv[l].cslot.empty() ? 0 : lv[l].cslot[s]; }
};

// Host phase of the build: geometry, octree, lists, directions and the
// directional far point sets.  Throws BuildError on failure.
struct BuildError {
    int code;
    std::string msg;
};

void host_setup(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k, double eps,
                const fda_options &opt, HostPlan &hp);
void fill_stats(const HostPlan &hp, fda_stats *st);

// Kernel evaluations shared by the host operator formation.
cplx green(const double *x, const double *y, double k);

}  // namespace fda
