// Device-side plan and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace fda {

// Work list of the gathered batched GEMM (k_ggemm) and of its reduction:
// per work item (matrix, first scratch column, column count, 0) and
// kGemmCols source states; per destination state the scratch columns summed
// into it.  tmp holds ncol scratch columns of length m per right-hand side.
// When every destination receives exactly one product, dst lists each
// item's destination states (kGemmCols per item) and the products are
// written to them directly (no scratch, no reduction).
// For many right-hand sides a list with a reduction runs destination-major
// instead (k_ggemm_dest, FP64 plans): per reduction-list entry its (matrix,
// source state), and one unit per wave (destination entry, 16-row tile).
struct GWork {
    int nwork = 0, nred = 0;
    int64_t ncol = 0;
    int4 *hdr = nullptr;
    int32_t *src = nullptr, *dst = nullptr, *rd_dst = nullptr, *rd_off = nullptr, *rd_list = nullptr;
    void *tmp = nullptr;  // storage type of the plan (double2 or float2)
    int2 *dm_ent = nullptr, *dm_units = nullptr;
    int dm_nunits = 0;
};

constexpr int kGemmCols = 32;

// The low-rank M2L of every level runs as one launch (the levels are
// independent once the upward pass is done): one work list whose items carry
// their level, one reduction list that writes every state of those levels
// (an empty list writes zero), and a per-level argument table.
struct M2LLevelArgs {
    const void *U = nullptr, *V = nullptr;  // low-rank factors (storage type): per translation
                                            // U^ kd x rmax, V^ rmax x (ku rounded up to 4)
    const int32_t *rank = nullptr;          // padded rank per translation
    const void *X = nullptr;                // outgoing states s of the level
    void *Y = nullptr;                      // incoming states c of the level
    int64_t xstride = 0, ystride = 0;       // elements per right-hand side
    int64_t tbase = 0;                      // first scratch element of the level
    int32_t kd = 0, ku = 0, rmax = 0, level = 0;
    int32_t ldt = 0;                        // scratch column stride: kd rounded up to a multiple of 4
                                            // (FP64 columns start on 64-byte boundaries)
    int64_t zbase = 0;                      // many-column form: first Z element of the level per
                                            // right-hand side (rmax rows per pair and column)
};
// Right-hand sides from which the merged M2L runs in its many-column form:
// phase 1 stores Z = V^ S per pair, and a destination-major kernel sums
// U^ Z over each incoming state's list on the matrix cores (the columns
// make that product dense), so no kd-row scratch column is written per pair.
// Products at N = 81,920, kD = 100: FP64 8 columns 6.60 ms against 7.10 in
// the per-pair form, 16 columns 11.5 against 14.1; FP32 8 columns 4.29
// against 4.24, 16 columns 7.50 against 8.18.
#ifndef FDA_M2L_MANY_COLS64
#define FDA_M2L_MANY_COLS64 8
#endif
#ifndef FDA_M2L_MANY_COLS32
#define FDA_M2L_MANY_COLS32 16
#endif
constexpr int kM2LManyCols64 = FDA_M2L_MANY_COLS64, kM2LManyCols32 = FDA_M2L_MANY_COLS32;
// Right-hand sides from which M2M / L2L lists with a reduction run
// destination-major (k_ggemm_dest) in FP64 plans.  At N = 81,920, kD = 100:
// 64 columns 36.1 ms per product against 40.4 (M2M 8.9 against 11.3 ms,
// L2L 10.1 against 12.2), 32 columns 19.0 against 20.7; at 16 columns
// 11.1 against 10.9 and at 8 columns 7.7 against 6.3 (half of each 16-column
// tile idle).  FP32 plans keep the staged gathered GEMM: the
// destination-major form was slower at every column count (64 columns: M2M
// 7.5 against 7.1 ms, L2L 8.5 against 7.7).
#ifndef FDA_GEMM_DEST_COLS64
#define FDA_GEMM_DEST_COLS64 32
#endif
constexpr int kGemmDestCols64 = FDA_GEMM_DEST_COLS64;
constexpr int kM2LVariants = 4;  // ring-depth variants of the low-rank M2L kernel
#ifndef FDA_P2P_SHORT_COLS
#define FDA_P2P_SHORT_COLS 1024
#endif
constexpr int kL2TChunk = 2048;  // incoming-state entries of a leaf staged in LDS at a time by L2T
constexpr int kP2PShortCols = FDA_P2P_SHORT_COLS;  // near-field rows up to this length: x staged in LDS
constexpr int kP2PGroup = 16;  // lanes per near-field row in k_p2p
constexpr int kP2PUnroll = 8;  // row loads in flight per lane in k_p2p (4: 0.077 ms, 8: 0.075 ms FP64 at N = 81,920)
constexpr int kP2PItemEntries = 24576;  // near-field block entries per work item (at least 4 rows)

struct M2LMerged {
    int nwork = 0, nred = 0, nlev = 0;
    int variant = 0;                       // kernel variant, 0 .. kM2LVariants - 1
    int64_t nscratch = 0;                  // scratch elements per right-hand side
    int4 *hdr = nullptr;                   // (translation, level-local scratch column, columns, level slot)
    int32_t *src = nullptr;
    int32_t *rd_dst = nullptr, *rd_off = nullptr, *rd_list = nullptr, *rd_lev = nullptr;
    // reduction blocks: level slot q covers blocks rd_block[q] .. rd_block[q + 1]
    // (kRedRows (state, row) entries each) and states rd_state[q] ..
    int32_t *rd_block = nullptr, *rd_state = nullptr;
    int nredblocks = 0;
    // many-column form: per reduction-list entry (pair, translation, rank / 4,
    // 0), per state the sum of its entries' rank / 4, and the units of the
    // destination-major kernel, one per wave (state, row tile, level slot, 0);
    // nzunits = 0 when the form is not available
    int4 *rd_ent = nullptr;
    int32_t *rd_nst = nullptr;
    int4 *zunits = nullptr;
    int nzunits = 0;
    M2LLevelArgs *args = nullptr;          // device table, refreshed with the work buffers
    std::vector<M2LLevelArgs> hargs;
    void *tmp = nullptr;
};

struct DevLevel {
    int64_t nbox = 0;
    int nslot = 1, ku = 0, kd = 0;
    int64_t sstride = 0, cstride = 0;  // elements per right-hand side of s and c
    // operator and state arrays hold the plan's storage type: double2
    // (FP64 plan) or float2 (FP32 plan)
    void *s = nullptr, *c = nullptr;
    // M2L grouped by translation; low-rank factors when rmax > 0
    GWork m2l;
    void *Ulr = nullptr, *Vlr = nullptr;
    int32_t *lr_rank = nullptr;
    int rmax = 0;
    bool merged = false;  // M2L runs in DevPlan::m2l_all
    void *K = nullptr;
    // parent-level operators towards level + 1 and their work lists
    void *M = nullptr, *Lo = nullptr;
    GWork m2m, l2l;
    // the leaves of this level (S2M and L2T): global leaf ids and box indices
    int nleaves = 0;
    int32_t *leaf_ids = nullptr, *leaf_box = nullptr;
};

// The operator-specific parts of the matvec: near-field blocks and leaf S2M
// (the tree, translations and L2T are shared).  DevPlan holds the left-hand
// operator A in its own fields; the right-hand operator B of eq. (eq_bm),
// which acts on Neumann data, is built on request into DevPlan::rhs.
struct NearFar {
    void *nf_vals = nullptr;     // near-field blocks (FP32 plans: self terms zeroed)
    double2 *nf_diag = nullptr;  // FP32 plans: FP64 self terms, tree order
    void *S = nullptr;           // leaf S2M
};

struct DevPlan {
    int64_t n = 0;
    M2LMerged m2l_all;
    int nleaf = 0, depth = 0, top = 0, max_leaf = 0, max_ncol = 0;
    bool has_far = false;
    double k = 0, h_max = 0;
    double2 alpha;
    int32_t *perm = nullptr;
    double *tri = nullptr, *cen = nullptr, *nrm = nullptr, *area = nullptr;
    int64_t *leaf_off = nullptr;
    // near-field work items (leaf, first row, end row, -): p2p_nshort items
    // whose rows have <= kP2PShortCols columns (LDS for p2p_cols_short), then
    // the rest (LDS for max_ncol)
    int4 *p2p_items = nullptr;
    int p2p_nitems = 0, p2p_nshort = 0, p2p_cols_short = 0;
    int32_t *nf_list_off = nullptr, *nf_list = nullptr, *nf_ncol = nullptr, *nf_self_col = nullptr, *nf_cols = nullptr;
    int64_t *nf_blk_off = nullptr, *nf_col_off = nullptr;
    int prec = 0;                   // 0: FP64 storage, 1: FP32 storage
    void *nf_vals = nullptr;        // near-field blocks (FP32 plans: self terms zeroed)
    double2 *nf_diag = nullptr;     // FP32 plans: FP64 self terms, tree order
    void *S = nullptr, *T = nullptr;
    int64_t *leaf_sop = nullptr, *leaf_top = nullptr;  // per leaf: offsets of its S~ and T~
    std::vector<DevLevel> lv;
    // block-Jacobi inverses of the leaf diagonal blocks
    int64_t *bj_off = nullptr;
    float *leaf_scalars = nullptr;  // per leaf: width and largest edge, in wavelengths
    // learned preconditioner rows: chunks of <= 64 consecutive tree
    // positions of one leaf (one row per leaf when n_L <= 64)
    int64_t mlp_nrows = 0;
    int64_t *mlp_row_off = nullptr;  // first tree position of the row
    int32_t *mlp_row_leaf = nullptr; // leaf of the row
    int32_t *mlp_row_n = nullptr;    // elements in the row
    double2 *bj_inv = nullptr;
    // The near field runs on `side`, concurrently with the far-field chain
    // (fork after the permutation of x, join before L2T adds the far field);
    // null: everything on the caller's stream.
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool has_rhs = false;  // B built (fda_options.neumann_rhs)
    NearFar rhs;
};

hipError_t set_quadrature_constants(const double r7b[7][3], const double r7w[7], const double glx[32],
                                    const double glw[32]);
// op 0: A's near-field blocks, op 1: B's
hipError_t launch_near_blocks(const DevPlan &d, double2 *vals64, hipStream_t st, int op = 0);
hipError_t launch_bj_invert(const DevPlan &d, const double2 *vals64, hipStream_t st);
hipError_t launch_near_split(const DevPlan &d, const double2 *vals64, void *out32, double2 *diag, hipStream_t st);
hipError_t launch_to_f32(const double2 *in, void *out, int64_t n, hipStream_t st);
// ev: 7 stage events or null; lev: 2 events per level around its M2L
// product kernel, or null.
// ops: the operator's near field and S2M (null: A's)
hipError_t launch_matvec_tree(const DevPlan &d, const double2 *xt, double2 *yt, int nrhs, hipStream_t st,
                              hipEvent_t *ev, hipEvent_t *lev, const NearFar *ops = nullptr);
// the merged low-rank M2L alone (product kernel and reduction); the
// outgoing states of the merged levels must be current
hipError_t launch_m2l_merged(const DevPlan &d, int nrhs, hipStream_t st);
hipError_t launch_permute_in(const DevPlan &d, const double2 *x, int64_t ld, double2 *xt, int nrhs, hipStream_t st);
hipError_t launch_permute_out(const DevPlan &d, const double2 *yt, double2 *y, int64_t ld, int nrhs, hipStream_t st);
hipError_t launch_rhs_planewave(const DevPlan &d, const double *dirs_dev, int nrhs, double2 *b, int64_t ld,
                                hipStream_t st);
hipError_t launch_multidot(const double2 *V, int m, int nrhs, const double2 *w, int64_t N, double2 *partial,
                           double2 *out, hipStream_t st);
hipError_t launch_multi_axpy(const double2 *V, int m, int nrhs, const double2 *h, double sign, double2 *w, int64_t N,
                             const int32_t *active, hipStream_t st);
hipError_t launch_inv_norm(const double2 *d, double2 *scale, int n, hipStream_t st);
hipError_t launch_scale_cols(const double2 *in, const double2 *scale, double2 *out, int64_t N, int nrhs,
                             hipStream_t st);
hipError_t launch_sub(const double2 *b, const double2 *y, double2 *r, int64_t n, hipStream_t st);
hipError_t launch_bj_apply(const DevPlan &d, const double2 *r, double2 *z, int nrhs, const int32_t *active,
                           hipStream_t st);
hipError_t launch_fill_zero(double2 *p, int64_t n, hipStream_t st);
constexpr int kLowRankMax = 72;  // largest rank the low-rank M2L kernel holds in LDS

// (state, row) entries per block of the merged M2L reduction.
constexpr int kRedRows = 256;

// Blocks used by the two-pass reductions.
constexpr int kRedBlocks = 240;

}  // namespace fda
