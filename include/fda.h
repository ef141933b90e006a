/*
 * fda.h -- C ABI of the MI355X fast directional BEM library (libfda.so).
 *
 * The library applies and solves the collocation Burton-Miller system of a
 * rigid (sound-hard) closed surface meshed with flat triangles and
 * piecewise-constant elements (Cao, Wen, Xiao, "A fast directional boundary
 * element method for high frequency acoustic problems in three dimensions",
 * Section 2 eqs. (eq_bm), (eq_sum) and Section 5):
 *
 *   (A u)_i = u_i / 2 + sum_j int_{D_j} [ dG/dn_y + alpha d2G/dn_x dn_y ](c_i, y) dy u_j
 *
 * with G = exp(ikR)/(4 pi R), c_i the centroid of triangle i and n the normal
 * pointing into the body (the triangles are wound counter-clockwise seen from
 * the fluid).  Far interactions are evaluated by the fast directional
 * algorithm of Section 3 (upward pass, M2L, downward pass, near field;
 * Algorithm, Steps 1-4) with the compressed translations of Section 4
 * (eqs. (eq_svdg)-(eq_cmpm2l), (eq_epsk) and the compressed S2M, M2M, L2L,
 * L2T matrices of Section 4.3).
 *
 * Conventions for every entry point:
 *   - Return 0 on success, a negative FDA_E* code on error, or (bm_solve
 *     only) the positive FDA_NOTCONV.  fda_last_error() then returns a
 *     thread-local message describing the failure.
 *   - Complex vectors are complex128, interleaved (re, im), column-major
 *     with leading dimension ld >= N (in elements), in the caller's element
 *     order (the library permutes internally).
 *   - Pointers named *_dev are device pointers on the plan's device; all
 *     other pointers are host pointers.  The library never takes ownership
 *     of caller buffers.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *   - Every entry point needs the GPU except fda_inspect, fda_plan_leaves
 *     and the two version / error helpers.
 *   - A plan keeps one set of work buffers (tree-order vectors, level
 *     states, one scratch buffer shared by the M2M / M2L / L2L products):
 *     calls on one plan must not overlap in time (issue them on one stream
 *     or synchronise between streams).
 */
#ifndef FDA_H
#define FDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDA_OK 0
#define FDA_EINVAL (-1)      /* bad argument: non-finite, k <= 0, eps outside (0,1), nrhs out of range */
#define FDA_EMESH (-2)       /* zero-area triangle or vertex index out of range */
#define FDA_ENOMEM (-3)      /* host or device allocation failed */
#define FDA_EHIP (-4)        /* a HIP / rocBLAS call failed */
#define FDA_EBREAKDOWN (-5)  /* GMRES breakdown or a non-finite value */
#define FDA_NOTCONV 1        /* bm_solve: maximum iterations reached (x holds the best iterate) */

/* Precision of the far-field translations and the near-field product. */
#define FDA_PREC_FP64 0
#define FDA_PREC_FP32 1

/* Preconditioners for bm_solve. */
#define FDA_PRECOND_NONE 0
#define FDA_PRECOND_BLOCK_JACOBI 1
#define FDA_PRECOND_MLP 2          /* learned per-leaf correction on top of block Jacobi (fda_plan_set_mlp) */

/* Shape of the learned preconditioner's rows (see fda_mlp_samples). */
#define FDA_MLP_IN 272
#define FDA_MLP_OUT 128

typedef struct fda_plan fda_plan;
typedef struct fda_mlp fda_mlp;
typedef struct fda_batch fda_batch;

/* Build options.  Zero-initialise and call fda_default_options(), then
 * override fields.  Every field has a documented default. */
typedef struct fda_options {
    int32_t max_leaf;      /* leaf capacity (elements per leaf box), default 64 */
    int32_t p_min;         /* smallest points per cube edge; 0 = ceil(log10(1/eps)) + p0 (Section 5.1) */
    int32_t p0;            /* the paper's p0, default 1 */
    double svd_eps;        /* SVD truncation threshold (eqs. (eq_epsg), (eq_epsk)); 0 = eps / 10 */
    double alpha_re;       /* Burton-Miller coupling in the body-pointing normal convention;
                              alpha_re = alpha_im = 0 selects -i/k, which is the coupling i/k of
                              Section 2 written for the fluid-side normal */
    double alpha_im;
    double hf_wavelengths; /* a box is high-frequency (directional) when its width >= this many
                              wavelengths, default 1.9 */
    double rho_c;          /* high-frequency far distance max(2w, rho_c w^2 / lambda), default 1 */
    double leaf_min_h;     /* leaves are at least this many largest-edges wide, default 2.5 */
    int32_t prec;          /* FDA_PREC_FP64 (default) or FDA_PREC_FP32 */
    int32_t nrhs_max;      /* largest nrhs accepted by fda_matvec / bm_solve, default 64 */
    int32_t device;        /* HIP device ordinal, default 0 */
    int32_t verbose;       /* print build statistics to stderr, default 0 */
    int32_t svd_method;    /* batched SVDs of the build (eqs. (eq_svdg), (eq_epsk)): 0 = bidiagonal QR
                              (rocSOLVER gesvd), 1 = one-sided Jacobi (gesvdj); default 1 (the
                              same ranks, a faster build) */
    double m2l_svd_eps;    /* truncation of the reduced M2L matrices alone (eq. (eq_epsk));
                              0 = svd_eps */
    int32_t neumann_rhs;   /* also build the right-hand operator B of eq. (eq_bm) for Neumann data
                              (bm_rhs_neumann): its near-field blocks and leaf S2M; default 0 */
    int32_t adaptive;      /* 0 (default): uniform tree, every leaf on the first level on which
                              all boxes qualify as leaves; 1: adaptive tree (Section 3.2), each box
                              a leaf as soon as it holds <= max_leaf elements (or its children
                              would be narrower than leaf_min_h largest edges), so leaves sit on
                              many levels.  Leaves are never directional: a directional box is
                              always subdivided.  Leaf pairs whose boxes lie on different levels
                              and are not separated by an interaction list (the U, W and X lists
                              of adaptive FMMs) are evaluated directly in the near field. */
    int32_t p_fixed;       /* 0 (default): p starts at p_min (or ceil(log10(1/eps)) + p0) and is raised
                              per level until the numerical rank of G_up uses at most 70 % of the
                              cube points; 1: that starting p on every level (Section 5.1's
                              p = log(1/eps) + p0 as printed) */
} fda_options;

/* Plan statistics (filled by fda_inspect / fda_plan_stats). */
typedef struct fda_stats {
    int64_t n;                  /* triangles */
    int32_t depth;              /* finest level (the leaf level of a uniform tree) */
    int32_t top_level;          /* coarsest level with interactions */
    int64_t nleaf;              /* non-empty leaves, all levels */
    int32_t max_leaf_count;     /* most elements in one leaf */
    int64_t near_nnz;           /* entries of the near-field block matrix */
    int64_t boxes[24];          /* non-empty boxes per level */
    int64_t m2l_pairs[24];      /* interaction-list (target, source) pairs per level */
    int64_t m2l_offsets[24];    /* distinct translations per level */
    int32_t hf[24];             /* 1 if the level is directional */
    int32_t ndir[24];           /* directions per level (0 for non-directional) */
    int32_t active_dirs[24];    /* directions that carry data */
    int32_t p[24];              /* points per cube edge per level */
    int32_t rank_up[24];        /* outgoing compressed rank per level (max over directions) */
    int32_t rank_dn[24];        /* incoming compressed rank per level */
    int32_t m2l_rank_max[24];   /* low-rank M2L: largest rank per level (0 = full reduced matrices) */
    double m2l_rank_mean[24];   /* low-rank M2L: mean numerical rank per level */
    double m2l_level_flops[24]; /* real flops of the M2L products per level, per right-hand side */
    int64_t m2l_flops;          /* real flops of one M2L pass per right-hand side */
    int64_t m2l_bytes;          /* bytes of the distinct reduced M2L matrices */
    double h_max;               /* largest mesh edge */
    double root_width;
    double build_seconds;       /* wall time of the last build (0 for fda_inspect) */
    int64_t device_bytes;       /* device memory held by the plan */
    double m2m_flops;           /* real flops of one upward pass (M2M, all levels, 8 per complex
                                   multiply-add) */
    double l2l_flops;           /* the same for the downward pass (L2L) */
    int64_t mlp_rows;           /* rows of the learned preconditioner: chunks of <= 64 consecutive
                                   elements of a leaf (see fda_mlp_samples) */
    double build_phase_seconds[8]; /* fda_build wall time by phase: tree and lists (host), factors of
                                      G_up / G_dn, translation matrices, low-rank M2L factors, leaf
                                      operators (host), upload, near-field quadrature; [7] unused */
    int64_t leaves[24];         /* leaves per level */
    int64_t u_pairs;            /* leaf pairs evaluated directly because the leaves touch (U lists) */
    int64_t w_pairs;            /* leaf pairs below a touching box that the target leaf does not touch
                                   (W lists; zero on uniform trees) */
    int64_t x_pairs;            /* leaf pairs from a coarser source leaf that does not touch the target
                                   (X lists; zero on uniform trees) */
    int64_t far_elem_pairs;     /* element pairs covered by interaction lists (M2L); every ordered
                                   element pair is covered once: near_nnz + far_elem_pairs = n^2 */
    int64_t max_near_cols;      /* longest near-field row (source elements of one leaf) */
    int64_t wx_elem_pairs;      /* entries of near_nnz that come from W and X pairs */
    int64_t m2l_factor_bytes;   /* low-rank M2L levels: bytes of the distinct factors U^ (kd x r) and
                                   V^ (r x ku) at the unpadded SVD ranks, in the plan's storage type */
    int64_t m2l_state_bytes;    /* low-rank M2L levels: bytes of the outgoing states read and the
                                   incoming states written by one pass, per right-hand side; with
                                   m2l_factor_bytes the pass's algorithmic traffic */
} fda_stats;

/* Fill *opt with the defaults listed above. */
void fda_default_options(fda_options *opt);

/* Build a plan for mesh (verts: nv x 3 doubles, tris: nt x 3 int32, 0-based),
 * wavenumber k > 0 and compression threshold eps in (0, 1) (Algorithm,
 * Step 1; Section 4).  opt may be NULL for the defaults.  The mesh is copied;
 * the plan owns all device memory and is released by fda_free.  Errors:
 * FDA_EINVAL, FDA_EMESH, FDA_ENOMEM, FDA_EHIP; *out is NULL on error. */
int fda_build(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k, double eps,
              const fda_options *opt, fda_plan **out);

/* Host-only dry run of fda_build's tree, list and point-set phase (no GPU
 * needed): fills *st with the counts a build would have.  Same errors. */
int fda_inspect(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k, double eps,
                const fda_options *opt, fda_stats *st);

/* y = A x for nrhs columns (Algorithm, Steps 2-4: upward pass, M2L,
 * downward pass, near field).  x_dev, y_dev: N x nrhs complex128 device
 * buffers with leading dimension ld (elements); x is not modified; x and y
 * must not overlap.  Asynchronous on stream: the near field may run on a
 * stream the plan owns, concurrently with the far field, but it is ordered
 * after the work already on `stream` and the product completes on `stream`
 * (while `stream` is being captured into a graph everything stays on it).
 * From 8 columns (FP64 plans; 16 in FP32 plans) the low-rank M2L sums its
 * terms per incoming state in another order (and, from 32 columns in FP64
 * plans, so do M2M and L2L), so a column of such a product equals the
 * single-column product to rounding, not bit for bit; a given nrhs always
 * gives the same bits.
 * Errors: FDA_EINVAL (nrhs < 1, nrhs > nrhs_max, ld < N, null pointers),
 * FDA_EHIP. */
int fda_matvec(fda_plan *plan, const void *x_dev, void *y_dev, int64_t nrhs, int64_t ld, void *stream);

/* Right-hand side of a rigid body under unit plane waves exp(ik d.x):
 * b_i = u_inc(c_i) + alpha du_inc/dn(c_i) (eq. (eq_bm) with zero Neumann
 * data).  dirs: nrhs x 3 host doubles (unit vectors); b_dev: N x nrhs
 * complex128 device buffer, leading dimension ld.  Asynchronous.  Errors:
 * FDA_EINVAL, FDA_EHIP. */
int bm_rhs_planewave(fda_plan *plan, const double *dirs, int64_t nrhs, void *b_dev, int64_t ld, void *stream);

/* b = B g: the right-hand side of eq. (eq_bm) for Neumann data du/dn = g on
 * the surface and no incident field (Section 2; the same fast directional
 * algorithm with the source kernel G, Section 4), with
 *   B_ij = -alpha/2 delta_ij + int_{D_j} [G + alpha dG/dn_x](c_i, y) dy.
 * g_dev, b_dev: N x nrhs complex128 device buffers, leading dimension ld
 * (elements), caller's element order; they must not overlap.  Asynchronous
 * on stream.  Errors: FDA_EINVAL (plan built without opt.neumann_rhs, nrhs <
 * 1 or > nrhs_max, ld < N, null pointers), FDA_EHIP. */
int bm_rhs_neumann(fda_plan *plan, const void *g_dev, void *b_dev, int64_t nrhs, int64_t ld, void *stream);

/* Per-solve results. */
typedef struct bm_stats {
    int32_t iterations;     /* matrix-vector products used (all columns together) */
    int32_t restarts;
    double rel_residual;    /* final true relative residual ||b - A x|| / ||b||, worst column */
    double seconds;         /* wall time of the solve */
    int32_t col_iterations[64]; /* per-column iterations (first 64 columns) */
    int32_t mlp_fallbacks;  /* FDA_PRECOND_MLP: applications whose network output was not finite and
                               that used the block-Jacobi correction instead */
    int32_t mlp_rejected;   /* FDA_PRECOND_MLP: 1 if the judge switched the solve to block Jacobi */
} bm_stats;

/* Solve A x = b by restarted GMRES(restart) from x = 0 (Section 5: GMRES, no
 * preconditioner in the paper), stopping when the true relative residual of
 * every column is <= tol or after maxit products.  Arnoldi orthogonalisation
 * (classical Gram-Schmidt, applied twice), the residual and the Givens
 * updates are FP64.  precond: FDA_PRECOND_NONE, FDA_PRECOND_BLOCK_JACOBI
 * (right preconditioning by the inverses of the leaf self-interaction
 * blocks) or FDA_PRECOND_MLP (the block-Jacobi correction plus the output of
 * the network attached by fda_plan_set_mlp; the preconditioner is then
 * nonlinear, so the solver keeps the preconditioned basis, i.e. flexible
 * GMRES, which it does for every precond).  With FDA_PRECOND_MLP block
 * Jacobi is the judge: the first 6 products use block Jacobi, the next 6 the
 * network, and if the network reduced the residual estimate by less over
 * its 6 steps than block Jacobi over its own, the solve continues with block
 * Jacobi (st->mlp_rejected = 1).  b_dev, x_dev: N x nrhs device buffers, leading dimension ld;
 * x is overwritten.  Synchronous: returns when the solve is done.  st may be
 * NULL.  Returns 0 when converged, FDA_NOTCONV when maxit was reached (x is
 * the last iterate), FDA_EBREAKDOWN on a non-finite value, or FDA_EINVAL /
 * FDA_ENOMEM / FDA_EHIP. */
int bm_solve(fda_plan *plan, const void *b_dev, void *x_dev, int64_t nrhs, int64_t ld, double tol, int32_t restart,
             int32_t maxit, int32_t precond, bm_stats *st, void *stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner.  The paper solves without a preconditioner
 * (Section 5); these calls add one.  A row R is a chunk of <= 64 consecutive
 * elements (tree order) of one leaf L (one row per leaf when n_L <= 64;
 * stats.mlp_rows rows in all).  For a residual v, with z = inv(A_LL) v_L the
 * block-Jacobi correction of the leaf restricted to the row, and the complex
 * row scale s_R = |v_R| * (phase of the entry of v_R with the largest
 * modulus, the first such entry on ties):
 *
 *   features (FDA_MLP_IN = 272 floats): Re v_R/s_R, Im v_R/s_R,
 *     Re z_R/s_R, Im z_R/s_R (each zero-padded to 64 entries), the leaf
 *     width and the mesh's largest edge in wavelengths, n_R/64, 1, then
 *     zeros (v_R = 0 gives zero features apart from the scalars);
 *   network: 272 -> h -> h -> 128, ReLU after the two hidden layers, BF16
 *     weights with FP32 accumulation in inference and training, FP32 master
 *     parameters updated by Adam (beta 0.9 / 0.999, eps 1e-8);
 *   output (FDA_MLP_OUT = 128): Re and Im of a 64-entry correction c_R;
 *   preconditioner: M(v)_R = z_R + s_R c_R, so M(a v) = a M(v) for every
 *     complex a.
 *
 * Parameters are one flat FP32 array: W1 (272 x h, row-major: input index
 * major), b1 (h), W2 (h x h), b2 (h), W3 (h x 128), b3 (128).  Rows of X,
 * T and masks are row-major float arrays on the device.
 * ------------------------------------------------------------------------- */

/* Create a network of hidden width h (1..4096) on `device`: He-normal
 * weights from a seeded generator (W3 scaled by 0.1), zero biases.
 * Synchronous.  Errors: FDA_EINVAL, FDA_EHIP. */
int fda_mlp_create(int32_t hidden, uint64_t seed, int32_t device, fda_mlp **out);

/* Release a network (NULL is allowed).  Detach it from plans first. */
void fda_mlp_free(fda_mlp *mlp);

/* Number of parameters (272h + h + h^2 + h + 128h + 128), or -1 for NULL. */
int64_t fda_mlp_num_params(const fda_mlp *mlp);

/* Hidden width, or -1 for NULL. */
int32_t fda_mlp_hidden(const fda_mlp *mlp);

/* Copy the FP32 parameters to / from a host array of n = num_params floats.
 * set_params rejects non-finite values and refreshes the BF16 copy.
 * Synchronous.  Errors: FDA_EINVAL (count mismatch, NULL), FDA_EHIP. */
int fda_mlp_get_params(const fda_mlp *mlp, float *params, int64_t n);
int fda_mlp_set_params(fda_mlp *mlp, const float *params, int64_t n);

/* Y_dev (rows x 128) = network(X_dev (rows x 272)) on `stream`.  Errors:
 * FDA_EINVAL, FDA_EHIP. */
int fda_mlp_forward(fda_mlp *mlp, const float *X_dev, int64_t rows, float *Y_dev, void *stream);

/* fda_mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, but the two hidden
 * activations (rows x hidden floats each) live in a statically allocated
 * device array of 8,388,608 floats (32 MiB), which each GPU the library runs
 * on holds until the process ends; the call allocates nothing (no hipMalloc,
 * no library allocation) and does not synchronise.  Limit: 2 x rows x hidden
 * <= 8,388,608, i.e. rows <= 16,384 at width 256.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (different
 * streams, or different networks) race and must be serialised by the caller.
 * The caller owns X_dev (rows x 272) and Y_dev (rows x 128), as for
 * fda_mlp_forward.  Asynchronous on `stream`.  Errors: FDA_EINVAL (NULL
 * argument, rows < 1 or above the limit; nothing is launched), FDA_EHIP. */
int fda_mlp_forward_noalloc(fda_mlp *mlp, const float *X_dev, int64_t rows, float *Y_dev, void *stream);

/* Gradient of the masked mean squared error
 *   L = sum (mask * (network(X) - T))^2 / (rows * 128)
 * with respect to every parameter (layout as above) into grad_dev (device,
 * num_params floats); *loss (host, may be NULL) receives L.  The products
 * with the weights use their BF16 copy (the gradient is taken as if the
 * rounding were the identity).  Synchronous.  Errors: FDA_EINVAL, FDA_EHIP. */
int fda_mlp_gradient(fda_mlp *mlp, const float *X_dev, const float *T_dev, const float *M_dev, int64_t rows,
                     float *grad_dev, double *loss, void *stream);

/* Train with Adam on (X, T, mask) rows for `epochs` passes over seeded
 * shuffles in mini-batches of `batch` rows.  losses (host, `epochs` doubles,
 * may be NULL) receives the mean training loss of each epoch.  Synchronous.
 * Errors: FDA_EINVAL, FDA_EBREAKDOWN (non-finite loss), FDA_EHIP. */
int fda_mlp_train(fda_mlp *mlp, const float *X_dev, const float *T_dev, const float *M_dev, int64_t rows,
                  int32_t epochs, int32_t batch, float lr, uint64_t seed, double *losses, void *stream);

/* Training and inference rows of the plan.  r_dev: N x nrhs residuals;
 * e_dev (may be NULL): the matching errors e = A^-1 r.  For column c and row
 * R (leaf order, then chunk order; stats.mlp_rows rows) row c*mlp_rows + R
 * of X_dev (272 floats) gets the features of r; if e_dev is given, the same
 * row of T_dev (128) gets (e_R - z_R)/s_R (s_R the row scale of r) and of M_dev (128) the mask of
 * the row's n_R entries (1 on Re and Im of each, 0 on padding).
 * Synchronous.  Errors: FDA_EINVAL (nrhs / ld out of range), FDA_EHIP. */
int fda_mlp_samples(fda_plan *plan, const void *r_dev, const void *e_dev, int64_t nrhs, int64_t ld, float *X_dev,
                    float *T_dev, float *M_dev, void *stream);

/* The plan's element order: perm (host, N entries) receives, for each tree
 * position, the caller's element index; leaf_off (host, nleaf + 1 entries)
 * the tree-position range of each leaf (leaf L holds positions
 * leaf_off[L] .. leaf_off[L+1]-1).  Leaves are in depth-first Morton order
 * (on adaptive trees they sit on several levels, and the leaves below any
 * box are consecutive).  Either pointer may be NULL.  Errors: FDA_EINVAL
 * (length mismatch). */
int fda_plan_leaves(const fda_plan *plan, int32_t *perm, int64_t n, int64_t *leaf_off, int64_t nleaf);

/* Attach a network to a plan for FDA_PRECOND_MLP (NULL detaches).  The plan
 * borrows it: it must outlive its use in bm_solve. */
int fda_plan_set_mlp(fda_plan *plan, fda_mlp *mlp);

/* ---------------------------------------------------------------------------
 * Many meshes at once.  A batch is one HIP graph that applies A_i x_i = y_i
 * (fda_matvec) for a set of built plans of any sizes and wavenumbers; the
 * plans run on up to 16 concurrent branches, so small meshes fill the GPU
 * together and the whole batch costs one launch.  The graph is captured
 * once with fixed buffers; the caller refills x_devs between launches.
 * ------------------------------------------------------------------------- */

/* Capture the batch: plans[i] (distinct, same device), x_devs[i] / y_devs[i]
 * device buffers of N_i x nrhs[i] complex128 (leading dimension N_i).  The
 * plans' work buffers are sized here (nothing allocates inside the graph)
 * and the graph keeps pointers to them and to each plan's M2L work list.
 * While the batch exists: the plans must not run concurrently with it; a
 * call on one of its plans that would reallocate those buffers (fda_matvec,
 * bm_rhs_neumann, bm_solve or fda_profile_matvec with more columns than the
 * work buffers hold, fda_m2l_set_config with another item order or width,
 * fda_autotune) fails with FDA_EINVAL; and its plans must not be freed (free
 * the batch first).  The same holds for a graph the caller captures around
 * fda_matvec: it records the work buffers of that call's column count.
 * Errors: FDA_EINVAL, FDA_ENOMEM, FDA_EHIP; *out is NULL on error. */
int fda_batch_create(fda_plan *const *plans, int32_t nplans, const void *const *x_devs, void *const *y_devs,
                     const int64_t *nrhs, fda_batch **out);

/* Launch the captured products on `stream` (asynchronous).  Errors:
 * FDA_EINVAL, FDA_EHIP. */
int fda_batch_launch(fda_batch *batch, void *stream);

/* Release a batch (waits for the device; NULL is allowed).  Plans and
 * buffers are not touched. */
void fda_batch_free(fda_batch *batch);

/* Statistics of a built plan. */
int fda_plan_stats(const fda_plan *plan, fda_stats *st);

/* Stage timings of fda_matvec (milliseconds, HIP events on the given
 * stream, averaged over `reps` back-to-back products of nrhs columns). */
typedef struct fda_profile_result {
    double near_ms, s2m_ms, m2m_ms, m2l_ms, l2l_ms, l2t_ms, total_ms;
    double m2l_gemm_ms[24];     /* the full-rank M2L product kernel of each level that is not low-rank
                                   (without its reduction) */
    double perm_ms;             /* the permutations into and out of tree order */
    double m2l_lowrank_ms;      /* the one launch of the low-rank M2L product kernel that serves every
                                   low-rank level (without its reduction) */
} fda_profile_result;

/* Configuration of the merged low-rank M2L launch (Section 4.2: the
 * reduced translations grouped by translation into batched products).  The
 * kernel variant and the item order do not change the product (bit for bit);
 * the width changes how the waves of an item split the first product's
 * k-loop, so products of different widths agree to rounding.
 *   variant    kernel variant 0 .. FDA_M2L_VARIANTS - 1 (register-ring depths
 *              of the two product phases)
 *   xcd_order  1: work items dealt into eight per-XCD queues (block b runs on
 *              XCD b mod 8), 0: items in translation order
 *   width[l]   pairs per work item at tree level l: 32 or 16 (translations of
 *              rank above 64 always take 16); 0 for levels without low-rank M2L */
#define FDA_M2L_VARIANTS 4
typedef struct fda_m2l_config {
    int32_t variant;
    int32_t xcd_order;
    int32_t width[24];
} fda_m2l_config;

/* The plan's current configuration (the default after fda_build: variant 0,
 * xcd_order 1, width 32).  Errors: FDA_EINVAL. */
int fda_m2l_get_config(const fda_plan *plan, fda_m2l_config *out);

/* Rebuild the merged M2L work list for *cfg (width entries of levels without
 * low-rank M2L are ignored).  Synchronises the device first (the old list
 * may be in use); not for use during graph capture.  Errors: FDA_EINVAL
 * (variant out of range, xcd_order not 0/1, a width other than 16 or 32),
 * FDA_ENOMEM, FDA_EHIP; on error the previous configuration stays. */
int fda_m2l_set_config(fda_plan *plan, const fda_m2l_config *cfg);

/* Autotuner of the merged M2L launch: starting from the current
 * configuration it times (HIP events on `stream`, median of `reps` launches
 * of the M2L product kernel plus its reduction, one right-hand side) every
 * kernel variant, then the other item order, then width 16 / 32 per level,
 * keeping a change when it is at least 3 % faster, and leaves the plan in the
 * best configuration found.  The plan's work buffers are overwritten.
 * Synchronous.  Errors: FDA_EINVAL (reps < 1 or > 1000), FDA_ENOMEM,
 * FDA_EHIP. */
typedef struct fda_tune_result {
    fda_m2l_config best;
    double ms_before;    /* configuration on entry */
    double ms_after;     /* best configuration, timed again */
    int32_t candidates;  /* configurations timed */
    int32_t nlevels;     /* low-rank levels in the merged launch */
} fda_tune_result;
int fda_autotune(fda_plan *plan, int32_t reps, void *stream, fda_tune_result *out);

/* Profile fda_matvec: x_dev/y_dev as in fda_matvec.  Synchronous. */
int fda_profile_matvec(fda_plan *plan, const void *x_dev, void *y_dev, int64_t nrhs, int64_t ld, int32_t reps,
                       void *stream, fda_profile_result *out);

/* Release a plan and all its device memory (NULL is allowed). */
void fda_free(fda_plan *plan);

/* Thread-local description of the last error ("" if none). */
const char *fda_last_error(void);

/* Library version string. */
const char *fda_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDA_H */
