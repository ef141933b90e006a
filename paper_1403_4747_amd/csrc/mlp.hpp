// Learned per-leaf preconditioner (device MLP) -- see mlp.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace fda {

constexpr int kMlpIn = 272;   // features per leaf
constexpr int kMlpOut = 128;  // Re / Im of a 64-element correction
constexpr int kMlpLeaf = 64;  // largest leaf the features cover
// Floats of the static per-device scratch of the allocation-free forward
// pass (32 MiB): both hidden activations, rows x hidden each.
constexpr int64_t kMlpNoAllocFloats = (int64_t)8 << 20;

struct MlpError {
    std::string msg;
};

struct Mlp {
    int hidden = 256;
    size_t nparam = 0;
    float *w = nullptr;      // FP32 master parameters: W1 (272 x h), b1, W2 (h x h), b2, W3 (h x 128), b3
    uint16_t *wb = nullptr;  // BF16 copy used by the forward pass
    int64_t cap_rows = 0;
    float *h1 = nullptr, *h2 = nullptr;  // activations of the last forward pass
    std::vector<void *> work;
    void offsets(size_t &w1, size_t &b1, size_t &w2, size_t &b2, size_t &w3, size_t &b3) const;
    void sync_bf16(hipStream_t st);
    void ensure_rows(int64_t rows);
    void forward(const float *X, int64_t rows, float *Y, hipStream_t st);
    void forward_into(const float *X, int64_t rows, float *Y, float *a1, float *a2, hipStream_t st) const;
    // the forward pass with its activations in the static scratch of
    // `device` (the current device); rows <= mlp_noalloc_max_rows(hidden)
    void forward_noalloc(const float *X, int64_t rows, float *Y, int device, hipStream_t st) const;
};

// Largest row count of the allocation-free forward pass at width `hidden`.
int64_t mlp_noalloc_max_rows(int hidden);

// Scratch for one gradient evaluation of up to `batch` rows.
struct MlpGradWork {
    float *yb = nullptr, *dy = nullptr, *dh2 = nullptr, *dh1 = nullptr, *part = nullptr;
    std::vector<void *> bufs;
    MlpGradWork(const Mlp *m, int batch);
    ~MlpGradWork();
    MlpGradWork(const MlpGradWork &) = delete;
    MlpGradWork &operator=(const MlpGradWork &) = delete;
    float *al(size_t count);
    double run(Mlp *m, const float *xb, const float *tb, const float *mb, int rows, float *g, hipStream_t st);
};

Mlp *mlp_create(int hidden, uint64_t seed);
// Full-batch gradient of the masked MSE into g (device, nparam floats);
// returns the sum of squared masked errors.  Synchronous.
double mlp_gradient(Mlp *m, const float *X, const float *T, const float *Mk, int64_t n, float *g, hipStream_t st);
void mlp_free(Mlp *m);
std::vector<double> mlp_train(Mlp *m, const float *X, const float *T, const float *Mk, int64_t n, int epochs,
                              int batch, float lr, uint64_t seed, hipStream_t st);
// Features of a tree-ordered residual column; also its per-leaf norms and
// block-Jacobi correction z (tree order).
void mlp_features(const DevPlan &d, const double2 *vt, const float *leaf_scalars, float *feat, double2 *rscale,
                  double2 *z, hipStream_t st);
// out = z + s * MLP output, per row; *bad = 1 if any output is not finite.
void mlp_apply(const DevPlan &d, const float *Y, const double2 *rscale, const double2 *z, double2 *out, int *bad,
               hipStream_t st);
void mlp_targets(const DevPlan &d, const double2 *et, const double2 *z, const double2 *rscale, float *tgt,
                 float *mask, hipStream_t st);

}  // namespace fda
