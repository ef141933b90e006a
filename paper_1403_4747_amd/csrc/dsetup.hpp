// Device part of the plan build (SVD factors and translation matrices).
#pragma once

#include <rocblas/rocblas.h>

#include <vector>

#include "plan.hpp"

namespace fda {

// Truncated SVD factors of a batch of matrices (see factor_batch).
struct LowRank {
    double2 *U = nullptr, *V = nullptr;  // device, m x rmax and rmax x n per matrix
    int32_t *rank = nullptr;             // device, padded rank per matrix
    int rmax = 0;                        // 0: the factors were not kept
    int rtrue_max = 0;                   // largest unpadded rank
    double mean = 0;                     // mean unpadded rank
    std::vector<int32_t> rtrue;          // unpadded rank per matrix
};

struct DevTranslations {
    std::vector<double2 *> K, M, Lo;  // per level, device arrays (layouts as in DevLevel)
    // low-rank reduced M2L (eq. (eq_epsk)): per level, per translation
    // U^ (kd x rmax) and V^ (rmax x ku), rank rounded up to 4; rmax = 0 when
    // the level keeps the full matrices
    std::vector<double2 *> Ulr, Vlr;
    std::vector<int32_t *> lr_rank;
    std::vector<int> rmax;
    std::vector<double> mean_rank;
    std::vector<std::vector<int32_t>> true_rank;  // per level and offset: SVD rank before padding to 4
    std::vector<void *> allocs;
    int64_t bytes = 0;
};

// p per level and the truncated SVD factors of G_up / G_dn for every
// level >= top and every active direction (filled into hp.lv[l]).
void device_factors(HostPlan &hp, rocblas_handle h);

// Reduced M2L matrices per distinct offset, compressed M2M / L2L matrices
// per (octant, direction), on the device.
void device_translations(const HostPlan &hp, rocblas_handle h, DevTranslations &out);

// Low-rank factorisation of every reduced M2L matrix (Section 4.2): SVD,
// truncation at svd_eps times the largest singular value, K~ = U^ V^ with
// V^ = S^ Q^^H.  Frees the full matrices of levels that switch to it.
void device_lowrank_m2l(const HostPlan &hp, rocblas_handle h, DevTranslations &out, int max_rank);

}  // namespace fda
