// Device part of the plan build (SVD factors and translation matrices).
#pragma once

#include <rocblas/rocblas.h>

#include <vector>

#include "plan.hpp"

namespace fda {

struct DevTranslations {
    std::vector<double2 *> K, M, Lo;  // per level, device arrays (layouts as in DevLevel)
    std::vector<void *> allocs;
    int64_t bytes = 0;
};

// p per level and the truncated SVD factors of G_up / G_dn for every
// level >= top and every active direction (filled into hp.lv[l]).
void device_factors(HostPlan &hp, rocblas_handle h);

// Reduced M2L matrices per distinct offset, compressed M2M / L2L matrices
// per (octant, direction), on the device.
void device_translations(const HostPlan &hp, rocblas_handle h, DevTranslations &out);

}  // namespace fda
