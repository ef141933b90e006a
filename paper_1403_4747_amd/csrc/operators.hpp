// Host-formed translation operators, before upload.
#pragma once

#include "plan.hpp"

namespace fda {

struct HostOps {
    // per leaf, with ku, kd the ranks of the leaf's level (leaves above the
    // coarsest level with interactions have none: ku = kd = 0)
    std::vector<int64_t> sop, top;  // offsets of each leaf's S~ and T~ (nleaf + 1 each)
    std::vector<cplx> S;  // leaf S2M, ku x n_leaf column-major at sop[leaf]
    std::vector<cplx> T;  // leaf L2T, n_leaf x kd column-major at top[leaf]
    std::vector<cplx> SB; // leaf S2M of the right-hand operator B (source kernel G), as S; empty
                          // unless the plan is built for Neumann data
};

void form_operators(const HostPlan &hp, HostOps &ops);

}  // namespace fda
