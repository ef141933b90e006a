// Host-formed translation operators, before upload.
#pragma once

#include "plan.hpp"

namespace fda {

struct HostOps {
    std::vector<cplx> S;  // leaf S2M, ku x n_leaf column-major at ku * leaf_off
    std::vector<cplx> T;  // leaf L2T, n_leaf x kd column-major at kd * leaf_off
    std::vector<cplx> SB; // leaf S2M of the right-hand operator B (source kernel G), as S; empty
                          // unless the plan is built for Neumann data
};

void form_operators(const HostPlan &hp, HostOps &ops);

}  // namespace fda
