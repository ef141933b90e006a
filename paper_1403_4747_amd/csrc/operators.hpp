// Host-formed translation operators, before upload.
#pragma once

#include "plan.hpp"

namespace fda {

struct HostOps {
    std::vector<cplx> S;  // leaf S2M, ku x n_leaf column-major at ku * leaf_off
    std::vector<cplx> T;  // leaf L2T, n_leaf x kd column-major at kd * leaf_off
};

void form_operators(const HostPlan &hp, HostOps &ops);

}  // namespace fda
