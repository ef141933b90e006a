// Host-formed translation operators, before upload.
#pragma once

#include "plan.hpp"

namespace fda {

struct HostOps {
    // per leaf, with ku, kd the ranks of the leaf's level and ns its number
    // of direction slots (1 on non-directional levels; leaves above the
    // coarsest level with interactions have none: ku = kd = 0)
    std::vector<int64_t> sop, top;  // offsets of each leaf's S~ and T~ (nleaf + 1 each)
    std::vector<cplx> S;  // leaf S2M, (ns ku) x n_leaf column-major at sop[leaf]: slot s in rows s ku ..
    std::vector<cplx> T;  // leaf L2T, n_leaf x (ns kd) column-major at top[leaf]: slot s in columns s kd ..
    std::vector<cplx> SB; // leaf S2M of the right-hand operator B (source kernel G), as S; empty
                          // unless the plan is built for Neumann data
};

void form_operators(const HostPlan &hp, HostOps &ops);

// Point sets of a level's direction slot, relative to the box centre
// (dsetup.hip): outgoing check points and incoming equivalent points (the
// cube at 2.95 r on non-directional levels, the slot's cone far set on
// directional ones, reflected through the centre for the incoming side).
std::vector<double> out_check(const Level &lv, int slot);
std::vector<double> in_equiv(const Level &lv, int slot);

}  // namespace fda
