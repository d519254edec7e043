// lb_launch.hpp -- host-side launchers of the step kernels.  Each storage x
// collision combination is compiled in its own translation unit (lb_step.hip
// built with LB_S / LB_C defined), so the heavy kernel instantiations build in
// parallel; the host code picks a launcher at context creation.
#pragma once
#include <hip/hip_runtime.h>

#include "lb_device.hpp"

namespace lbdev {
struct LbArgs;
}

namespace lbhost {

using LbLaunch = void (*)(dim3, hipStream_t, const lbdev::LbArgs&);
using ChainLaunch = void (*)(int, hipStream_t, const lbdev::BoxDesc*, const lbdev::ChainDesc*,
                             const void*, const void*, void*, void*, int, int4*, void*, void*, int*,
                             lbdev::DevState*, double, int, long long*, const int4*, int,
                             float*, unsigned, unsigned);

// fused step launcher: storage S (0 FP64, 1 FP32, 2 FP16 deviations), collision
// C (0 BGK, 1 MRT, 2 MRT with ghost rate 1), periodic or not; ext: the
// extended collision (accelerated-frame body force, thermal fluctuations)
template <int S, int C>
LbLaunch pick_lb(bool periodic, bool ext, bool in_place);

// chain forcing pass after the fused step (grid: one workgroup per chain)
template <int S, int C>
LbLaunch pick_force(bool periodic, bool ext);

// chain kernel launcher for storage S; one wavefront per chain when no chain
// has more than 64 beads, else 256 threads; the same launch computes the
// x-face velocities of the step in workgroups after the chains; thermal: the
// beads' Langevin noise
template <int S>
ChainLaunch pick_chain(bool periodic, int max_beads, bool thermal);

}  // namespace lbhost
