// lb_step.hip -- instantiation of the step kernels for one storage type LB_S
// and one collision operator LB_C (both given on the compiler command line).
#include <hip/hip_runtime.h>

#include "lb_kernels.hpp"
#include "lb_launch.hpp"

#if !defined(LB_S) || !defined(LB_C)
#error "compile with -DLB_S=<0|1|2> -DLB_C=<0|1|2>"
#endif

namespace lbhost {

using namespace lbdev;

template <int S, int C, bool P, bool E, bool AA>
void launch_lb(dim3 g, hipStream_t s, const LbArgs& a) {
  hipLaunchKernelGGL((k_lb<S, C, P, WG, E, AA>), g, dim3(WG), 0, s, a);
}

template <int S, int C>
LbLaunch pick_lb(bool periodic, bool ext, bool in_place) {
  if (periodic) return ext ? launch_lb<S, C, true, true, false> : launch_lb<S, C, true, false, false>;
  if (in_place) return ext ? launch_lb<S, C, false, true, true> : launch_lb<S, C, false, false, true>;
  return ext ? launch_lb<S, C, false, true, false> : launch_lb<S, C, false, false, false>;
}

template LbLaunch pick_lb<LB_S, LB_C>(bool, bool, bool);

template <int S, int C, bool P, bool E>
void launch_force(dim3 g, hipStream_t s, const LbArgs& a) {
  hipLaunchKernelGGL((k_force<S, C, P, E>), g, dim3(WG), 0, s, a);
}

template <int S, int C>
LbLaunch pick_force(bool periodic, bool ext) {
  if (ext) return periodic ? launch_force<S, C, true, true> : launch_force<S, C, false, true>;
  return periodic ? launch_force<S, C, true, false> : launch_force<S, C, false, false>;
}

template LbLaunch pick_force<LB_S, LB_C>(bool, bool);

#if LB_C == 0
template <int S, bool P, int CB, bool TH>
void launch_chain(int nch, hipStream_t s, const BoxDesc* boxes, const ChainDesc* chains,
                  const void* a0, const void* a1, void* pos, void* vel, int total, int4* rb,
                  void* rd, void* rp, int* bbox, DevState* st, double rho0, int pre,
                  long long* stamp, const int4* xf_items, int n_xf, float* xface, unsigned key0,
                  unsigned key1) {
  using T = typename Store<S>::T;
  // one workgroup per chain, then CB / 64 x-face work items per workgroup
  const int nxb = (n_xf + CB / 64 - 1) / (CB / 64);
  hipLaunchKernelGGL((k_chain<S, P, CB, TH>), dim3(nch + nxb), dim3(CB), 0, s, boxes, chains,
                     (const T*)a0, (const T*)a1, (double*)pos, (double*)vel, total, rb, (double*)rd,
                     (double*)rp, bbox, st, rho0, pre, stamp, nch, xf_items, n_xf, xface, key0, key1);
}

template <int S, bool TH>
ChainLaunch pick_chain_th(bool periodic, int max_beads) {
  if (max_beads <= 64) return periodic ? launch_chain<S, true, 64, TH> : launch_chain<S, false, 64, TH>;
  return periodic ? launch_chain<S, true, WG, TH> : launch_chain<S, false, WG, TH>;
}

template <int S>
ChainLaunch pick_chain(bool periodic, int max_beads, bool thermal) {
  return thermal ? pick_chain_th<S, true>(periodic, max_beads)
                 : pick_chain_th<S, false>(periodic, max_beads);
}

template ChainLaunch pick_chain<LB_S>(bool, int, bool);
#endif

}  // namespace lbhost
