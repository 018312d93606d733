// Choice of the fused search kernel for a plan.
#include "kernels.h"

namespace fringe {

hipError_t launch_fused_p1_w3(const FusedArgs& a, bool dump, hipStream_t st);
hipError_t launch_fused_p1_w5(const FusedArgs& a, bool dump, hipStream_t st);
hipError_t launch_fused_p2_w3(const FusedArgs& a, bool dump, hipStream_t st);
hipError_t launch_fused_p2_w5(const FusedArgs& a, bool dump, hipStream_t st);

// APs per unrolled period of the kernel that serves w_max.
int fused_period(int w_max) { return w_max <= 8 ? 4 : 16; }

hipError_t launch_fused(const FusedArgs& a, int pad_t, int w_max, bool dump, hipStream_t st) {
  if (a.hf > 16 || w_max > kFusedMaxWindow) return hipErrorInvalidValue;
  if (pad_t == 1) return w_max <= 8 ? launch_fused_p1_w3(a, dump, st) : launch_fused_p1_w5(a, dump, st);
  if (pad_t == 2) return w_max <= 8 ? launch_fused_p2_w3(a, dump, st) : launch_fused_p2_w5(a, dump, st);
  return hipErrorInvalidValue;
}

}  // namespace fringe
