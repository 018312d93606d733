// Instantiations of the fused search kernel: pad_time = 1, windows up to 32 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_p1_w5(const FusedArgs& a, bool dump, hipStream_t st) {
  if (dump) return launch_fused_t<1, 5, 16, true>(a, st);
  if (a.hf <= 4) return launch_fused_t<1, 5, 4, false>(a, st);
  return launch_fused_t<1, 5, 16, false>(a, st);
}

}  // namespace fringe
