// Instantiations of the fused search kernel: pad_time = 2, windows up to 8 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_p2_w3(const FusedArgs& a, bool dump, hipStream_t st) {
  if (dump) return launch_fused_t<2, 3, 16, true>(a, st);
  if (a.hf <= 4) return launch_fused_t<2, 3, 4, false>(a, st);
  return launch_fused_t<2, 3, 16, false>(a, st);
}

}  // namespace fringe
