// Instantiations of the fused search kernel: pad_time = 1, windows up to 64 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_p1_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                               bool dump, hipStream_t st) {
  if (dump) return launch_fused_t<1, 6, 16, true>(tab, n, blocks, st);
  if (hf_max <= 4) return launch_fused_t<1, 6, 4, false>(tab, n, blocks, st);
  return launch_fused_t<1, 6, 16, false>(tab, n, blocks, st);
}

}  // namespace fringe
