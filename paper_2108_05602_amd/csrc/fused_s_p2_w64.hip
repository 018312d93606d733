// Instantiations of the fused search kernel for streaming plans (chunks
// read where the caller holds them): pad_time = 2, windows up to 64 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_s_p2_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ) {
  if (hf_max <= 4) return launch_fused_t<2, 6, 4, false, false, true>(tab, n, blocks, st, occ);
  if (hf_max <= 8) return launch_fused_t<2, 6, 8, false, false, true>(tab, n, blocks, st, occ);
  return launch_fused_t<2, 6, 16, false, false, true>(tab, n, blocks, st, occ);
}

}  // namespace fringe
