// Instantiations of the fused search kernel reading delay spectra:
// pad_time = 2, windows up to 8, 32 or 64 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_x_p2(const FusedArgs* tab, int n, int64_t blocks, int w_max, bool dump,
                              hipStream_t st, int* occ) {
  if (w_max <= 8)
    return dump ? launch_fused_t<2, 3, 4, true, true>(tab, n, blocks, st, occ)
                : launch_fused_t<2, 3, 4, false, true>(tab, n, blocks, st, occ);
  if (w_max <= 32)
    return dump ? launch_fused_t<2, 5, 4, true, true>(tab, n, blocks, st, occ)
                : launch_fused_t<2, 5, 4, false, true>(tab, n, blocks, st, occ);
  return dump ? launch_fused_t<2, 6, 4, true, true>(tab, n, blocks, st, occ)
              : launch_fused_t<2, 6, 4, false, true>(tab, n, blocks, st, occ);
}

}  // namespace fringe
