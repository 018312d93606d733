// Instantiations of the fused search kernel reading delay spectra:
// delay-only search (rate bin 0), windows up to 8, 32 or 64 APs.
#include "fused_search.h"

namespace fringe {

hipError_t launch_fused_x_d(const FusedArgs* tab, int n, int64_t blocks, int w_max,
                            hipStream_t st, int* occ) {
  if (w_max <= 8) return launch_fused_t<0, 3, 4, false, true>(tab, n, blocks, st, occ);
  if (w_max <= 32) return launch_fused_t<0, 5, 4, false, true>(tab, n, blocks, st, occ);
  return launch_fused_t<0, 6, 4, false, true>(tab, n, blocks, st, occ);
}

}  // namespace fringe
