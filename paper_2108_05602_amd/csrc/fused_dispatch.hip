// Choice of the fused search kernel for a plan.
#include "kernels.h"

namespace fringe {

hipError_t launch_fused_p1_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_p1_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_p2_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_p2_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_p1_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_p2_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max, bool dump,
                              hipStream_t st, int* occ);
hipError_t launch_fused_d_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                             hipStream_t st, int* occ);
hipError_t launch_fused_d_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                             hipStream_t st, int* occ);
hipError_t launch_fused_d_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                             hipStream_t st, int* occ);

hipError_t launch_fused_s_p1_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_p1_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_p1_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_p2_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_p2_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_p2_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                                hipStream_t st, int* occ);
hipError_t launch_fused_s_d_w3(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                               hipStream_t st, int* occ);
hipError_t launch_fused_s_d_w5(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                               hipStream_t st, int* occ);
hipError_t launch_fused_s_d_w6(const FusedArgs* tab, int n, int64_t blocks, int hf_max,
                               hipStream_t st, int* occ);

hipError_t launch_fused_x_p1(const FusedArgs* tab, int n, int64_t blocks, int w_max, bool dump,
                             hipStream_t st, int* occ);
hipError_t launch_fused_x_p2(const FusedArgs* tab, int n, int64_t blocks, int w_max, bool dump,
                             hipStream_t st, int* occ);
hipError_t launch_fused_x_d(const FusedArgs* tab, int n, int64_t blocks, int w_max,
                            hipStream_t st, int* occ);

// Fold class of a band of F channels: the HFMAX of the instantiation that
// serves it (64-channel folds per lane, rounded up to 4, 8 or 16).
int fused_fold_class(int F) {
  const int hf = (F + kBinsPerWave - 1) / kBinsPerWave;
  return hf <= 4 ? 4 : (hf <= 8 ? 8 : 16);
}

int fused_waves_per_pair(int fc, int M, bool delay_only) {
  const int nc = delay_only ? delay_only_classes(fc) : 1;
  return (M / kBinsPerWave + nc - 1) / nc;
}

// APs per unrolled period of the kernel that serves w_max.
int fused_period(int w_max) { return w_max <= 8 ? 4 : (w_max <= 32 ? 16 : 32); }

// One block per (baseline, chunk, class); the classes of a (baseline, chunk)
// pair and its XCD are fixed by the block index, so an entry spans
// 8 * R * ceil(pairs / 8) blocks.
int64_t fused_blocks(const FusedArgs& a) {
  return a.n_pairs == 0 ? 0 : ((int64_t(a.n_pairs) + 7) / 8) * 8 * a.R;
}

hipError_t launch_fused(const FusedArgs* d_tab, int n_tab, int64_t n_blocks, int pad_t,
                        int w_max, int hf_max, bool dump, hipStream_t st, int* occ,
                        bool two_bufs) {
  if (hf_max > 16 || w_max > kFusedMaxWindow) return hipErrorInvalidValue;
  if (two_bufs && hf_max != kFoldSpectra) {
    if (dump || pad_t < 0 || pad_t > 2) return hipErrorInvalidValue;
    const int lw = w_max <= 8 ? 3 : (w_max <= 32 ? 5 : 6);
    if (pad_t == 0)
      return lw == 3 ? launch_fused_s_d_w3(d_tab, n_tab, n_blocks, hf_max, st, occ)
           : lw == 5 ? launch_fused_s_d_w5(d_tab, n_tab, n_blocks, hf_max, st, occ)
                     : launch_fused_s_d_w6(d_tab, n_tab, n_blocks, hf_max, st, occ);
    if (pad_t == 1)
      return lw == 3 ? launch_fused_s_p1_w3(d_tab, n_tab, n_blocks, hf_max, st, occ)
           : lw == 5 ? launch_fused_s_p1_w5(d_tab, n_tab, n_blocks, hf_max, st, occ)
                     : launch_fused_s_p1_w6(d_tab, n_tab, n_blocks, hf_max, st, occ);
    return lw == 3 ? launch_fused_s_p2_w3(d_tab, n_tab, n_blocks, hf_max, st, occ)
         : lw == 5 ? launch_fused_s_p2_w5(d_tab, n_tab, n_blocks, hf_max, st, occ)
                   : launch_fused_s_p2_w6(d_tab, n_tab, n_blocks, hf_max, st, occ);
  }
  if (hf_max == kFoldSpectra) {
    if (pad_t == 0)
      return dump ? hipErrorInvalidValue : launch_fused_x_d(d_tab, n_tab, n_blocks, w_max, st, occ);
    if (pad_t == 1) return launch_fused_x_p1(d_tab, n_tab, n_blocks, w_max, dump, st, occ);
    if (pad_t == 2) return launch_fused_x_p2(d_tab, n_tab, n_blocks, w_max, dump, st, occ);
    return hipErrorInvalidValue;
  }
  if (pad_t == 0) {
    if (dump) return hipErrorInvalidValue;
    if (w_max <= 8) return launch_fused_d_w3(d_tab, n_tab, n_blocks, hf_max, st, occ);
    if (w_max <= 32) return launch_fused_d_w5(d_tab, n_tab, n_blocks, hf_max, st, occ);
    return launch_fused_d_w6(d_tab, n_tab, n_blocks, hf_max, st, occ);
  }
  if (pad_t == 1) {
    if (w_max <= 8) return launch_fused_p1_w3(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
    if (w_max <= 32) return launch_fused_p1_w5(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
    return launch_fused_p1_w6(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
  }
  if (pad_t == 2) {
    if (w_max <= 8) return launch_fused_p2_w3(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
    if (w_max <= 32) return launch_fused_p2_w5(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
    return launch_fused_p2_w6(d_tab, n_tab, n_blocks, hf_max, dump, st, occ);
  }
  return hipErrorInvalidValue;
}

}  // namespace fringe
