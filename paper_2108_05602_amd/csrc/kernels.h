// Host-side interface of the fringe-search kernels (internal to libfringe).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fringe.h"

namespace fringe {

constexpr int kMaxLevels = 8;
constexpr int kMaxWindowAp = 128;
constexpr int kMinMf = 64;
constexpr int kMaxMf = 4096;
constexpr int kBinsPerWave = 64;
// Delay-bin classes per wave of the delay-only search, by the fold class of
// the instantiation (64-channel folds per lane): 4 for bands of up to 4 x 64
// channels, 2 for wider ones (1 in the full search and from spectra).
constexpr int delay_only_classes(int fc) { return fc == 4 ? 4 : ((fc == 8 || fc == 16) ? 2 : 1); }

// Window lengths of a plan, ascending; stride = max(1, W / 2).
struct LevelTable {
  int n;
  int W[kMaxLevels];
  int logW[kMaxLevels];
  int s[kMaxLevels];
};

// Per-window result kept on the device: peak power's amplitude, SNR,
// energy and the peak's flat index k_t * M_f + k_f.
struct WindowRec {
  float amp, snr, energy;
  uint32_t flat;
};

// Per-scan constants on the device (window numbering and units).
struct ScanDev {
  int64_t win_off;                    // id of the scan's first window
  int64_t t_origin;                   // absolute AP of the searched data's first AP
  int32_t nb, T, M_f, log_mf, nwb, pad_t;
  double df, tap;
  int32_t lvl_off[kMaxLevels + 1];    // per-baseline window offsets of each length
  int32_t lvl_j0[kMaxLevels];         // start / stride of each length's first window
};

struct DelayArgs {
  const float2* vis;   // [nb][T][F] visibilities of the slab
  const float2* gains; // [nb][F] calibration gains of the slab, or nullptr
  const int32_t* shifts;  // [F] dedispersion shifts in APs, or nullptr
  int64_t vis_stride;  // elements between baselines of vis (>= T_rows * F)
  // a streamed chunk read where the caller holds it: rows [halo, T_rows) of
  // baseline b at vis2 + b * vis2_stride + (t - halo) * F, rows below halo
  // in vis; nullptr when vis holds every row
  const float2* vis2;
  int64_t vis2_stride;
  int halo;
  float2* X;           // [nb][T][M] delay spectra (out)
  float* e;            // [nb][T] per-AP energy sum |x|^2 (out)
  const float2* tw;    // [M] exp(-2 pi i k / M)
  int nb, T, F, M, log_m, pad_f;
  int T_rows;          // APs of vis a shifted read may reach (>= T; reads past them are 0)
};

struct RateArgs {
  const float2* X;     // [nb][T][M]
  uint64_t* part;      // [n_kb][slab_windows] per bin-block peak keys (out)
  float2* dump;        // full grids (FRINGE_DUMP_GRID) or nullptr
  int64_t slab_windows;
  int64_t dump_base;   // grid element offset of this slab's first baseline
  int64_t grid_per_bl; // grid elements per baseline
  int64_t lvl_goff[kMaxLevels];  // per-baseline grid offset of each length
  int nb, T, M, log_m, n_kb, chunk, n_chunks, w_max, buf_slots, pad_t;
  int nwb;
  int t_emit;          // windows must end at or after this AP (streaming)
  int l0;              // first level searched here (shorter ones go to the fused kernel)
  int lvl_off[kMaxLevels + 1];
  int lvl_j0[kMaxLevels];
  LevelTable lv;
};

// One entry of a fused launch: a slab of baselines of one scan.  A launch
// covers several entries; entry k owns blocks [block_off, next block_off).
struct FusedArgs {
  int64_t block_off;   // first block of this entry in the launch (a multiple of 8)
  const float2* vis;   // [nb][T][F] visibilities of the slab
  const float2* gains; // [nb][F] calibration gains of the slab, or nullptr
  const int32_t* shifts;  // [F] dedispersion shifts in APs, or nullptr
  int64_t vis_stride;  // elements between baselines of vis (>= T * F)
  uint64_t* part;      // [R][slab_windows] per residue-class peak keys (out)
  float* epart;        // [R][slab_windows] per residue-class sum of |G_0|^2 (delay-only, out)
  float* e;            // [nb][T] per-AP energies (out)
  float2* dump;        // full grids (FRINGE_DUMP_GRID) or nullptr
  const float2* tw;    // [M] exp(-2 pi i k / M)
  int64_t slab_windows;
  int64_t dump_base;
  int64_t grid_per_bl;
  int64_t lvl_goff[kMaxLevels];
  int nb, T, F, M, R, hf, chunk, n_chunks, n_pairs, nwb;
  int T_rows;          // APs of vis a shifted read may reach (>= T; reads past them are 0)
  int t_emit;          // windows must end at or after this AP (streaming)
  int lvl_off[kMaxLevels + 1];
  int lvl_j0[kMaxLevels];
  int lvl_of_log[8];   // level index of the length 2^L, -1 if not searched
  // a streamed chunk read in place: rows [halo, T_rows) in vis2 (as in
  // DelayArgs), nullptr when vis holds every row
  const float2* vis2;
  int64_t vis2_stride;
  int halo;
};

// One entry of a finalize launch; entry k owns the launch's windows
// [win_begin, next win_begin).
struct FinalizeArgs {
  int64_t win_begin;
  const uint64_t* part;
  const float* epart;  // delay-only: per-class power sums; nullptr otherwise
  const float* e;
  WindowRec* table;    // records of this slab's windows (already offset)
  int64_t slab_windows;
  int n_kb, nb, T, nwb, pad_t, M;
  int lvl_off[kMaxLevels + 1];
  int lvl_j0[kMaxLevels];
  LevelTable lv;
};

struct CompactArgs {
  const WindowRec* table;
  int64_t n_windows;
  float threshold;
  int32_t* blk_counts;
  int64_t* blk_offsets;
  int64_t n_blocks;
  fringe_candidate* out;
  int64_t max_out;
  int64_t* total;
  const ScanDev* scans;
  int n_scans;
  LevelTable lv;
};

constexpr int kCompactBlock = 1024;  // windows per compaction block

// exp(-2 pi i k / m), k < m, for m a power of two in [64, 4096]: device
// address of the library's compile-time table on the current device.
hipError_t twiddles_for(int m, const float2** out);

hipError_t launch_delay_fft(const DelayArgs& a, hipStream_t st);
hipError_t launch_rate_peak(const RateArgs& a, hipStream_t st);
// Fused path for plans whose longest window is at most kFusedMaxWindow APs.
constexpr int kFusedMaxWindow = 64;
int fused_period(int w_max);
// Blocks that entry `a` occupies in a fused launch.
int64_t fused_blocks(const FusedArgs& a);
// Fold class (4, 8 or 16 folds of 64 channels per lane) serving F channels.
int fused_fold_class(int F);
// The fused kernel's waves per (baseline, chunk) for a band of fold class
// fc and M delay bins, which is the number of partial peaks per window:
// M / 64, over delay_only_classes(fc) rounded up for delay-only bands.
int fused_waves_per_pair(int fc, int M, bool delay_only);
// The fold class value that selects the kernel reading delay spectra
// (entries' vis = X[b][t][M], F = M, no gains or shifts).
constexpr int kFoldSpectra = 0;
// d_tab: n_tab entries in device memory; hf_max: the largest entry hf, or
// kFoldSpectra; pad_t = 0 selects the delay-only search (rate bin 0 only).
// With occ set, nothing is launched: *occ receives the chosen
// instantiation's resident work groups (of one wave) per CU.  two_bufs:
// the instantiations whose entries may read their rows from two buffers
// (vis2; streaming plans), not for spectra or grid dumps.
hipError_t launch_fused(const FusedArgs* d_tab, int n_tab, int64_t n_blocks, int pad_t,
                        int w_max, int hf_max, bool dump, hipStream_t st, int* occ = nullptr,
                        bool two_bufs = false);
hipError_t launch_finalize(const FinalizeArgs* d_tab, int n_tab, int64_t n_windows,
                           hipStream_t st);
hipError_t launch_compact(const CompactArgs& a, hipStream_t st);
hipError_t launch_gather(const WindowRec* table, const int64_t* ids, int64_t n,
                         fringe_candidate* out, const ScanDev* scans, int n_scans,
                         const LevelTable& lv, hipStream_t st);

}  // namespace fringe
