// Host side of libfringe: parameter validation, window enumeration, plan
// sizing and device memory, streaming state, and the launch sequence of one
// search.
//
// Window numbering (the order of every table and of the candidate list):
//   id = scan_offset + baseline * n_per_baseline + level_offset[level] + j,
//   t_start = t_origin + (j0[level] + j) * stride(W),  stride(W) = max(1, W / 2),
// for window lengths in ascending order.  A batch search numbers all windows
// of each scan (t_origin = 0, j0 = 0); a streaming call numbers the windows
// whose last AP lies in the call's chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "tune_table.h"

namespace fringe {
int rate_buffer_slots(int w_max);
}

using namespace fringe;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FRINGE_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int log2i(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}
int64_t floor_to(int64_t v, int64_t m) { return v >= 0 ? (v / m) * m : -(((-v) + m - 1) / m) * m; }
int64_t ceil_to(int64_t v, int64_t m) { return -floor_to(-v, m); }

constexpr uint64_t kDefaultScratchCap = 8ull << 30;  // work buffers when no budget is given
constexpr uint64_t kMaxDumpBytes = 1ull << 30;
// candidate records copied to pinned host memory at the end of every search,
// so candidates_get needs no further device round trip when they suffice
constexpr int64_t kCandPrefetch = 2048;

// Windows of one scan in one search: their numbering and where their data is.
struct CallScan {
  int T = 0;                          // APs of the searched data: windows end before it
  int T_rows = 0;                     // APs the data hold (> T: a dedispersion lookahead)
  int t_emit = 0;                     // windows end at or after this AP
  int64_t t_origin = 0;               // absolute AP of the data's AP 0
  int64_t nwb = 0;                    // windows per baseline
  int64_t lvl_off[kMaxLevels + 1] = {};
  int lvl_j0[kMaxLevels] = {};
  int64_t win_off = 0;                // first window id
  // where the kernels read the data: rows [0, split) at the call's data
  // pointer with `stride` elements between baselines; with data2 set (a
  // streamed chunk read in place), rows [split, T_rows) at data2 with
  // stride2 between baselines
  int64_t stride = 0;
  const float2* data2 = nullptr;
  int64_t stride2 = 0;
  int split = 0;
};

// Windows of every length in the data [0, T) that end at or after t_emit.
void enumerate(CallScan* c, const LevelTable& lv) {
  int64_t off = 0;
  for (int l = 0; l < lv.n; ++l) {
    const int64_t w = lv.W[l], s = lv.s[l];
    const int64_t first = ceil_to(std::max<int64_t>(0, c->t_emit - w + 1), s);
    const int64_t last = floor_to(int64_t(c->T) - w, s);
    const int64_t n = last >= first ? (last - first) / s + 1 : 0;
    c->lvl_off[l] = off;
    c->lvl_j0[l] = int(first / s);
    off += n;
  }
  for (int l = lv.n; l <= kMaxLevels; ++l) c->lvl_off[l] = off;
  for (int l = lv.n; l < kMaxLevels; ++l) c->lvl_j0[l] = 0;
  c->nwb = off;
}

struct ScanInfo {
  fringe_scan_desc d;
  int F, M, log_m, n_kb, pad_t;
  CallScan full;                      // batch search: every window of the scan
  int64_t nwb_max;                    // windows per baseline of any one call
  int64_t grid_per_bl;                // grid elements per baseline (dump)
  int64_t lvl_goff[kMaxLevels];
  int64_t grid_off;                   // first grid element of the scan (dump)
  int stage_len;                      // streaming: APs of halo + chunk
  int lookahead;                      // streaming with shifts: APs a window's reads run ahead
  int slab_nb;                        // baselines per pass
  int chunk;                          // search-kernel time tiling
  // Spectra mode: each slab's delay spectra X[b][t][k_f] are written to HBM
  // by the delay-transform kernel and the rate kernels read them (windows
  // longer than 64 APs need it; wide bands use it by default).  x_short:
  // the windows of at most 64 APs read X too (a baseline's spectra under
  // 4 GiB), rather than transforming the visibilities themselves.
  bool spectra;
  bool x_short;
  // the fused kernel's instantiation class (fused_fold_class(F), or kFoldSpectra
  // for x_short) and its waves per (baseline, chunk) = partial peaks per
  // window (every partial-peak consumer reads n_part of them)
  int fc;
  int n_part;
};

// A slab of baselines of one scan: one entry of a fused (or finalize)
// launch, with its place in the work buffers.
struct Unit {
  int scan, b0, nb;
  int fc;                             // kernel of its short windows: fold class or kFoldSpectra
  bool spectra;                       // spectra mode (a group of its own)
  uint64_t e_off, part_off;           // element offsets in the energy / peak buffers
};

// Units [u0, u1) share one fused launch and one finalize launch; every unit
// of a group has the group's kernel class, so each launch runs the kernel
// instantiation its own bands need.  A spectra-mode unit is a group of its
// own: delay transform into the spectra buffer, rate kernels, finalize.
struct Group {
  int u0, u1;
  int fc;
  bool spectra;
};

// Bands of at least this fold class are searched in spectra mode by
// default: with 16 folds per lane the fused kernel's reads of every
// channel by each of the 64 delay-bin classes bound it, and the spectra
// round trip through HBM costs less.
constexpr int kSpectraMinFold = 16;

constexpr int64_t kMaxPlainWindows = int64_t(1) << 21;
constexpr size_t kArenaAlign = 256;
size_t align_up(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

struct Sizing {
  std::vector<ScanInfo> scans;
  std::vector<Unit> units;
  std::vector<Group> groups;
  size_t arena_bytes = 0;             // per-call descriptor tables
  LevelTable lv;
  int w_max = 0;
  bool fused = false;                 // fused kernel (w_max <= kFusedMaxWindow)
  bool streaming = false;
  int align = 1;                      // streaming: stage origins are multiples of this
  int64_t n_windows = 0;              // windows of one call, at most
  int64_t n_blocks = 0;
  bool delay_only = false;            // FRINGE_DELAY_ONLY: rate bin 0 only
  uint64_t scratch_x = 0, scratch_e = 0, scratch_part = 0, scratch_epart = 0, stage_bytes = 0;
  uint64_t table_bytes = 0, blk_bytes = 0, cand_bytes = 0, grid_bytes = 0, fixed_bytes = 0;
  uint64_t total = 0;
};

int data_len(const ScanInfo& s, bool streaming) { return streaming ? s.stage_len : s.d.n_ap; }

int unit_class(const ScanInfo& si) { return si.fc; }

// Bytes per window and delay-bin class: the peak key, and with the
// delay-only search the class's power sum.
size_t part_bytes(bool delay_only) { return sizeof(uint64_t) + (delay_only ? sizeof(float) : 0); }

uint64_t per_baseline_scratch(const ScanInfo& s, bool streaming, bool delay_only) {
  const uint64_t t = uint64_t(data_len(s, streaming));
  const uint64_t x = s.spectra ? t * s.M * sizeof(float2) : 0;
  return x + t * sizeof(float) + uint64_t(s.n_part) * s.nwb_max * part_bytes(delay_only);
}

// A per-scan choice that overrides the defaults of validate_and_size and
// tune_chunks (the autotuner's): the search mode (-1: default) and the time
// chunk (0: default), taken exactly or as an upper bound on the device-sized
// chunk.
struct ScanForce {
  int spectra = -1;
  int chunk = 0;
  bool exact = false;
};

int validate_and_size(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* p,
                      Sizing* out, bool allow_spectra = true,
                      const std::vector<ScanForce>* force = nullptr,
                      const std::vector<int>* lookahead = nullptr) {
  if (!scans || !p || !out) return fail(FRINGE_E_INVALID, "null argument");
  if (n_scans < 1) return fail(FRINGE_E_INVALID, "n_scans must be >= 1 (got %d)", n_scans);
  if (!p->window_aps) return fail(FRINGE_E_INVALID, "window_aps is null");
  if (p->n_window_lengths < 1 || p->n_window_lengths > kMaxLevels)
    return fail(FRINGE_E_INVALID, "n_window_lengths must be in [1, %d]", kMaxLevels);
  if (p->flags & ~(FRINGE_STREAMING | FRINGE_DUMP_GRID | FRINGE_PROFILE | FRINGE_PLAIN | FRINGE_GRAPH |
                   FRINGE_DELAY_ONLY | FRINGE_AUTOTUNE))
    return fail(FRINGE_E_INVALID, "unknown flag bits 0x%x", p->flags);
  if ((p->flags & FRINGE_DELAY_ONLY) && (p->flags & FRINGE_DUMP_GRID))
    return fail(FRINGE_E_INVALID, "FRINGE_DELAY_ONLY has no grid to dump");
  if ((p->flags & FRINGE_GRAPH) && (p->flags & (FRINGE_STREAMING | FRINGE_PROFILE | FRINGE_PLAIN)))
    return fail(FRINGE_E_INVALID, "FRINGE_GRAPH is for batch plans without FRINGE_PROFILE or FRINGE_PLAIN");
  if ((p->flags & FRINGE_STREAMING) && (p->flags & FRINGE_DUMP_GRID))
    return fail(FRINGE_E_INVALID, "FRINGE_DUMP_GRID is for batch plans only");
  if ((p->flags & FRINGE_PLAIN) && (p->flags & (FRINGE_STREAMING | FRINGE_DUMP_GRID)))
    return fail(FRINGE_E_INVALID, "FRINGE_PLAIN is for batch plans without FRINGE_DUMP_GRID");
  if (!(p->snr_threshold >= 0.f) || !std::isfinite(p->snr_threshold))
    return fail(FRINGE_E_INVALID, "snr_threshold must be finite and >= 0");
  if (p->max_candidates < 0) return fail(FRINGE_E_INVALID, "max_candidates must be >= 0");
  if (p->pad_freq != 1 && p->pad_freq != 2 && p->pad_freq != 4)
    return fail(FRINGE_E_UNSUPPORTED, "pad_freq must be 1, 2 or 4 (got %d)", p->pad_freq);
  if (p->pad_time != 1 && p->pad_time != 2)
    return fail(FRINGE_E_UNSUPPORTED, "pad_time must be 1 or 2 (got %d)", p->pad_time);

  Sizing sz;
  sz.streaming = (p->flags & FRINGE_STREAMING) != 0;
  sz.lv.n = p->n_window_lengths;
  for (int i = 0; i < sz.lv.n; ++i) {
    const int w = p->window_aps[i];
    if (w < 1) return fail(FRINGE_E_INVALID, "window length %d must be >= 1", w);
    if (!is_pow2(w) || w > kMaxWindowAp)
      return fail(FRINGE_E_UNSUPPORTED, "window length %d must be a power of two <= %d", w,
                  kMaxWindowAp);
    if (i > 0 && w <= sz.lv.W[i - 1])
      return fail(FRINGE_E_INVALID, "window lengths must be strictly ascending");
    sz.lv.W[i] = w;
    sz.lv.logW[i] = log2i(w);
    sz.lv.s[i] = std::max(1, w / 2);
  }
  for (int i = sz.lv.n; i < kMaxLevels; ++i) sz.lv.W[i] = sz.lv.logW[i] = sz.lv.s[i] = 0;
  sz.w_max = sz.lv.W[sz.lv.n - 1];
  sz.fused = sz.w_max <= kFusedMaxWindow;
  sz.delay_only = (p->flags & FRINGE_DELAY_ONLY) != 0;
  if (sz.delay_only && !sz.fused)
    return fail(FRINGE_E_UNSUPPORTED, "FRINGE_DELAY_ONLY needs windows of at most %d APs",
                kFusedMaxWindow);
  if ((p->flags & FRINGE_PLAIN) && !sz.fused)
    return fail(FRINGE_E_UNSUPPORTED, "FRINGE_PLAIN needs windows of at most %d APs", kFusedMaxWindow);
  // the kernels count window strides (and the fused kernel its period) from
  // AP 0 of the data they read, so streaming stages start on multiples
  sz.align = std::max(std::max(1, sz.w_max / 2), sz.fused ? fused_period(sz.w_max) : 1);

  int64_t win_off = 0, grid_off = 0;
  for (int s = 0; s < n_scans; ++s) {
    const fringe_scan_desc& d = scans[s];
    if (d.n_baselines < 1 || d.n_ap < 1 || d.n_if < 1 || d.n_chan < 1)
      return fail(FRINGE_E_INVALID, "scan %d: every dimension must be >= 1", s);
    if (!(d.ap_seconds > 0.0) || !(d.chan_width_hz > 0.0) || !std::isfinite(d.ap_seconds) ||
        !std::isfinite(d.chan_width_hz))
      return fail(FRINGE_E_INVALID, "scan %d: ap_seconds and chan_width_hz must be > 0", s);
    const int64_t F = int64_t(d.n_if) * d.n_chan;
    if (!is_pow2(F))
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: n_if * n_chan = %lld is not a power of two", s,
                  (long long)F);
    const int64_t M = F * p->pad_freq;
    if (M < kMinMf || M > kMaxMf)
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: pad_freq * F = %lld outside [%d, %d]", s,
                  (long long)M, kMinMf, kMaxMf);
    ScanInfo si{};
    si.d = d;
    si.F = int(F);
    si.M = int(M);
    si.log_m = log2i(M);
    si.n_kb = int(M / kBinsPerWave);
    si.pad_t = p->pad_time;
    si.full.T = d.n_ap;
    si.full.T_rows = d.n_ap;
    enumerate(&si.full, sz.lv);
    si.lookahead = (sz.streaming && lookahead) ? std::max(0, (*lookahead)[size_t(s)]) : 0;
    int64_t goff = 0;
    for (int l = 0; l < sz.lv.n; ++l) {
      si.lvl_goff[l] = goff;
      goff += (si.full.lvl_off[l + 1] - si.full.lvl_off[l]) * int64_t(p->pad_time) * sz.lv.W[l] * M;
    }
    si.grid_per_bl = goff;
    if (sz.streaming) {
      // halo: the last W_max - 1 APs, plus up to align - 1 to start aligned
      si.stage_len = (sz.w_max - 1) + (sz.align - 1) + d.n_ap + si.lookahead;
      int64_t nmax = 0;
      for (int l = 0; l < sz.lv.n; ++l) nmax += (int64_t(d.n_ap) - 1) / sz.lv.s[l] + 1;
      si.nwb_max = nmax;
    } else {
      si.nwb_max = si.full.nwb;
    }
    const int64_t nw = si.nwb_max * d.n_baselines;
    if (si.nwb_max > (int64_t(1) << 30) || nw > (int64_t(1) << 40) ||
        int64_t(data_len(si, sz.streaming)) > (int64_t(1) << 30))
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: too many windows", s);
    // the fused kernel (every plan's windows of at most kFusedMaxWindow APs)
    // addresses one baseline's samples with 32-bit offsets
    if (sz.lv.W[0] <= kFusedMaxWindow &&
        (int64_t(data_len(si, sz.streaming)) + 1) * F * int64_t(sizeof(float2)) >= (int64_t(1) << 32))
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: a baseline holds 4 GiB or more of samples", s);
    // ... and folds at most 16 x 64 channels per lane
    if (sz.lv.W[0] <= kFusedMaxWindow && F > 16 * kBinsPerWave)
      return fail(FRINGE_E_UNSUPPORTED,
                  "scan %d: windows of at most %d APs need n_if * n_chan <= %d (got %lld)", s,
                  kFusedMaxWindow, 16 * kBinsPerWave, (long long)F);
    si.full.win_off = win_off;
    si.grid_off = grid_off;
    win_off += nw;
    grid_off += si.grid_per_bl * d.n_baselines;
    // time chunk of one work item: a multiple of the fused kernel's period
    si.chunk = sz.fused ? 256 : std::min(1024, std::max(128, 8 * sz.w_max));
    // spectra mode: required for windows longer than 64 APs; by default for
    // wide bands of the full search (not with FRINGE_PLAIN, whose launches
    // are one window each)
    const bool x_fits =
        (int64_t(data_len(si, sz.streaming)) + 1) * M * int64_t(sizeof(float2)) < (int64_t(1) << 32);
    si.spectra = !sz.fused || (allow_spectra && !sz.delay_only && !(p->flags & FRINGE_PLAIN) &&
                               x_fits && fused_fold_class(si.F) >= kSpectraMinFold);
    if (sz.fused && force && (*force)[size_t(s)].spectra >= 0)
      si.spectra = (*force)[size_t(s)].spectra > 0 && allow_spectra && x_fits &&
                   !(p->flags & FRINGE_PLAIN);
    si.x_short = si.spectra && x_fits;
    si.fc = si.x_short ? kFoldSpectra : fused_fold_class(si.F);
    si.n_part = fused_waves_per_pair(si.fc, si.M, sz.delay_only);
    if (sz.streaming)
      sz.stage_bytes += 2 * uint64_t(d.n_baselines) * si.stage_len * F * sizeof(float2);
    sz.scans.push_back(si);
  }
  sz.n_windows = win_off;
  sz.n_blocks = (sz.n_windows + kCompactBlock - 1) / kCompactBlock;
  sz.table_bytes = uint64_t(sz.n_windows) * sizeof(WindowRec);
  sz.blk_bytes = uint64_t(sz.n_blocks) * (sizeof(int32_t) + sizeof(int64_t));
  sz.cand_bytes = uint64_t(p->max_candidates) * sizeof(fringe_candidate);
  if (p->flags & FRINGE_DUMP_GRID) {
    sz.grid_bytes = uint64_t(grid_off) * sizeof(float2);
    if (sz.grid_bytes > kMaxDumpBytes)
      return fail(FRINGE_E_INVALID, "FRINGE_DUMP_GRID needs %llu bytes (> %llu): tests only",
                  (unsigned long long)sz.grid_bytes, (unsigned long long)kMaxDumpBytes);
  }
  if ((p->flags & FRINGE_PLAIN) && sz.n_windows > kMaxPlainWindows)
    return fail(FRINGE_E_UNSUPPORTED, "FRINGE_PLAIN is for at most %lld windows (timing subsets)",
                (long long)kMaxPlainWindows);
  sz.fixed_bytes = sz.table_bytes + sz.blk_bytes + sz.cand_bytes + sz.grid_bytes +
                   sz.stage_bytes + 64;

  // Work buffers: process each scan in slabs of baselines that fit.
  uint64_t cap = kDefaultScratchCap;
  if (p->hbm_budget_bytes > 0) {
    if (p->hbm_budget_bytes <= sz.fixed_bytes)
      return fail(FRINGE_E_NOMEM, "hbm_budget_bytes %llu below the %llu bytes of results%s",
                  (unsigned long long)p->hbm_budget_bytes, (unsigned long long)sz.fixed_bytes,
                  sz.streaming ? " and stream history" : "");
    cap = p->hbm_budget_bytes - sz.fixed_bytes;
  }
  for (auto& si : sz.scans) {
    const uint64_t per = per_baseline_scratch(si, sz.streaming, sz.delay_only);
    int64_t nb = int64_t(cap / per);
    if (nb < 1) {
      if (p->hbm_budget_bytes > 0)
        return fail(FRINGE_E_NOMEM, "one baseline of scan needs %llu work bytes, budget leaves %llu",
                    (unsigned long long)per, (unsigned long long)cap);
      nb = 1;
    }
    si.slab_nb = int(std::min<int64_t>(nb, si.d.n_baselines));
  }
  // Units: slabs of baselines, in scan and baseline order within each fold
  // class.  Fused plans pack consecutive units of one class into groups
  // whose work buffers fit the cap, so one launch serves many scans with
  // the instantiation their bands need; two-pass plans give every unit a
  // group of its own.
  std::vector<Unit> all;
  for (int s = 0; s < n_scans; ++s) {
    const ScanInfo& si = sz.scans[s];
    for (int b0 = 0; b0 < si.d.n_baselines; b0 += si.slab_nb)
      all.push_back(Unit{s, b0, std::min(si.slab_nb, si.d.n_baselines - b0), unit_class(si),
                         si.spectra, 0, 0});
  }
  std::stable_sort(all.begin(), all.end(), [](const Unit& x, const Unit& y) {
    return x.spectra != y.spectra ? y.spectra : x.fc < y.fc;
  });
  uint64_t g_e = 0, g_part = 0, max_e = 0, max_part = 0;
  for (Unit u : all) {
    const ScanInfo& si = sz.scans[u.scan];
    const uint64_t t = uint64_t(data_len(si, sz.streaming));
    const uint64_t e_u = uint64_t(u.nb) * t;
    const uint64_t part_u = uint64_t(si.n_part) * u.nb * si.nwb_max;
    const bool open = !sz.groups.empty() && !sz.groups.back().spectra && !u.spectra &&
                      sz.groups.back().fc == u.fc;
    if (!open || (g_e + e_u) * sizeof(float) + (g_part + part_u) * part_bytes(sz.delay_only) > cap) {
      sz.groups.push_back(Group{int(sz.units.size()), int(sz.units.size()), u.fc, u.spectra});
      g_e = g_part = 0;
    }
    u.e_off = g_e;
    u.part_off = g_part;
    sz.units.push_back(u);
    sz.groups.back().u1 = int(sz.units.size());
    g_e += e_u;
    g_part += part_u;
    max_e = std::max(max_e, g_e);
    max_part = std::max(max_part, g_part);
    if (u.spectra)
      sz.scratch_x = std::max<uint64_t>(sz.scratch_x, uint64_t(u.nb) * t * si.M * sizeof(float2));
  }
  sz.scratch_e = max_e * sizeof(float);
  sz.scratch_part = max_part * sizeof(uint64_t);
  sz.scratch_epart = sz.delay_only ? max_part * sizeof(float) : 0;
  const size_t entries = (p->flags & FRINGE_PLAIN) ? size_t(sz.n_windows) : sz.units.size();
  sz.arena_bytes = align_up(size_t(n_scans) * sizeof(ScanDev)) +
                   align_up(entries * sizeof(FusedArgs)) + align_up(entries * sizeof(FinalizeArgs));
  sz.total = sz.fixed_bytes + sz.scratch_x + sz.scratch_e + sz.scratch_part + sz.scratch_epart +
             2 * sz.arena_bytes;
  *out = std::move(sz);
  return FRINGE_OK;
}

// Time chunk of the fused kernel's work items.  A wave searches the windows
// starting in its chunk and transforms the chunk plus W_max - 1 APs of halo,
// so long chunks waste less on halos and short chunks give more, shorter
// waves.  Per fold class (one kernel instantiation), take the longest chunk
// (a multiple of the kernel period, at least 64 APs) that still gives every
// wave slot of the device kWaveRounds waves, the slots being the CUs times
// the waves that instantiation keeps resident per CU; when even 64 does not,
// 64 (the latency-bound case of small grids).  Waves are counted in
// delay-bin classes: a delay-only wave of delay_only_classes classes counts
// as that many (with one wave per class the shorter chunk it would get
// measured 6-20 % slower).
constexpr int kWaveRounds = 16;
int tune_chunks(Sizing* sz, int n_cu, int pad_t_kernel,
                const std::vector<ScanForce>* force = nullptr) {
  if (!sz->fused) return FRINGE_OK;  // windows longer than 64 APs: the plan's fixed chunk
  const int period = fused_period(sz->w_max);
  for (int fc : {kFoldSpectra, 4, 8, 16}) {
    int n_class = 0;
    for (const auto& si : sz->scans) n_class += unit_class(si) == fc ? 1 : 0;
    if (n_class == 0) continue;
    int occ = 0;
    const hipError_t he =
        launch_fused(nullptr, 0, 0, pad_t_kernel, sz->w_max, fc, false, nullptr, &occ,
                     sz->streaming);
    if (he != hipSuccess) return hip_fail(he, "fused kernel occupancy");
    const int64_t target = int64_t(kWaveRounds) * n_cu * std::max(1, occ);
    int best = 64;
    for (int c = 1024; c >= 64; c /= 2) {
      if (c % period) continue;
      int64_t waves = 0;
      for (const auto& si : sz->scans)
        if (unit_class(si) == fc)
          waves += int64_t(si.d.n_baselines) * ((si.d.n_ap + c - 1) / c) * si.n_kb;
      if (waves >= target) {
        best = c;
        break;
      }
    }
    for (size_t k = 0; k < sz->scans.size(); ++k) {
      ScanInfo& si = sz->scans[k];
      if (unit_class(si) != fc) continue;
      si.chunk = best;
      const ScanForce* f = force ? &(*force)[k] : nullptr;
      if (f && f->chunk >= 64 && f->chunk % period == 0)
        si.chunk = f->exact ? f->chunk : std::min(best, f->chunk);
    }
  }
  return FRINGE_OK;
}

ScanDev make_scan_dev(const ScanInfo& si, const CallScan& c) {
  ScanDev d{};
  d.win_off = c.win_off;
  d.t_origin = c.t_origin;
  d.nb = si.d.n_baselines;
  d.T = c.T;
  d.M_f = si.M;
  d.log_mf = si.log_m;
  d.nwb = int32_t(c.nwb);
  d.pad_t = si.pad_t;
  d.df = si.d.chan_width_hz;
  d.tap = si.d.ap_seconds;
  for (int l = 0; l <= kMaxLevels; ++l) d.lvl_off[l] = int32_t(c.lvl_off[l]);
  for (int l = 0; l < kMaxLevels; ++l) d.lvl_j0[l] = c.lvl_j0[l];
  return d;
}

}  // namespace

// Per-subarray state of a streaming plan: the last APs received, on the
// device, in one of two stage buffers [nb][stage_len][F].
struct StreamState {
  float2* stage[2] = {nullptr, nullptr};
  int cur = 0;            // stage holding the newest data
  int64_t consumed = 0;   // APs received so far
  int64_t origin = 0;     // absolute AP of stage[cur] AP 0
  int len = 0;            // APs held in stage[cur]
};

struct fringe_plan_s {
  Sizing sz;
  fringe_params params{};
  std::vector<int32_t> window_aps;
  int device = 0;
  float2* X = nullptr;
  float* e = nullptr;
  uint64_t* part = nullptr;
  float* epart = nullptr;          // delay-only: per-class power sums
  WindowRec* table = nullptr;
  int32_t* blk_counts = nullptr;
  int64_t* blk_offsets = nullptr;
  fringe_candidate* cands = nullptr;
  int64_t* d_total = nullptr;
  ScanDev* d_scans = nullptr;      // scan table of the last search (inside an arena)
  float2* grid = nullptr;
  const float2* tw[13] = {};        // twiddle tables (the library's, not owned)
  int64_t* h_total = nullptr;      // pinned
  fringe_candidate* h_cands = nullptr;  // pinned, the first n_prefetch records
  int64_t n_prefetch = 0;
  int64_t* d_ids = nullptr;        // windows_get staging
  fringe_candidate* d_recs = nullptr;
  int64_t staging_cap = 0;
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool searched = false;
  // per-call descriptor tables: built in host memory, staged through one of
  // two pinned buffers into one of two device arenas (skipped when equal to
  // the last upload); arena_free[k] fires when the last search reading
  // d_arena[k] has finished
  std::vector<char> tables;
  std::vector<char> last_upload;
  char* h_arena[2] = {nullptr, nullptr};
  char* d_arena[2] = {nullptr, nullptr};
  hipEvent_t arena_free[2] = {nullptr, nullptr};
  int arena_last = -1;
  // FRINGE_GRAPH: the device work of a search captured on a private stream,
  // replayed while the descriptor tables (hence every pointer) are unchanged
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_arena = -1;
  std::vector<const float2*> gains;  // per scan: [n_baselines][F] device gains or nullptr
  std::vector<const int32_t*> shifts;  // per scan: [F] dedispersion shifts or nullptr
  // streaming
  std::vector<StreamState> streams;
  std::vector<CallScan> call;      // numbering of the last search
  std::vector<char> call_present;
  int64_t call_windows = 0;
  // FRINGE_PROFILE: an event pair per launch, kind 0..3 = delay, rate, finalize, compact
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
  size_t prof_used = 0;
  // FRINGE_AUTOTUNE: the tune entries of the plan's classes of scans
  std::vector<std::pair<TuneKey, TuneVal>> tuned;
  // what the plan was made from, to make it again (a streaming plan whose
  // dedispersion shifts need a longer stage)
  std::vector<fringe_scan_desc> descs;
  std::vector<ScanForce> force;
  std::vector<int> lookahead;
};

namespace {

void release(fringe_plan_t p) {
  if (!p) return;
  if (p->searched && p->done) (void)hipEventSynchronize(p->done);
  void* bufs[] = {p->X, p->e, p->part, p->epart, p->table, p->blk_counts, p->blk_offsets, p->cands,
                  p->d_total, p->grid, p->d_ids, p->d_recs, p->d_arena[0], p->d_arena[1]};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (auto& st : p->streams)
    for (auto* b : st.stage)
      if (b) (void)hipFree(b);
  for (int k = 0; k < 2; ++k) {
    if (p->h_arena[k]) (void)hipHostFree(p->h_arena[k]);
    if (p->arena_free[k]) (void)hipEventDestroy(p->arena_free[k]);
  }
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->cap_st) (void)hipStreamDestroy(p->cap_st);
  if (p->h_total) (void)hipHostFree(p->h_total);
  if (p->h_cands) (void)hipHostFree(p->h_cands);
  for (auto ev : p->prof_ev) (void)hipEventDestroy(ev);
  if (p->done) (void)hipEventDestroy(p->done);
  delete p;
}

template <typename T>
int dev_alloc(T** ptr, uint64_t bytes, const char* what) {
  *ptr = nullptr;
  if (bytes == 0) return FRINGE_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(FRINGE_E_NOMEM, "hipMalloc(%s, %llu bytes): %s", what, (unsigned long long)bytes,
                hipGetErrorString(e));
  }
  return FRINGE_OK;
}

// Record the start event of a profiled launch (no-op without FRINGE_PROFILE).
hipError_t prof_begin(fringe_plan_s* p, int kind, hipStream_t st) {
  if (!(p->params.flags & FRINGE_PROFILE)) return hipSuccess;
  while (p->prof_ev.size() < 2 * (p->prof_used + 1)) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    p->prof_ev.push_back(ev);
  }
  if (p->prof_kind.size() < p->prof_used + 1) p->prof_kind.resize(p->prof_used + 1);
  p->prof_kind[p->prof_used] = kind;
  return hipEventRecord(p->prof_ev[2 * p->prof_used], st);
}

hipError_t prof_end(fringe_plan_s* p, hipStream_t st) {
  if (!(p->params.flags & FRINGE_PROFILE)) return hipSuccess;
  hipError_t e = hipEventRecord(p->prof_ev[2 * p->prof_used + 1], st);
  ++p->prof_used;
  return e;
}

// Window id of the last search -> (scan, baseline, level, j relative to j0).
int decode_id(const fringe_plan_s* p, int64_t id, int* scan, int* b, int* li, int64_t* j) {
  if (id < 0 || id >= p->call_windows)
    return fail(FRINGE_E_INVALID, "window id %lld out of range", (long long)id);
  int s = -1;
  for (int k = 0; k < int(p->call.size()); ++k)
    if (p->call_present[k] && p->call[k].win_off <= id) s = k;
  const CallScan& c = p->call[s];
  const int64_t loc = id - c.win_off;
  const int64_t bb = loc / c.nwb;
  const int64_t rem = loc - bb * c.nwb;
  int l = 0;
  while (l + 1 < p->sz.lv.n && rem >= c.lvl_off[l + 1]) ++l;
  *scan = s;
  *b = int(bb);
  *li = l;
  *j = rem - c.lvl_off[l];
  return FRINGE_OK;
}

// Subarray s's next chunk: the data the call's kernels read and the call's
// numbering.  The halo (the APs before the chunk that the chunk's windows
// reach back to, from an aligned absolute AP on) is in a stage buffer.
// Without dedispersion shifts the kernels read the chunk where the caller
// holds it, and the APs the next call's halo needs are copied from the
// halo and the chunk into the other stage buffer now, on the call's
// stream, so the caller may reuse the chunk's memory once the search has
// finished.  With shifts (a lane's row depends on its channel) the chunk is
// copied after the halo and the stage is read as one buffer.
int stage_chunk(fringe_plan_s* p, int s, const float2* chunk, hipStream_t st, CallScan* c,
                const float2** data) {
  const ScanInfo& si = p->sz.scans[s];
  StreamState& ss = p->streams[s];
  const int64_t A = ss.consumed;
  const int C = si.d.n_ap;
  const int D = si.lookahead;
  // start APs are reported as int32 (fringe_candidate.t_start)
  if (A + C > int64_t(INT32_MAX))
    return fail(FRINGE_E_UNSUPPORTED,
                "subarray %d: the stream would pass 2^31 - 1 APs (start APs are int32)", s);
  // windows ending in [A - D, A + C - D) are reported: with dedispersion
  // shifts up to D, their reads reach AP A + C - 1 at most
  const int64_t origin =
      std::max<int64_t>(0, floor_to(A - D - (p->sz.w_max - 1), p->sz.align));
  const int halo = int(A - origin);
  const int nxt = ss.cur ^ 1;
  const size_t row = size_t(si.stage_len) * si.F * sizeof(float2);  // one baseline of a stage
  const size_t ap_bytes = size_t(si.F) * sizeof(float2);
  hipError_t he;
  if (!p->shifts[size_t(s)]) {
    // stage[cur] holds APs [ss.origin, ss.origin + ss.len) ⊇ [origin, A)
    const float2* held = ss.stage[ss.cur];
    const int64_t o2 = std::max<int64_t>(0, floor_to(A + C - D - (p->sz.w_max - 1), p->sz.align));
    if (o2 < A) {
      he = hipMemcpy2DAsync(ss.stage[nxt], row, held + (o2 - ss.origin) * si.F, row,
                            size_t(A - o2) * ap_bytes, si.d.n_baselines,
                            hipMemcpyDeviceToDevice, st);
      if (he != hipSuccess) return hip_fail(he, "stream halo copy");
    }
    const int64_t c0 = std::max(o2, A);
    if (A + C > c0) {
      he = hipMemcpy2DAsync(ss.stage[nxt] + (c0 - o2) * si.F, row, chunk + (c0 - A) * si.F,
                            C * ap_bytes, size_t(A + C - c0) * ap_bytes, si.d.n_baselines,
                            hipMemcpyDeviceToDevice, st);
      if (he != hipSuccess) return hip_fail(he, "stream halo copy from the chunk");
    }
    if (halo > 0) {
      *data = held + (origin - ss.origin) * si.F;
      c->stride = int64_t(si.stage_len) * si.F;
      c->data2 = chunk;
      c->stride2 = int64_t(C) * si.F;
      c->split = halo;
    } else {
      *data = chunk;
      c->stride = int64_t(C) * si.F;
    }
    ss.cur = nxt;
    ss.origin = o2;
    ss.len = int(A + C - o2);
    ss.consumed = A + C;
    c->T_rows = halo + C;
    c->T = std::max(0, halo + C - D);
    c->t_emit = int(std::max<int64_t>(0, A - D - origin));
    c->t_origin = origin;
    enumerate(c, p->sz.lv);
    return FRINGE_OK;
  }
  if (halo > 0) {
    const float2* src = ss.stage[ss.cur] + (origin - ss.origin) * si.F;
    he = hipMemcpy2DAsync(ss.stage[nxt], row, src, row, halo * ap_bytes, si.d.n_baselines,
                          hipMemcpyDeviceToDevice, st);
    if (he != hipSuccess) return hip_fail(he, "stream halo copy");
  }
  he = hipMemcpy2DAsync(ss.stage[nxt] + size_t(halo) * si.F, row, chunk, C * ap_bytes,
                        C * ap_bytes, si.d.n_baselines, hipMemcpyDeviceToDevice, st);
  if (he != hipSuccess) return hip_fail(he, "stream chunk copy");
  ss.cur = nxt;
  ss.origin = origin;
  ss.len = halo + C;
  ss.consumed = A + C;
  c->T_rows = halo + C;
  c->T = std::max(0, halo + C - D);
  c->t_emit = int(std::max<int64_t>(0, A - D - origin));
  c->t_origin = origin;
  c->stride = int64_t(si.stage_len) * si.F;
  enumerate(c, p->sz.lv);
  *data = ss.stage[nxt];
  return FRINGE_OK;
}

// The device buffers a search's descriptor tables point into.
struct WorkBufs {
  float2* X = nullptr;                // delay spectra of the slab (spectra mode)
  float* e = nullptr;                 // AP energies
  uint64_t* part = nullptr;           // per-class partial peaks
  float* epart = nullptr;             // per-class power sums (delay-only)
  WindowRec* table = nullptr;         // window records
  float2* grid = nullptr;             // grid dump
  const float2* tw = nullptr;         // twiddles of the scan's M_f
  const float2* gains = nullptr;      // the scan's [n_baselines][F] gains
  const int32_t* shifts = nullptr;    // the scan's [F] shifts
};

WorkBufs plan_bufs(const fringe_plan_s* p, int scan) {
  WorkBufs w;
  w.X = p->X;
  w.e = p->e;
  w.part = p->part;
  w.epart = p->epart;
  w.table = p->table;
  w.grid = p->grid;
  w.tw = p->tw[p->sz.scans[size_t(scan)].log_m];
  w.gains = p->gains.empty() ? nullptr : p->gains[size_t(scan)];
  w.shifts = p->shifts.empty() ? nullptr : p->shifts[size_t(scan)];
  return w;
}

FusedArgs fused_entry(const Sizing& z, const WorkBufs& w, const ScanInfo& si, const CallScan& c,
                      const Unit& u, const float2* data, int64_t vis_stride) {
  FusedArgs fu{};
  fu.vis = data ? data + int64_t(u.b0) * vis_stride : nullptr;
  fu.gains = w.gains ? w.gains + int64_t(u.b0) * si.F : nullptr;
  fu.shifts = w.shifts;
  fu.vis_stride = vis_stride;
  if (c.data2) {
    fu.vis2 = c.data2 + int64_t(u.b0) * c.stride2;
    fu.vis2_stride = c.stride2;
    fu.halo = c.split;
  }
  fu.part = w.part + u.part_off;
  fu.epart = w.epart ? w.epart + u.part_off : nullptr;
  fu.e = w.e + u.e_off;
  fu.dump = w.grid;
  fu.tw = w.tw;
  fu.slab_windows = int64_t(u.nb) * c.nwb;
  fu.dump_base = si.grid_off + int64_t(u.b0) * si.grid_per_bl;
  fu.grid_per_bl = si.grid_per_bl;
  for (int l = 0; l < kMaxLevels; ++l) fu.lvl_goff[l] = si.lvl_goff[l];
  fu.nb = u.nb;
  fu.T = c.T;
  fu.T_rows = std::max(c.T, c.T_rows);
  fu.F = si.F;
  fu.M = si.M;
  fu.R = si.n_part;
  fu.hf = (si.F + kBinsPerWave - 1) / kBinsPerWave;
  fu.chunk = si.chunk;
  fu.n_chunks = (c.T + si.chunk - 1) / si.chunk;
  fu.n_pairs = fu.slab_windows > 0 ? u.nb * fu.n_chunks : 0;
  fu.nwb = int(c.nwb);
  fu.t_emit = c.t_emit;
  for (int l = 0; l <= kMaxLevels; ++l) fu.lvl_off[l] = int(c.lvl_off[l]);
  for (int l = 0; l < kMaxLevels; ++l) fu.lvl_j0[l] = c.lvl_j0[l];
  for (int L = 0; L < 8; ++L) fu.lvl_of_log[L] = -1;
  for (int l = 0; l < z.lv.n; ++l) fu.lvl_of_log[z.lv.logW[l]] = l;
  if (si.x_short) {
    // the short windows read the slab's delay spectra, into which the
    // delay-transform kernel has applied gains and shifts
    fu.vis = w.X;
    fu.vis_stride = int64_t(c.T) * si.M;
    fu.vis2 = nullptr;
    fu.T_rows = c.T;
    fu.F = si.M;
    fu.gains = nullptr;
    fu.shifts = nullptr;
  }
  return fu;
}

FinalizeArgs finalize_entry(const Sizing& z, const WorkBufs& w, const ScanInfo& si,
                            const CallScan& c, const Unit& u) {
  FinalizeArgs fa{};
  fa.part = w.part + u.part_off;
  fa.epart = w.epart ? w.epart + u.part_off : nullptr;
  fa.e = w.e + u.e_off;
  fa.table = w.table + c.win_off + int64_t(u.b0) * c.nwb;
  fa.slab_windows = int64_t(u.nb) * c.nwb;
  fa.n_kb = si.n_part;
  fa.nb = u.nb;
  fa.T = c.T;
  fa.nwb = int(c.nwb);
  fa.pad_t = si.pad_t;
  fa.M = si.M;
  for (int l = 0; l <= kMaxLevels; ++l) fa.lvl_off[l] = int(c.lvl_off[l]);
  for (int l = 0; l < kMaxLevels; ++l) fa.lvl_j0[l] = c.lvl_j0[l];
  fa.lv = z.lv;
  return fa;
}

// Byte offsets of the three tables inside an arena.
struct ArenaLayout {
  size_t scans, fused, fin;
};

ArenaLayout arena_layout(const Sizing& z, size_t n_entries) {
  ArenaLayout L;
  L.scans = 0;
  L.fused = align_up(z.scans.size() * sizeof(ScanDev));
  L.fin = L.fused + align_up(n_entries * sizeof(FusedArgs));
  return L;
}

// Upload the host tables into a device arena (unless they equal the last
// upload) and return its index.
int upload_tables(fringe_plan_s* p, hipStream_t st, int* k_out, bool* uploaded) {
  hipError_t he;
  *uploaded = false;
  if (p->arena_last >= 0 && p->tables == p->last_upload) {
    *k_out = p->arena_last;
    return FRINGE_OK;
  }
  *uploaded = true;
  const int k = p->arena_last < 0 ? 0 : (p->arena_last ^ 1);
  if ((he = hipEventSynchronize(p->arena_free[k])) != hipSuccess)
    return hip_fail(he, "descriptor staging");
  std::memcpy(p->h_arena[k], p->tables.data(), p->tables.size());
  if ((he = hipMemcpyAsync(p->d_arena[k], p->h_arena[k], p->tables.size(), hipMemcpyHostToDevice,
                           st)) != hipSuccess)
    return hip_fail(he, "descriptor upload");
  p->last_upload = p->tables;
  p->arena_last = k;
  *k_out = k;
  return FRINGE_OK;
}

// FRINGE_PLAIN: every window searched by its own launch of the fused kernel
// (data = the window's W APs of one baseline, one length) and its own
// finalize launch; the table and candidate list come out as in a batch
// search.  A baseline for timing the batched launches against.
int plain_tables(fringe_plan_s* p, const std::vector<const float2*>& data) {
  const Sizing& z = p->sz;
  const ArenaLayout L = arena_layout(z, size_t(p->call_windows));
  auto* fus = reinterpret_cast<FusedArgs*>(p->tables.data() + L.fused);
  auto* fin = reinterpret_cast<FinalizeArgs*>(p->tables.data() + L.fin);
  int64_t i = 0;
  for (size_t s = 0; s < z.scans.size(); ++s) {
    const ScanInfo& si = z.scans[s];
    const CallScan& c = p->call[s];
    for (int b = 0; b < si.d.n_baselines; ++b) {
      for (int li = 0; li < z.lv.n; ++li) {
        const int w = z.lv.W[li], stride = z.lv.s[li];
        const int64_t n_l = c.lvl_off[li + 1] - c.lvl_off[li];
        for (int64_t j = 0; j < n_l; ++j, ++i) {
          // a one-window "scan": W APs of baseline b from AP j * stride
          CallScan one{};
          one.T = w;
          one.T_rows = w;
          one.nwb = 1;
          for (int l = 0; l <= kMaxLevels; ++l) one.lvl_off[l] = l <= li ? 0 : 1;
          Unit u{int(s), 0, 1, 0, 0};
          const float2* base = data[s] + (int64_t(b) * si.d.n_ap + j * stride) * si.F;
          fus[i] = fused_entry(z, plan_bufs(p, int(s)), si, one, u, base,
                               int64_t(si.d.n_ap) * si.F);
          fus[i].gains = p->gains[s] ? p->gains[s] + int64_t(b) * si.F : nullptr;
          fus[i].block_off = 0;
          // only this length: the shorter windows inside these W APs are
          // other entries' work
          for (int L = 0; L < 8; ++L) fus[i].lvl_of_log[L] = -1;
          fus[i].lvl_of_log[z.lv.logW[li]] = li;
          fin[i] = finalize_entry(z, plan_bufs(p, int(s)), si, one, u);
          fin[i].table = p->table + c.win_off + int64_t(b) * c.nwb + c.lvl_off[li] + j;
          fin[i].win_begin = 0;
        }
      }
    }
  }
  return FRINGE_OK;
}

// ---- the allocation-free search (fringe_search_noalloc) ----------------
//
// Every work buffer of the search (descriptors, per-class partial peaks, AP
// energies, window records, compaction counts) lives in one static device
// array per GPU, reached through the address hipGetSymbolAddress gives for
// it on that device (the array's name is a host-side stand-in).

constexpr uint64_t kNoAllocScratchBytes = uint64_t(64) << 20;
constexpr int kMaxScratchDevices = 64;

// The descriptors of one search, written into the scratch by a kernel that
// takes them as its argument (no host-to-device copy).
struct NoAllocDesc {
  ScanDev sd;
  FusedArgs fa;
  FinalizeArgs fi;
};

__global__ void put_desc_kernel(NoAllocDesc d, NoAllocDesc* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxScratchDevices] = {};

// The scratch's device address on the current device, looked up the first
// time this device calls.
int scratch_base(char** out) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(FRINGE_E_UNSUPPORTED, "device %d: the no-alloc scratch serves devices 0-%d", dev,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (he != hipSuccess || !ptr) return hip_fail(he, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return FRINGE_OK;
}

}  // namespace

extern "C" {

const char* fringe_strerror(int code) {
  switch (code) {
    case FRINGE_OK: return "ok";
    case FRINGE_E_INVALID: return "invalid argument";
    case FRINGE_E_UNSUPPORTED: return "unsupported shape or parameter";
    case FRINGE_E_NOMEM: return "out of device memory or HBM budget";
    case FRINGE_E_HIP: return "HIP runtime error";
    case FRINGE_E_CAPACITY: return "output capacity too small";
    case FRINGE_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

const char* fringe_last_error(void) { return g_last_error.c_str(); }

int fringe_plan_check(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* params,
                      fringe_plan_summary* out) {
  if (!out) return fail(FRINGE_E_INVALID, "null summary pointer");
  Sizing sz;
  const int rc = validate_and_size(scans, n_scans, params, &sz);
  if (rc != FRINGE_OK) return rc;
  out->n_windows = sz.n_windows;
  out->device_bytes = int64_t(sz.total);
  out->scratch_bytes = int64_t(sz.scratch_x + sz.scratch_e + sz.scratch_part + sz.scratch_epart);
  out->max_window_ap = sz.w_max;
  int mn = 1 << 30;
  for (auto& si : sz.scans) mn = std::min(mn, si.slab_nb);
  out->slab_baselines = mn;
  return FRINGE_OK;
}

}  // extern "C"

namespace {

// fringe_plan with per-scan overrides of the search mode and chunk.
int make_plan(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* params,
              const std::vector<ScanForce>* force, fringe_plan_t* out,
              const std::vector<int>* lookahead = nullptr) {
  *out = nullptr;
  Sizing sz;
  int rc = validate_and_size(scans, n_scans, params, &sz, true, force, lookahead);
  if (rc != FRINGE_OK) return rc;
  auto* p = new fringe_plan_s();
  p->descs.assign(scans, scans + n_scans);
  if (force) p->force = *force;
  p->lookahead = lookahead ? *lookahead : std::vector<int>(size_t(n_scans), 0);
  p->sz = std::move(sz);
  p->params = *params;
  p->gains.assign(size_t(n_scans), nullptr);
  p->shifts.assign(size_t(n_scans), nullptr);
  p->window_aps.assign(params->window_aps, params->window_aps + params->n_window_lengths);
  p->params.window_aps = p->window_aps.data();
  hipError_t he = hipGetDevice(&p->device);
  if (he != hipSuccess) {
    release(p);
    return hip_fail(he, "hipGetDevice");
  }
  int n_cu = 0;
  if ((he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device)) !=
      hipSuccess) {
    release(p);
    return hip_fail(he, "hipDeviceGetAttribute");
  }
  if ((rc = tune_chunks(&p->sz, std::max(1, n_cu), p->sz.delay_only ? 0 : params->pad_time,
                        force)) != FRINGE_OK) {
    release(p);
    return rc;
  }
  const Sizing& z = p->sz;
  const int ns = int(z.scans.size());
  if ((rc = dev_alloc(&p->X, z.scratch_x, "delay spectra")) ||
      (rc = dev_alloc(&p->e, z.scratch_e, "AP energies")) ||
      (rc = dev_alloc(&p->part, z.scratch_part, "bin-block peaks")) ||
      (rc = dev_alloc(&p->epart, z.scratch_epart, "bin-block power sums")) ||
      (rc = dev_alloc(&p->table, z.table_bytes, "window table")) ||
      (rc = dev_alloc(&p->blk_counts, uint64_t(z.n_blocks) * sizeof(int32_t), "block counts")) ||
      (rc = dev_alloc(&p->blk_offsets, uint64_t(z.n_blocks) * sizeof(int64_t), "block offsets")) ||
      (rc = dev_alloc(&p->cands, z.cand_bytes, "candidates")) ||
      (rc = dev_alloc(&p->d_total, sizeof(int64_t), "candidate count")) ||
      (rc = dev_alloc(&p->d_arena[0], z.arena_bytes, "descriptor arena")) ||
      (rc = dev_alloc(&p->d_arena[1], z.arena_bytes, "descriptor arena")) ||
      (rc = dev_alloc(&p->grid, z.grid_bytes, "grid dump"))) {
    release(p);
    return rc;
  }
  if (z.streaming) {
    p->streams.resize(ns);
    for (int s = 0; s < ns; ++s) {
      const ScanInfo& si = z.scans[s];
      const uint64_t bytes = uint64_t(si.d.n_baselines) * si.stage_len * si.F * sizeof(float2);
      for (int k = 0; k < 2; ++k)
        if ((rc = dev_alloc(&p->streams[s].stage[k], bytes, "stream stage"))) {
          release(p);
          return rc;
        }
    }
  }
  for (int k = 0; k < 2; ++k) {
    if ((he = hipHostMalloc(reinterpret_cast<void**>(&p->h_arena[k]), z.arena_bytes,
                            hipHostMallocDefault)) != hipSuccess ||
        (he = hipEventCreateWithFlags(&p->arena_free[k], hipEventDisableTiming)) != hipSuccess) {
      release(p);
      return hip_fail(he, "descriptor staging");
    }
  }
  // twiddle tables exp(-2 pi i k / M): the library's compile-time tables
  for (auto& si : z.scans) {
    if (p->tw[si.log_m]) continue;
    if ((he = twiddles_for(si.M, &p->tw[si.log_m])) != hipSuccess) {
      release(p);
      return hip_fail(he, "twiddle table");
    }
  }
  p->n_prefetch = std::min(p->params.max_candidates, kCandPrefetch);
  if ((he = hipHostMalloc(reinterpret_cast<void**>(&p->h_total), sizeof(int64_t), hipHostMallocDefault)) !=
          hipSuccess ||
      (p->n_prefetch > 0 &&
       (he = hipHostMalloc(reinterpret_cast<void**>(&p->h_cands),
                           size_t(p->n_prefetch) * sizeof(fringe_candidate), hipHostMallocDefault)) !=
           hipSuccess) ||
      (he = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess ||
      ((params->flags & FRINGE_GRAPH) &&
       (he = hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking)) != hipSuccess)) {
    release(p);
    return hip_fail(he, "plan host resources");
  }
  *out = p;
  return FRINGE_OK;
}

// Pseudo-random samples for the tuner's timing runs (their values do not
// change the kernels' work).
__global__ void tune_fill_kernel(float* x, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = static_cast<uint32_t>(i) * 0x9E3779B1u ^ static_cast<uint32_t>(i >> 32);
  h ^= h >> 15;
  h *= 0x85EBCA77u;
  h ^= h >> 13;
  x[i] = static_cast<float>(h & 0xFFFFu) * (1.f / 32768.f) - 1.f;
}

constexpr int kTuneSampleAps = 16384;
constexpr int kTuneWavesPerCu = 24;

// Time every launch configuration of one class of scans on a synthetic
// sample of its shape (enough waves for several rounds of the device at the
// longest chunk) and keep the fastest: search mode x time chunk.
int tune_class(const TuneKey& key, const fringe_params* params, int w_max, TuneVal* best) {
  const int F = key.n_freq;
  const int R = key.pad_freq * F / kBinsPerWave;
  const int64_t target = int64_t(kTuneWavesPerCu) * key.cus;
  const int per_bl = (kTuneSampleAps / 1024) * std::max(1, R);
  fringe_scan_desc d{};
  d.n_baselines = int32_t(std::max<int64_t>(1, (target + per_bl - 1) / per_bl));
  d.n_ap = kTuneSampleAps;
  d.n_chan = std::min(F, 64);
  d.n_if = F / d.n_chan;
  d.ap_seconds = 1e-3;
  d.chan_width_hz = 1e6;
  fringe_params q = *params;
  q.flags = (params->flags & FRINGE_DELAY_ONLY) | FRINGE_PROFILE;
  q.hbm_budget_bytes = 0;
  q.max_candidates = 1 << 16;
  const int64_t n_samples = int64_t(d.n_baselines) * d.n_ap * F;
  float2* cube = nullptr;
  int rc = dev_alloc(&cube, uint64_t(n_samples) * sizeof(float2), "tuning sample");
  if (rc != FRINGE_OK) return rc;
  const int64_t n_fl = 2 * n_samples;
  hipLaunchKernelGGL(tune_fill_kernel, dim3(static_cast<unsigned>((n_fl + 255) / 256)), dim3(256),
                     0, nullptr, reinterpret_cast<float*>(cube), n_fl);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) {
    (void)hipFree(cube);
    return hip_fail(he, "tuning sample fill");
  }
  const int period = fused_period(w_max);
  float ms_best[2] = {-1.f, -1.f};
  int chunk_best[2] = {0, 0};
  for (int mode = 0; mode < 2; ++mode) {
    for (int chunk = 128; chunk <= 1024; chunk *= 2) {
      if (chunk % period) continue;
      std::vector<ScanForce> f(1);
      f[0].spectra = mode;
      f[0].chunk = chunk;
      f[0].exact = true;
      fringe_plan_t tp = nullptr;
      rc = make_plan(&d, 1, &q, &f, &tp);
      if (rc == FRINGE_E_NOMEM) continue;  // this configuration does not fit now
      if (rc != FRINGE_OK) {
        (void)hipFree(cube);
        return rc;
      }
      if (tp->sz.scans[0].spectra != (mode == 1)) {  // the mode is not available here
        fringe_plan_destroy(tp);
        break;
      }
      const fringe_cf32* vis[1] = {reinterpret_cast<const fringe_cf32*>(cube)};
      float ms = -1.f;
      for (int rep = 0; rep < 3 && rc == FRINGE_OK; ++rep) {
        rc = fringe_search(tp, vis, nullptr);
        fringe_profile pr{};
        if (rc == FRINGE_OK) rc = fringe_profile_get(tp, &pr);
        const float t = float(pr.delay_ms + pr.rate_ms + pr.finalize_ms + pr.compact_ms);
        if (rc == FRINGE_OK && rep > 0 && (ms < 0.f || t < ms)) ms = t;  // the first warms up
      }
      fringe_plan_destroy(tp);
      if (rc != FRINGE_OK) {
        (void)hipFree(cube);
        return rc;
      }
      if (ms_best[mode] < 0.f || ms < ms_best[mode]) {
        ms_best[mode] = ms;
        chunk_best[mode] = chunk;
      }
    }
  }
  (void)hipFree(cube);
  if (ms_best[0] < 0.f && ms_best[1] < 0.f)
    return fail(FRINGE_E_NOMEM, "autotune: no configuration of class F = %d fits", F);
  const int m = (ms_best[0] < 0.f || (ms_best[1] >= 0.f && ms_best[1] < ms_best[0])) ? 1 : 0;
  best->spectra = m;
  best->chunk = chunk_best[m];
  best->ms_fused = ms_best[0];
  best->ms_spectra = ms_best[1];
  return FRINGE_OK;
}

// Make an unsearched plan again with other search modes / chunks or
// dedispersion lookaheads, keeping the caller's handle, its gains, shifts
// and tune entries; on failure the plan is left as it was.
int remake_plan(fringe_plan_t p, const std::vector<ScanForce>& force,
                const std::vector<int>& lookahead) {
  fringe_plan_t np = nullptr;
  const int rc = make_plan(p->descs.data(), int32_t(p->descs.size()), &p->params,
                           force.empty() ? nullptr : &force, &np, &lookahead);
  if (rc != FRINGE_OK) return rc;
  std::swap(np->gains, p->gains);
  std::swap(np->shifts, p->shifts);
  std::swap(np->tuned, p->tuned);
  std::swap(*np, *p);
  fringe_plan_destroy(np);
  return FRINGE_OK;
}

// FRINGE_AUTOTUNE: the tune table's configuration of every scan's class,
// tuning the classes it lacks.
int autotune_plan(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* params,
                  const Sizing& z, std::vector<ScanForce>* force,
                  std::vector<std::pair<TuneKey, TuneVal>>* used) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  hipDeviceProp_t prop{};
  if (he == hipSuccess) he = hipGetDeviceProperties(&prop, dev);
  if (he != hipSuccess) return hip_fail(he, "device properties");
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  force->assign(size_t(n_scans), ScanForce{});
  for (int s = 0; s < n_scans; ++s) {
    TuneKey k;
    k.arch = arch;
    k.cus = prop.multiProcessorCount;
    k.n_freq = z.scans[size_t(s)].F;
    k.pad_freq = params->pad_freq;
    k.pad_time = z.delay_only ? 0 : params->pad_time;
    k.log2_wmax = log2i(z.w_max);
    TuneVal v;
    if (!tune_lookup(k, &v)) {
      const int rc = tune_class(k, params, z.w_max, &v);
      if (rc != FRINGE_OK) return rc;
      tune_store(k, v);
    }
    (*force)[size_t(s)].spectra = v.spectra;
    (*force)[size_t(s)].chunk = v.chunk;
    bool seen = false;
    for (const auto& e : *used) seen = seen || e.first.n_freq == k.n_freq;
    if (!seen) used->emplace_back(k, v);
  }
  return FRINGE_OK;
}

}  // namespace

extern "C" {

int fringe_plan(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* params,
                fringe_plan_t* out) {
  if (!out) return fail(FRINGE_E_INVALID, "null plan output pointer");
  *out = nullptr;
  std::vector<ScanForce> force;
  std::vector<std::pair<TuneKey, TuneVal>> used;
  if (params && (params->flags & FRINGE_AUTOTUNE)) {
    Sizing probe;
    int rc = validate_and_size(scans, n_scans, params, &probe);
    if (rc != FRINGE_OK) return rc;
    if (probe.fused && (rc = autotune_plan(scans, n_scans, params, probe, &force, &used)) != FRINGE_OK)
      return rc;
  }
  const int rc = make_plan(scans, n_scans, params, force.empty() ? nullptr : &force, out);
  if (rc == FRINGE_OK) (*out)->tuned = std::move(used);
  return rc;
}

int fringe_tune_load(const char* path) {
  if (!path) return fail(FRINGE_E_INVALID, "null path");
  std::string err;
  if (tune_load(path, &err) != 0) return fail(FRINGE_E_INVALID, "%s", err.c_str());
  return FRINGE_OK;
}

int fringe_tune_save(const char* path) {
  if (!path) return fail(FRINGE_E_INVALID, "null path");
  std::string err;
  if (tune_save(path, &err) != 0) return fail(FRINGE_E_INVALID, "%s", err.c_str());
  return FRINGE_OK;
}

void fringe_tune_clear(void) { tune_clear(); }

int fringe_plan_tuning(fringe_plan_t p, fringe_tune_entry* out, int32_t capacity, int32_t* n) {
  if (!p || !n) return fail(FRINGE_E_INVALID, "null argument");
  if (capacity < 0 || (capacity > 0 && !out)) return fail(FRINGE_E_INVALID, "bad output buffer");
  *n = int32_t(p->tuned.size());
  for (int32_t i = 0; i < std::min(capacity, *n); ++i) {
    const TuneKey& k = p->tuned[size_t(i)].first;
    const TuneVal& v = p->tuned[size_t(i)].second;
    out[i] = fringe_tune_entry{k.n_freq, k.pad_freq, k.pad_time, k.log2_wmax, v.spectra, v.chunk,
                               v.ms_fused, v.ms_spectra};
  }
  if (*n > capacity) return fail(FRINGE_E_CAPACITY, "%d tune entries", int(*n));
  return FRINGE_OK;
}

int fringe_search(fringe_plan_t p, const fringe_cf32* const* d_vis, void* hip_stream) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  if (!d_vis) return fail(FRINGE_E_INVALID, "null visibility pointer array");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const Sizing& z = p->sz;
  const int ns = int(z.scans.size());
  if (!z.streaming)
    for (int s = 0; s < ns; ++s)
      if (!d_vis[s]) return fail(FRINGE_E_INVALID, "scan %d: null visibility pointer", s);
  hipError_t he;
  // The plan's buffers (work buffers, window table, candidates, streaming
  // stages) are reused by every search: a search on another stream than the
  // last one first waits for the last one to finish.
  if (p->searched && st != p->last_stream && (he = hipStreamWaitEvent(st, p->done, 0)) != hipSuccess)
    return hip_fail(he, "waiting for the previous search");
  p->prof_used = 0;
#define FRINGE_TIMED(kind, call, what)                                        \
  do {                                                                        \
    if ((he = prof_begin(p, kind, st)) != hipSuccess) return hip_fail(he, "profiling event"); \
    if ((he = (call)) != hipSuccess) return hip_fail(he, what);               \
    if ((he = prof_end(p, st)) != hipSuccess) return hip_fail(he, "profiling event"); \
  } while (0)

  // numbering of this call's windows and the data each scan's kernels read
  p->call.assign(ns, CallScan{});
  p->call_present.assign(ns, 0);
  std::vector<const float2*> data(ns, nullptr);
  int64_t win_off = 0;
  for (int s = 0; s < ns; ++s) {
    CallScan& c = p->call[s];
    if (!d_vis[s]) {  // no chunk: an empty id range at the running offset
      c.win_off = win_off;
      continue;
    }
    if (z.streaming) {
      const int rc = stage_chunk(p, s, reinterpret_cast<const float2*>(d_vis[s]), st, &c, &data[s]);
      if (rc != FRINGE_OK) return rc;
    } else {
      c = z.scans[s].full;
      c.stride = int64_t(z.scans[s].d.n_ap) * z.scans[s].F;
      data[s] = reinterpret_cast<const float2*>(d_vis[s]);
    }
    c.win_off = win_off;
    win_off += c.nwb * z.scans[s].d.n_baselines;
    p->call_present[s] = 1;
  }
  p->call_windows = win_off;
  // descriptor tables of this call: scan table, then one fused and one
  // finalize entry per unit (per window with FRINGE_PLAIN)
  const bool plain = (p->params.flags & FRINGE_PLAIN) != 0;
  const size_t n_entries = plain ? size_t(p->call_windows) : z.units.size();
  const ArenaLayout L = arena_layout(z, n_entries);
  p->tables.assign(L.fin + n_entries * sizeof(FinalizeArgs), 0);
  auto* sdev = reinterpret_cast<ScanDev*>(p->tables.data() + L.scans);
  for (int s = 0; s < ns; ++s) sdev[s] = make_scan_dev(z.scans[s], p->call[s]);
  std::vector<int64_t> grp_blocks(z.groups.size(), 0), grp_windows(z.groups.size(), 0);
  if (plain) {
    plain_tables(p, data);
  } else {
    auto* fus = reinterpret_cast<FusedArgs*>(p->tables.data() + L.fused);
    auto* fin = reinterpret_cast<FinalizeArgs*>(p->tables.data() + L.fin);
    for (size_t g = 0; g < z.groups.size(); ++g) {
      for (int ui = z.groups[g].u0; ui < z.groups[g].u1; ++ui) {
        const Unit& u = z.units[ui];
        const ScanInfo& si = z.scans[u.scan];
        const CallScan& c = p->call[u.scan];
        fus[ui] = fused_entry(z, plan_bufs(p, u.scan), si, c, u, data[u.scan], c.stride);
        if (!p->call_present[u.scan]) fus[ui].n_pairs = 0;
        fus[ui].block_off = grp_blocks[g];
        grp_blocks[g] += fused_blocks(fus[ui]);
        fin[ui] = finalize_entry(z, plan_bufs(p, u.scan), si, c, u);
        if (!p->call_present[u.scan]) fin[ui].slab_windows = 0;
        fin[ui].win_begin = grp_windows[g];
        grp_windows[g] += fin[ui].slab_windows;
      }
    }
  }
  int k = 0;
  bool uploaded = false;
  {
    const int rc = upload_tables(p, st, &k, &uploaded);
    if (rc != FRINGE_OK) return rc;
  }
  char* arena = p->d_arena[k];
  p->d_scans = reinterpret_cast<ScanDev*>(arena + L.scans);
  const FusedArgs* d_fus = reinterpret_cast<const FusedArgs*>(arena + L.fused);
  const FinalizeArgs* d_fin = reinterpret_cast<const FinalizeArgs*>(arena + L.fin);
  const hipStream_t user_st = st;
  const int kernel_pad_t = z.delay_only ? 0 : z.scans[0].pad_t;  // 0: the delay-only kernels

  // Every kernel of the search, enqueued on stream st (the caller's, or the
  // capture stream of FRINGE_GRAPH).
  auto enqueue = [&](hipStream_t st) -> int {
  if (plain) {
    for (int64_t i = 0; i < p->call_windows; ++i) {
      const FusedArgs& h = reinterpret_cast<const FusedArgs*>(p->tables.data() + L.fused)[i];
      FRINGE_TIMED(1, launch_fused(d_fus + i, 1, fused_blocks(h), kernel_pad_t, z.w_max,
                                   fused_fold_class(h.F),
                                   false, st), "plain fused launch");
      FRINGE_TIMED(2, launch_finalize(d_fin + i, 1, 1, st), "plain finalize launch");
    }
  } else {
    const auto* hfus = reinterpret_cast<const FusedArgs*>(p->tables.data() + L.fused);
    // levels served by the fused kernel (windows of at most 64 APs)
    int l0 = 0;
    while (l0 < z.lv.n && z.lv.W[l0] <= kFusedMaxWindow) ++l0;
    for (size_t g = 0; g < z.groups.size(); ++g) {
      const Group& gr = z.groups[g];
      if (grp_windows[g] == 0) continue;
      if (!gr.spectra) {
        FRINGE_TIMED(1, launch_fused(d_fus + gr.u0, gr.u1 - gr.u0, grp_blocks[g], kernel_pad_t,
                                     z.w_max, gr.fc, p->grid != nullptr, st, nullptr,
                                     z.streaming),
                     "fused search launch");
        FRINGE_TIMED(2, launch_finalize(d_fin + gr.u0, gr.u1 - gr.u0, grp_windows[g], st),
                     "finalize launch");
        continue;
      }
      // spectra mode: one unit; its delay spectra to HBM, then the rate kernels
      const int ui = gr.u0;
      const Unit& u = z.units[ui];
      const ScanInfo& si = z.scans[u.scan];
      const CallScan& c = p->call[u.scan];
      DelayArgs da{};
      da.vis = data[u.scan] + int64_t(u.b0) * c.stride;
      da.gains = p->gains[u.scan] ? p->gains[u.scan] + int64_t(u.b0) * si.F : nullptr;
      da.shifts = p->shifts[u.scan];
      da.vis_stride = c.stride;
      if (c.data2) {
        da.vis2 = c.data2 + int64_t(u.b0) * c.stride2;
        da.vis2_stride = c.stride2;
        da.halo = c.split;
      }
      da.X = p->X;
      da.e = p->e + u.e_off;
      da.tw = p->tw[si.log_m];
      da.nb = u.nb;
      da.T = c.T;
      da.T_rows = std::max(c.T, c.T_rows);
      da.F = si.F;
      da.M = si.M;
      da.log_m = si.log_m;
      da.pad_f = p->params.pad_freq;
      FRINGE_TIMED(0, launch_delay_fft(da, st), "delay transform launch");
      if (l0 > 0 && hfus[ui].n_pairs > 0) {
        // the windows of at most kFusedMaxWindow APs: from the spectra, or
        // (a baseline's spectra of 4 GiB or more) by the kernel's own delay
        // transform of the visibilities; same numbering and partials
        FRINGE_TIMED(1, launch_fused(d_fus + ui, 1, fused_blocks(hfus[ui]), kernel_pad_t,
                                     z.lv.W[l0 - 1], unit_class(si),
                                     p->grid != nullptr, st, nullptr, z.streaming),
                     "fused search launch (short windows)");
      }
      if (l0 < z.lv.n) {
        RateArgs ra{};
        ra.X = p->X;
        ra.part = p->part + u.part_off;
        ra.dump = p->grid;
        ra.slab_windows = int64_t(u.nb) * c.nwb;
        ra.dump_base = si.grid_off + int64_t(u.b0) * si.grid_per_bl;
        ra.grid_per_bl = si.grid_per_bl;
        for (int l = 0; l < kMaxLevels; ++l) ra.lvl_goff[l] = si.lvl_goff[l];
        ra.nb = u.nb;
        ra.T = c.T;
        ra.M = si.M;
        ra.log_m = si.log_m;
        ra.n_kb = si.n_kb;
        ra.chunk = si.chunk;
        ra.n_chunks = (c.T + si.chunk - 1) / si.chunk;
        ra.w_max = z.w_max;
        ra.buf_slots = rate_buffer_slots(z.w_max);
        ra.pad_t = si.pad_t;
        ra.nwb = int(c.nwb);
        ra.t_emit = c.t_emit;
        ra.l0 = l0;
        for (int l = 0; l <= kMaxLevels; ++l) ra.lvl_off[l] = int(c.lvl_off[l]);
        for (int l = 0; l < kMaxLevels; ++l) ra.lvl_j0[l] = c.lvl_j0[l];
        ra.lv = z.lv;
        FRINGE_TIMED(1, launch_rate_peak(ra, st), "rate transform launch");
      }
      FRINGE_TIMED(2, launch_finalize(d_fin + ui, 1, grp_windows[g], st), "finalize launch");
    }
  }
  CompactArgs ca{};
  ca.table = p->table;
  ca.n_windows = p->call_windows;
  ca.threshold = p->params.snr_threshold;
  ca.blk_counts = p->blk_counts;
  ca.blk_offsets = p->blk_offsets;
  ca.n_blocks = (p->call_windows + kCompactBlock - 1) / kCompactBlock;
  ca.out = p->cands;
  ca.max_out = p->params.max_candidates;
  ca.total = p->d_total;
  ca.scans = p->d_scans;
  ca.n_scans = ns;
  ca.lv = z.lv;
  FRINGE_TIMED(3, launch_compact(ca, st), "compaction launch");
  return FRINGE_OK;
  };
#undef FRINGE_TIMED

  st = user_st;
  if (p->params.flags & FRINGE_GRAPH) {
    // new tables (other inputs or a first search): capture the work anew
    if (uploaded || !p->gexec || p->g_arena != k) {
      if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
      }
      if ((he = hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(he, "hipStreamBeginCapture");
      const int rc = enqueue(p->cap_st);
      hipGraph_t graph = nullptr;
      const hipError_t he_end = hipStreamEndCapture(p->cap_st, &graph);
      if (rc != FRINGE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (he_end != hipSuccess) return hip_fail(he_end, "hipStreamEndCapture");
      he = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (he != hipSuccess) {
        p->gexec = nullptr;
        return hip_fail(he, "hipGraphInstantiate");
      }
      p->g_arena = k;
    }
    if ((he = hipGraphLaunch(p->gexec, st)) != hipSuccess) return hip_fail(he, "hipGraphLaunch");
  } else {
    const int rc = enqueue(st);
    if (rc != FRINGE_OK) return rc;
  }
  // the count and the first records to pinned host memory
  if ((he = hipMemcpyAsync(p->h_total, p->d_total, sizeof(int64_t), hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (p->n_prefetch > 0 &&
       (he = hipMemcpyAsync(p->h_cands, p->cands, size_t(p->n_prefetch) * sizeof(fringe_candidate),
                            hipMemcpyDeviceToHost, st)) != hipSuccess))
    return hip_fail(he, "candidate prefetch");
  if ((he = hipEventRecord(p->done, st)) != hipSuccess ||
      (he = hipEventRecord(p->arena_free[k], st)) != hipSuccess)
    return hip_fail(he, "hipEventRecord");
  p->last_stream = st;
  p->searched = true;
  return FRINGE_OK;
}

int candidates_get(fringe_plan_t p, fringe_candidate* host_out, int64_t capacity, int64_t* n_total) {
  if (!p || !n_total) return fail(FRINGE_E_INVALID, "null argument");
  if (capacity < 0 || (capacity > 0 && !host_out)) return fail(FRINGE_E_INVALID, "bad output buffer");
  if (!p->searched) return fail(FRINGE_E_STATE, "candidates_get before fringe_search");
  hipError_t he = hipEventSynchronize(p->done);
  if (he != hipSuccess) return hip_fail(he, "hipEventSynchronize");
  // the count and the first n_prefetch records reached pinned memory before
  // the done event
  const int64_t total = *p->h_total;
  *n_total = total;
  const int64_t avail = std::min(total, p->params.max_candidates);
  const int64_t n = std::min(avail, capacity);
  if (n > 0 && n <= p->n_prefetch) {
    std::memcpy(host_out, p->h_cands, size_t(n) * sizeof(fringe_candidate));
  } else if (n > 0) {
    if ((he = hipMemcpyAsync(host_out, p->cands, size_t(n) * sizeof(fringe_candidate),
                             hipMemcpyDeviceToHost, p->last_stream)) != hipSuccess ||
        (he = hipStreamSynchronize(p->last_stream)) != hipSuccess)
      return hip_fail(he, "copying candidates");
  }
  if (total > n)
    return fail(FRINGE_E_CAPACITY, "%lld candidates, %lld copied (capacity %lld, max_candidates %lld)",
                (long long)total, (long long)n, (long long)capacity,
                (long long)p->params.max_candidates);
  return FRINGE_OK;
}

int fringe_windows_get(fringe_plan_t p, const int64_t* ids, int64_t n, fringe_candidate* host_out) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  if (n < 0 || (n > 0 && (!ids || !host_out))) return fail(FRINGE_E_INVALID, "bad id list");
  if (!p->searched) return fail(FRINGE_E_STATE, "fringe_windows_get before fringe_search");
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= p->call_windows)
      return fail(FRINGE_E_INVALID, "window id %lld out of range", (long long)ids[i]);
  if (n == 0) return FRINGE_OK;
  hipError_t he = hipEventSynchronize(p->done);
  if (he != hipSuccess) return hip_fail(he, "hipEventSynchronize");
  if (n > p->staging_cap) {
    if (p->d_ids) (void)hipFree(p->d_ids);
    if (p->d_recs) (void)hipFree(p->d_recs);
    p->d_ids = nullptr;
    p->d_recs = nullptr;
    p->staging_cap = 0;
    int rc;
    if ((rc = dev_alloc(&p->d_ids, uint64_t(n) * sizeof(int64_t), "id staging")) ||
        (rc = dev_alloc(&p->d_recs, uint64_t(n) * sizeof(fringe_candidate), "record staging")))
      return rc;
    p->staging_cap = n;
  }
  hipStream_t st = p->last_stream;
  if ((he = hipMemcpyAsync(p->d_ids, ids, size_t(n) * sizeof(int64_t), hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return hip_fail(he, "copying ids");
  if ((he = launch_gather(p->table, p->d_ids, n, p->d_recs, p->d_scans, int(p->sz.scans.size()),
                          p->sz.lv, st)) != hipSuccess)
    return hip_fail(he, "gather launch");
  if ((he = hipMemcpyAsync(host_out, p->d_recs, size_t(n) * sizeof(fringe_candidate),
                           hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return hip_fail(he, "copying records");
  return FRINGE_OK;
}

int fringe_window_id(fringe_plan_t p, int32_t scan, int32_t baseline, int32_t window_ap,
                     int32_t t_start, int64_t* id) {
  if (!p || !id) return fail(FRINGE_E_INVALID, "null argument");
  if (scan < 0 || scan >= int(p->sz.scans.size())) return fail(FRINGE_E_INVALID, "scan %d out of range", scan);
  const ScanInfo& si = p->sz.scans[scan];
  if (baseline < 0 || baseline >= si.d.n_baselines)
    return fail(FRINGE_E_INVALID, "baseline %d out of range", baseline);
  int li = -1;
  for (int l = 0; l < p->sz.lv.n; ++l)
    if (p->sz.lv.W[l] == window_ap) li = l;
  if (li < 0) return fail(FRINGE_E_INVALID, "window length %d not in the plan", window_ap);
  // the batch numbering, or the last streaming call's
  const CallScan* c = &si.full;
  if (p->sz.streaming) {
    if (!p->searched || !p->call_present[scan])
      return fail(FRINGE_E_STATE, "scan %d had no chunk in the last search", scan);
    c = &p->call[scan];
  }
  const int s = p->sz.lv.s[li];
  const int64_t rel = int64_t(t_start) - c->t_origin;
  const int64_t j = (rel >= 0 ? rel / s : -1) - c->lvl_j0[li];
  const int64_t n_l = c->lvl_off[li + 1] - c->lvl_off[li];
  if (rel < 0 || rel % s != 0 || j < 0 || j >= n_l)
    return fail(FRINGE_E_INVALID, "no window of length %d starts at %d", window_ap, t_start);
  *id = c->win_off + int64_t(baseline) * c->nwb + c->lvl_off[li] + j;
  return FRINGE_OK;
}

int fringe_grid_get(fringe_plan_t p, int64_t id, fringe_cf32* host_out, int64_t capacity) {
  if (!p || !host_out) return fail(FRINGE_E_INVALID, "null argument");
  if (!p->grid) return fail(FRINGE_E_STATE, "plan was made without FRINGE_DUMP_GRID");
  if (!p->searched) return fail(FRINGE_E_STATE, "fringe_grid_get before fringe_search");
  int s, b, li;
  int64_t j;
  int rc = decode_id(p, id, &s, &b, &li, &j);
  if (rc) return rc;
  const ScanInfo& si = p->sz.scans[s];
  const int64_t mt = int64_t(si.pad_t) * p->sz.lv.W[li];
  const int64_t n = mt * si.M;
  if (capacity < n) return fail(FRINGE_E_CAPACITY, "grid has %lld samples", (long long)n);
  const int64_t off = si.grid_off + int64_t(b) * si.grid_per_bl + si.lvl_goff[li] + j * n;
  hipError_t he = hipEventSynchronize(p->done);
  if (he == hipSuccess)
    he = hipMemcpy(host_out, p->grid + off, size_t(n) * sizeof(float2), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(he, "copying grid");
  return FRINGE_OK;
}

int fringe_set_gains(fringe_plan_t p, int32_t scan, const fringe_cf32* d_gains) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  if (scan < 0 || scan >= int32_t(p->gains.size()))
    return fail(FRINGE_E_INVALID, "scan %d out of range [0, %d)", scan, int(p->gains.size()));
  p->gains[size_t(scan)] = reinterpret_cast<const float2*>(d_gains);
  return FRINGE_OK;
}

int fringe_set_shifts(fringe_plan_t p, int32_t scan, const int32_t* d_shifts) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  if (scan < 0 || scan >= int32_t(p->shifts.size()))
    return fail(FRINGE_E_INVALID, "scan %d out of range [0, %d)", scan, int(p->shifts.size()));
  if (d_shifts && (p->params.flags & FRINGE_PLAIN))
    return fail(FRINGE_E_UNSUPPORTED, "dedispersion needs the whole scan: not with FRINGE_PLAIN");
  if (p->sz.streaming) {
    // the stage must hold the lookahead of the largest shift: set before
    // the plan's first search, the plan is made again with that stage
    const size_t k = size_t(scan);
    if (p->searched)
      return fail(FRINGE_E_STATE, "streaming plans take shifts before their first search");
    int d_max = 0;
    if (d_shifts) {
      const ScanInfo& si = p->sz.scans[k];
      std::vector<int32_t> h(size_t(si.F));
      const hipError_t he =
          hipMemcpy(h.data(), d_shifts, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (he != hipSuccess) return hip_fail(he, "reading the shifts");
      for (int32_t v : h) d_max = std::max(d_max, int(v));
      if (d_max > (1 << 20))
        return fail(FRINGE_E_UNSUPPORTED, "subarray %d: shifts above 2^20 APs", scan);
    }
    if (d_max != p->lookahead[k]) {
      std::vector<int> la = p->lookahead;
      la[k] = d_max;
      const int rc = remake_plan(p, p->force, la);
      if (rc != FRINGE_OK) return rc;
    }
  }
  if (d_shifts) {
    const ScanInfo& si = p->sz.scans[size_t(scan)];
    if (int64_t(data_len(si, p->sz.streaming)) * si.F * int64_t(sizeof(float2)) >= (int64_t(1) << 30))
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: dedispersion needs baselines under 1 GiB", scan);
  }
  p->shifts[size_t(scan)] = d_shifts;
  return FRINGE_OK;
}

int fringe_plan_set_chunk(fringe_plan_t p, int32_t scan, int32_t chunk) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  const int ns = int(p->sz.scans.size());
  if (scan < 0 || scan >= ns) return fail(FRINGE_E_INVALID, "scan %d out of range [0, %d)", scan, ns);
  if (!p->sz.fused)
    return fail(FRINGE_E_UNSUPPORTED, "plans with windows longer than 64 APs have a fixed chunk");
  const int period = fused_period(p->sz.w_max);
  if (chunk != 0 && (chunk < 64 || chunk > 1024 || chunk % period != 0))
    return fail(FRINGE_E_INVALID, "chunk %d: 0, or a multiple of %d in [64, 1024]", chunk, period);
  if (p->searched) return fail(FRINGE_E_STATE, "the chunk is set before the plan's first search");
  std::vector<ScanForce> f = p->force;
  if (f.empty()) f.assign(size_t(ns), ScanForce{});
  f[size_t(scan)].chunk = chunk;
  f[size_t(scan)].exact = chunk != 0;
  return remake_plan(p, f, p->lookahead);
}

int fringe_plan_get_chunk(fringe_plan_t p, int32_t scan, int32_t* chunk) {
  if (!p || !chunk) return fail(FRINGE_E_INVALID, "null argument");
  const int ns = int(p->sz.scans.size());
  if (scan < 0 || scan >= ns) return fail(FRINGE_E_INVALID, "scan %d out of range [0, %d)", scan, ns);
  *chunk = p->sz.scans[size_t(scan)].chunk;
  return FRINGE_OK;
}

int fringe_profile_get(fringe_plan_t p, fringe_profile* out) {
  if (!p || !out) return fail(FRINGE_E_INVALID, "null argument");
  if (!(p->params.flags & FRINGE_PROFILE)) return fail(FRINGE_E_STATE, "plan was made without FRINGE_PROFILE");
  if (!p->searched) return fail(FRINGE_E_STATE, "fringe_profile_get before fringe_search");
  hipError_t he = hipEventSynchronize(p->done);
  if (he != hipSuccess) return hip_fail(he, "hipEventSynchronize");
  double ms[4] = {0, 0, 0, 0};
  int n[4] = {0, 0, 0, 0};
  for (size_t i = 0; i < p->prof_used; ++i) {
    float t = 0.f;
    he = hipEventElapsedTime(&t, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]);
    if (he != hipSuccess) return hip_fail(he, "hipEventElapsedTime");
    ms[p->prof_kind[i]] += t;
    n[p->prof_kind[i]] += 1;
  }
  out->delay_ms = ms[0];
  out->rate_ms = ms[1];
  out->finalize_ms = ms[2];
  out->compact_ms = ms[3];
  out->delay_launches = n[0];
  out->rate_launches = n[1];
  out->finalize_launches = n[2];
  out->compact_launches = n[3];
  return FRINGE_OK;
}

int fringe_plan_info(fringe_plan_t p, fringe_plan_summary* out) {
  if (!p || !out) return fail(FRINGE_E_INVALID, "null argument");
  out->n_windows = p->sz.streaming ? p->call_windows : p->sz.n_windows;
  out->device_bytes = int64_t(p->sz.total);
  out->scratch_bytes = int64_t(p->sz.scratch_x + p->sz.scratch_e + p->sz.scratch_part +
                               p->sz.scratch_epart);
  out->max_window_ap = p->sz.w_max;
  int mn = 1 << 30;
  for (auto& si : p->sz.scans) mn = std::min(mn, si.slab_nb);
  out->slab_baselines = mn;
  return FRINGE_OK;
}

void fringe_plan_destroy(fringe_plan_t p) { release(p); }

int fringe_search_noalloc(const fringe_scan_desc* scan, const fringe_params* params,
                          const fringe_cf32* d_vis, fringe_candidate* d_out, int64_t capacity,
                          int64_t* d_total, void* hip_stream) {
  if (!scan || !params || !d_vis || !d_total)
    return fail(FRINGE_E_INVALID, "null scan, params, visibility or count pointer");
  if (capacity < 0 || (capacity > 0 && !d_out))
    return fail(FRINGE_E_INVALID, "bad candidate buffer (capacity %lld)", (long long)capacity);
  if (params->flags & ~uint32_t(FRINGE_DELAY_ONLY))
    return fail(FRINGE_E_INVALID, "fringe_search_noalloc takes no flags but FRINGE_DELAY_ONLY");
  fringe_params q = *params;
  q.hbm_budget_bytes = 0;
  q.max_candidates = 0;
  Sizing z;
  int rc = validate_and_size(scan, 1, &q, &z, /*allow_spectra=*/false);
  if (rc != FRINGE_OK) return rc;
  if (!z.fused)
    return fail(FRINGE_E_UNSUPPORTED, "fringe_search_noalloc: windows of at most %d APs",
                kFusedMaxWindow);
  const ScanInfo& si0 = z.scans[0];
  // work buffers, 256-byte aligned, in the scratch
  const uint64_t n_win = uint64_t(z.n_windows);
  const uint64_t n_blk = uint64_t(z.n_blocks);
  const uint64_t b_desc = align_up(sizeof(NoAllocDesc));
  const uint64_t b_part = align_up(size_t(si0.n_kb) * n_win * sizeof(uint64_t));
  const uint64_t b_epart = z.delay_only ? align_up(size_t(si0.n_kb) * n_win * sizeof(float)) : 0;
  const uint64_t b_e = align_up(size_t(si0.d.n_baselines) * si0.d.n_ap * sizeof(float));
  const uint64_t b_table = align_up(n_win * sizeof(WindowRec));
  const uint64_t b_cnt = align_up(n_blk * sizeof(int32_t));
  const uint64_t b_off = align_up(n_blk * sizeof(int64_t));
  const uint64_t need = b_desc + b_part + b_epart + b_e + b_table + b_cnt + b_off;
  if (z.units.size() != 1 || need > kNoAllocScratchBytes)
    return fail(FRINGE_E_NOMEM, "fringe_search_noalloc: the scan needs %llu bytes of work "
                "buffers, the static scratch holds %llu",
                (unsigned long long)need, (unsigned long long)kNoAllocScratchBytes);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0, n_cu = 0;
  hipError_t he;
  if ((he = hipGetDevice(&dev)) != hipSuccess ||
      (he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(he, "device attributes");
  const int pad_t_kernel = z.delay_only ? 0 : params->pad_time;
  if ((rc = tune_chunks(&z, std::max(1, n_cu), pad_t_kernel)) != FRINGE_OK) return rc;
  char* base = nullptr;
  if ((rc = scratch_base(&base)) != FRINGE_OK) return rc;
  const ScanInfo& si = z.scans[0];
  WorkBufs w;
  char* cur = base + b_desc;
  w.part = reinterpret_cast<uint64_t*>(cur);
  cur += b_part;
  w.epart = z.delay_only ? reinterpret_cast<float*>(cur) : nullptr;
  cur += b_epart;
  w.e = reinterpret_cast<float*>(cur);
  cur += b_e;
  w.table = reinterpret_cast<WindowRec*>(cur);
  cur += b_table;
  int32_t* blk_counts = reinterpret_cast<int32_t*>(cur);
  cur += b_cnt;
  int64_t* blk_offsets = reinterpret_cast<int64_t*>(cur);
  if ((he = twiddles_for(si.M, &w.tw)) != hipSuccess) return hip_fail(he, "twiddle table");
  CallScan c = si.full;
  c.win_off = 0;
  const Unit& u = z.units[0];
  NoAllocDesc d{};
  d.sd = make_scan_dev(si, c);
  d.fa = fused_entry(z, w, si, c, u, reinterpret_cast<const float2*>(d_vis),
                     int64_t(si.d.n_ap) * si.F);
  d.fa.block_off = 0;
  d.fi = finalize_entry(z, w, si, c, u);
  d.fi.win_begin = 0;
  NoAllocDesc* dd = reinterpret_cast<NoAllocDesc*>(base);
  hipLaunchKernelGGL(put_desc_kernel, dim3(1), dim3(64), 0, st, d, dd);
  if ((he = hipGetLastError()) != hipSuccess) return hip_fail(he, "descriptor launch");
  if (n_win > 0) {
    if ((he = launch_fused(&dd->fa, 1, fused_blocks(d.fa), pad_t_kernel, z.w_max, u.fc, false,
                           st)) != hipSuccess)
      return hip_fail(he, "fused search launch");
    if ((he = launch_finalize(&dd->fi, 1, int64_t(n_win), st)) != hipSuccess)
      return hip_fail(he, "finalize launch");
  }
  CompactArgs ca{};
  ca.table = w.table;
  ca.n_windows = int64_t(n_win);
  ca.threshold = params->snr_threshold;
  ca.blk_counts = blk_counts;
  ca.blk_offsets = blk_offsets;
  ca.n_blocks = int64_t(n_blk);
  ca.out = d_out;
  ca.max_out = capacity;
  ca.total = d_total;
  ca.scans = &dd->sd;
  ca.n_scans = 1;
  ca.lv = z.lv;
  if ((he = launch_compact(ca, st)) != hipSuccess) return hip_fail(he, "compaction launch");
  return FRINGE_OK;
}

}  // extern "C"

namespace fringe {
// Lets the host-only consumers (matching, localization) report their
// failures through fringe_last_error.
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace fringe
