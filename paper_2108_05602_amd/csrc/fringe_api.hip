// Host side of libfringe: parameter validation, window enumeration, plan
// sizing and device memory, and the launch sequence of one search.
//
// Window numbering (the order of every table and of the candidate list):
//   id = scan_offset + baseline * n_per_baseline + level_offset[level] + j,
//   t_start = j * stride(W),  stride(W) = max(1, W / 2),
// for window lengths in ascending order and starts t with t + W <= n_ap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

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

constexpr uint64_t kDefaultScratchCap = 8ull << 30;  // work buffers when no budget is given
constexpr uint64_t kMaxDumpBytes = 1ull << 30;

struct ScanInfo {
  fringe_scan_desc d;
  int F, M, log_m, n_kb, pad_t;
  int64_t nwb;                        // windows per baseline
  int64_t lvl_off[kMaxLevels + 1];
  int64_t n_windows;                  // nb * nwb
  int64_t win_off;                    // first window id
  int64_t grid_per_bl;                // grid elements per baseline (dump)
  int64_t lvl_goff[kMaxLevels];
  int64_t grid_off;                   // first grid element of the scan (dump)
  int slab_nb;                        // baselines per pass
  int chunk, n_chunks;                // rate-kernel time tiling
};

struct Sizing {
  std::vector<ScanInfo> scans;
  LevelTable lv;
  int w_max = 0;
  int64_t n_windows = 0;
  int64_t n_blocks = 0;
  uint64_t scratch_x = 0, scratch_e = 0, scratch_part = 0;
  uint64_t table_bytes = 0, blk_bytes = 0, cand_bytes = 0, grid_bytes = 0, fixed_bytes = 0;
  uint64_t total = 0;
};

uint64_t per_baseline_scratch(const ScanInfo& s) {
  return uint64_t(s.d.n_ap) * s.M * sizeof(float2) + uint64_t(s.d.n_ap) * sizeof(float) +
         uint64_t(s.n_kb) * s.nwb * sizeof(uint64_t);
}

int validate_and_size(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* p,
                      Sizing* out) {
  if (!scans || !p || !out) return fail(FRINGE_E_INVALID, "null argument");
  if (n_scans < 1) return fail(FRINGE_E_INVALID, "n_scans must be >= 1 (got %d)", n_scans);
  if (!p->window_aps) return fail(FRINGE_E_INVALID, "window_aps is null");
  if (p->n_window_lengths < 1 || p->n_window_lengths > kMaxLevels)
    return fail(FRINGE_E_INVALID, "n_window_lengths must be in [1, %d]", kMaxLevels);
  if (p->flags & ~(FRINGE_STREAMING | FRINGE_DUMP_GRID | FRINGE_PROFILE))
    return fail(FRINGE_E_INVALID, "unknown flag bits 0x%x", p->flags);
  if (p->flags & FRINGE_STREAMING)
    return fail(FRINGE_E_UNSUPPORTED, "FRINGE_STREAMING is not available in this build");
  if (!(p->snr_threshold >= 0.f) || !std::isfinite(p->snr_threshold))
    return fail(FRINGE_E_INVALID, "snr_threshold must be finite and >= 0");
  if (p->max_candidates < 0) return fail(FRINGE_E_INVALID, "max_candidates must be >= 0");
  if (p->pad_freq != 1 && p->pad_freq != 2 && p->pad_freq != 4)
    return fail(FRINGE_E_UNSUPPORTED, "pad_freq must be 1, 2 or 4 (got %d)", p->pad_freq);
  if (p->pad_time != 1 && p->pad_time != 2)
    return fail(FRINGE_E_UNSUPPORTED, "pad_time must be 1 or 2 (got %d)", p->pad_time);

  Sizing sz;
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
    int64_t off = 0, goff = 0;
    for (int l = 0; l < sz.lv.n; ++l) {
      const int w = sz.lv.W[l];
      const int64_t nl = d.n_ap >= w ? (int64_t(d.n_ap) - w) / sz.lv.s[l] + 1 : 0;
      si.lvl_off[l] = off;
      si.lvl_goff[l] = goff;
      off += nl;
      goff += nl * int64_t(p->pad_time) * w * M;
    }
    for (int l = sz.lv.n; l <= kMaxLevels; ++l) si.lvl_off[l] = off;
    si.nwb = off;
    si.grid_per_bl = goff;
    si.n_windows = off * d.n_baselines;
    if (si.nwb > (int64_t(1) << 30) || si.n_windows > (int64_t(1) << 40))
      return fail(FRINGE_E_UNSUPPORTED, "scan %d: too many windows", s);
    si.win_off = win_off;
    si.grid_off = grid_off;
    win_off += si.n_windows;
    grid_off += si.grid_per_bl * d.n_baselines;
    si.chunk = std::min(1024, std::max(128, 8 * sz.w_max));
    si.n_chunks = int((int64_t(d.n_ap) + si.chunk - 1) / si.chunk);
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
  uint64_t tw_bytes = 0;
  for (int lm = 6; lm <= 12; ++lm)
    for (auto& si : sz.scans)
      if (si.log_m == lm) { tw_bytes += (uint64_t(1) << lm) * sizeof(float2); break; }
  sz.fixed_bytes = sz.table_bytes + sz.blk_bytes + sz.cand_bytes + sz.grid_bytes + tw_bytes +
                   uint64_t(n_scans) * sizeof(ScanDev) + 64;

  // Work buffers: process each scan in slabs of baselines that fit.
  uint64_t cap = kDefaultScratchCap;
  if (p->hbm_budget_bytes > 0) {
    if (p->hbm_budget_bytes <= sz.fixed_bytes)
      return fail(FRINGE_E_NOMEM, "hbm_budget_bytes %llu below the %llu bytes of results",
                  (unsigned long long)p->hbm_budget_bytes, (unsigned long long)sz.fixed_bytes);
    cap = p->hbm_budget_bytes - sz.fixed_bytes;
  }
  for (auto& si : sz.scans) {
    const uint64_t per = per_baseline_scratch(si);
    int64_t nb = int64_t(cap / per);
    if (nb < 1) {
      if (p->hbm_budget_bytes > 0)
        return fail(FRINGE_E_NOMEM, "one baseline of scan needs %llu work bytes, budget leaves %llu",
                    (unsigned long long)per, (unsigned long long)cap);
      nb = 1;
    }
    si.slab_nb = int(std::min<int64_t>(nb, si.d.n_baselines));
    sz.scratch_x = std::max<uint64_t>(sz.scratch_x, uint64_t(si.slab_nb) * si.d.n_ap * si.M * sizeof(float2));
    sz.scratch_e = std::max<uint64_t>(sz.scratch_e, uint64_t(si.slab_nb) * si.d.n_ap * sizeof(float));
    sz.scratch_part = std::max<uint64_t>(sz.scratch_part, uint64_t(si.slab_nb) * si.nwb * si.n_kb * sizeof(uint64_t));
  }
  sz.total = sz.fixed_bytes + sz.scratch_x + sz.scratch_e + sz.scratch_part;
  *out = std::move(sz);
  return FRINGE_OK;
}

}  // namespace

struct fringe_plan_s {
  Sizing sz;
  fringe_params params{};
  std::vector<int32_t> window_aps;
  int device = 0;
  float2* X = nullptr;
  float* e = nullptr;
  uint64_t* part = nullptr;
  WindowRec* table = nullptr;
  int32_t* blk_counts = nullptr;
  int64_t* blk_offsets = nullptr;
  fringe_candidate* cands = nullptr;
  int64_t* d_total = nullptr;
  ScanDev* d_scans = nullptr;
  float2* grid = nullptr;
  float2* tw[13] = {};
  int64_t* h_total = nullptr;      // pinned
  int64_t* d_ids = nullptr;        // windows_get staging
  fringe_candidate* d_recs = nullptr;
  int64_t staging_cap = 0;
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool searched = false;
  // FRINGE_PROFILE: an event pair per launch, kind 0..3 = delay, rate, finalize, compact
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
  size_t prof_used = 0;
};

namespace {

void release(fringe_plan_t p) {
  if (!p) return;
  if (p->searched && p->done) (void)hipEventSynchronize(p->done);
  void* bufs[] = {p->X, p->e, p->part, p->table, p->blk_counts, p->blk_offsets, p->cands,
                  p->d_total, p->d_scans, p->grid, p->d_ids, p->d_recs};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (auto* t : p->tw)
    if (t) (void)hipFree(t);
  if (p->h_total) (void)hipHostFree(p->h_total);
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

int decode_id(const fringe_plan_s* p, int64_t id, int* scan, int* b, int* li, int64_t* j) {
  if (id < 0 || id >= p->sz.n_windows) return fail(FRINGE_E_INVALID, "window id %lld out of range", (long long)id);
  int s = 0;
  while (s + 1 < int(p->sz.scans.size()) && p->sz.scans[s + 1].win_off <= id) ++s;
  const ScanInfo& si = p->sz.scans[s];
  const int64_t loc = id - si.win_off;
  const int64_t bb = loc / si.nwb;
  const int64_t rem = loc - bb * si.nwb;
  int l = 0;
  while (l + 1 < p->sz.lv.n && rem >= si.lvl_off[l + 1]) ++l;
  *scan = s;
  *b = int(bb);
  *li = l;
  *j = rem - si.lvl_off[l];
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
  out->scratch_bytes = int64_t(sz.scratch_x + sz.scratch_e + sz.scratch_part);
  out->max_window_ap = sz.w_max;
  int mn = 1 << 30;
  for (auto& si : sz.scans) mn = std::min(mn, si.slab_nb);
  out->slab_baselines = mn;
  return FRINGE_OK;
}

int fringe_plan(const fringe_scan_desc* scans, int32_t n_scans, const fringe_params* params,
                fringe_plan_t* out) {
  if (!out) return fail(FRINGE_E_INVALID, "null plan output pointer");
  *out = nullptr;
  Sizing sz;
  int rc = validate_and_size(scans, n_scans, params, &sz);
  if (rc != FRINGE_OK) return rc;
  auto* p = new fringe_plan_s();
  p->sz = std::move(sz);
  p->params = *params;
  p->window_aps.assign(params->window_aps, params->window_aps + params->n_window_lengths);
  p->params.window_aps = p->window_aps.data();
  hipError_t he = hipGetDevice(&p->device);
  if (he != hipSuccess) {
    release(p);
    return hip_fail(he, "hipGetDevice");
  }
  const Sizing& z = p->sz;
  if ((rc = dev_alloc(&p->X, z.scratch_x, "delay spectra")) ||
      (rc = dev_alloc(&p->e, z.scratch_e, "AP energies")) ||
      (rc = dev_alloc(&p->part, z.scratch_part, "bin-block peaks")) ||
      (rc = dev_alloc(&p->table, z.table_bytes, "window table")) ||
      (rc = dev_alloc(&p->blk_counts, uint64_t(z.n_blocks) * sizeof(int32_t), "block counts")) ||
      (rc = dev_alloc(&p->blk_offsets, uint64_t(z.n_blocks) * sizeof(int64_t), "block offsets")) ||
      (rc = dev_alloc(&p->cands, z.cand_bytes, "candidates")) ||
      (rc = dev_alloc(&p->d_total, sizeof(int64_t), "candidate count")) ||
      (rc = dev_alloc(&p->d_scans, z.scans.size() * sizeof(ScanDev), "scan table")) ||
      (rc = dev_alloc(&p->grid, z.grid_bytes, "grid dump"))) {
    release(p);
    return rc;
  }
  // twiddle tables exp(-2 pi i k / M), rounded from double
  for (auto& si : z.scans) {
    if (p->tw[si.log_m]) continue;
    std::vector<float2> t(size_t(si.M));
    for (int k = 0; k < si.M; ++k) {
      const double a = -2.0 * M_PI * double(k) / double(si.M);
      t[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    if ((rc = dev_alloc(&p->tw[si.log_m], t.size() * sizeof(float2), "twiddles"))) {
      release(p);
      return rc;
    }
    he = hipMemcpy(p->tw[si.log_m], t.data(), t.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      release(p);
      return hip_fail(he, "hipMemcpy(twiddles)");
    }
  }
  std::vector<ScanDev> sd(z.scans.size());
  for (size_t s = 0; s < z.scans.size(); ++s) {
    const ScanInfo& si = z.scans[s];
    ScanDev d{};
    d.win_off = si.win_off;
    d.nb = si.d.n_baselines;
    d.T = si.d.n_ap;
    d.M_f = si.M;
    d.log_mf = si.log_m;
    d.nwb = int32_t(si.nwb);
    d.pad_t = si.pad_t;
    d.df = si.d.chan_width_hz;
    d.tap = si.d.ap_seconds;
    for (int l = 0; l <= kMaxLevels; ++l) d.lvl_off[l] = int32_t(si.lvl_off[l]);
    sd[s] = d;
  }
  he = hipMemcpy(p->d_scans, sd.data(), sd.size() * sizeof(ScanDev), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    release(p);
    return hip_fail(he, "hipMemcpy(scan table)");
  }
  if ((he = hipHostMalloc(reinterpret_cast<void**>(&p->h_total), sizeof(int64_t), hipHostMallocDefault)) !=
          hipSuccess ||
      (he = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess) {
    release(p);
    return hip_fail(he, "plan host resources");
  }
  *out = p;
  return FRINGE_OK;
}

int fringe_search(fringe_plan_t p, const fringe_cf32* const* d_vis, void* hip_stream) {
  if (!p) return fail(FRINGE_E_INVALID, "null plan");
  if (!d_vis) return fail(FRINGE_E_INVALID, "null visibility pointer array");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const Sizing& z = p->sz;
  for (size_t s = 0; s < z.scans.size(); ++s)
    if (!d_vis[s]) return fail(FRINGE_E_INVALID, "scan %zu: null visibility pointer", s);
  hipError_t he;
  p->prof_used = 0;
#define FRINGE_TIMED(kind, call, what)                                        \
  do {                                                                        \
    if ((he = prof_begin(p, kind, st)) != hipSuccess) return hip_fail(he, "profiling event"); \
    if ((he = (call)) != hipSuccess) return hip_fail(he, what);               \
    if ((he = prof_end(p, st)) != hipSuccess) return hip_fail(he, "profiling event"); \
  } while (0)
  for (size_t s = 0; s < z.scans.size(); ++s) {
    const ScanInfo& si = z.scans[s];
    const float2* vis = reinterpret_cast<const float2*>(d_vis[s]);
    for (int b0 = 0; b0 < si.d.n_baselines; b0 += si.slab_nb) {
      const int nb = std::min(si.slab_nb, si.d.n_baselines - b0);
      DelayArgs da{};
      da.vis = vis + int64_t(b0) * si.d.n_ap * si.F;
      da.X = p->X;
      da.e = p->e;
      da.tw = p->tw[si.log_m];
      da.nb = nb;
      da.T = si.d.n_ap;
      da.F = si.F;
      da.M = si.M;
      da.log_m = si.log_m;
      da.pad_f = p->params.pad_freq;
      FRINGE_TIMED(0, launch_delay_fft(da, st), "delay transform launch");

      RateArgs ra{};
      ra.X = p->X;
      ra.part = p->part;
      ra.dump = p->grid;
      ra.slab_windows = int64_t(nb) * si.nwb;
      ra.dump_base = si.grid_off + int64_t(b0) * si.grid_per_bl;
      ra.grid_per_bl = si.grid_per_bl;
      for (int l = 0; l < kMaxLevels; ++l) ra.lvl_goff[l] = si.lvl_goff[l];
      ra.nb = nb;
      ra.T = si.d.n_ap;
      ra.M = si.M;
      ra.log_m = si.log_m;
      ra.n_kb = si.n_kb;
      ra.chunk = si.chunk;
      ra.n_chunks = si.n_chunks;
      ra.w_max = z.w_max;
      ra.buf_slots = rate_buffer_slots(z.w_max);
      ra.pad_t = si.pad_t;
      ra.nwb = int(si.nwb);
      for (int l = 0; l <= kMaxLevels; ++l) ra.lvl_off[l] = int(si.lvl_off[l]);
      ra.lv = z.lv;
      FRINGE_TIMED(1, launch_rate_peak(ra, st), "rate transform launch");

      FinalizeArgs fa{};
      fa.part = p->part;
      fa.e = p->e;
      fa.table = p->table + si.win_off + int64_t(b0) * si.nwb;
      fa.slab_windows = ra.slab_windows;
      fa.n_kb = si.n_kb;
      fa.nb = nb;
      fa.T = si.d.n_ap;
      fa.nwb = int(si.nwb);
      for (int l = 0; l <= kMaxLevels; ++l) fa.lvl_off[l] = int(si.lvl_off[l]);
      fa.lv = z.lv;
      FRINGE_TIMED(2, launch_finalize(fa, st), "finalize launch");
    }
  }
  CompactArgs ca{};
  ca.table = p->table;
  ca.n_windows = z.n_windows;
  ca.threshold = p->params.snr_threshold;
  ca.blk_counts = p->blk_counts;
  ca.blk_offsets = p->blk_offsets;
  ca.n_blocks = z.n_blocks;
  ca.out = p->cands;
  ca.max_out = p->params.max_candidates;
  ca.total = p->d_total;
  ca.scans = p->d_scans;
  ca.n_scans = int(z.scans.size());
  ca.lv = z.lv;
  FRINGE_TIMED(3, launch_compact(ca, st), "compaction launch");
#undef FRINGE_TIMED
  if ((he = hipEventRecord(p->done, st)) != hipSuccess) return hip_fail(he, "hipEventRecord");
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
  if ((he = hipMemcpyAsync(p->h_total, p->d_total, sizeof(int64_t), hipMemcpyDeviceToHost,
                           p->last_stream)) != hipSuccess ||
      (he = hipStreamSynchronize(p->last_stream)) != hipSuccess)
    return hip_fail(he, "reading the candidate count");
  const int64_t total = *p->h_total;
  *n_total = total;
  const int64_t avail = std::min(total, p->params.max_candidates);
  const int64_t n = std::min(avail, capacity);
  if (n > 0) {
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
    if (ids[i] < 0 || ids[i] >= p->sz.n_windows)
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
  const int s = p->sz.lv.s[li];
  if (t_start < 0 || t_start % s != 0 || int64_t(t_start) + window_ap > si.d.n_ap)
    return fail(FRINGE_E_INVALID, "no window of length %d starts at %d", window_ap, t_start);
  *id = si.win_off + int64_t(baseline) * si.nwb + si.lvl_off[li] + t_start / s;
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
  out->n_windows = p->sz.n_windows;
  out->device_bytes = int64_t(p->sz.total);
  out->scratch_bytes = int64_t(p->sz.scratch_x + p->sz.scratch_e + p->sz.scratch_part);
  out->max_window_ap = p->sz.w_max;
  int mn = 1 << 30;
  for (auto& si : p->sz.scans) mn = std::min(mn, si.slab_nb);
  out->slab_baselines = mn;
  return FRINGE_OK;
}

void fringe_plan_destroy(fringe_plan_t p) { release(p); }

}  // extern "C"
