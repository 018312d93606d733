// Window results and candidate list.
//
// finalize: per window, the max of the bin-block peak keys (window_key.h),
//   the window energy E = sum of its APs' energies (= mean |G|^2 by
//   Parseval; delay-only: the classes' sums of |G_0|^2 over M_f),
//   amp = sqrt(P_peak), SNR = amp / sqrt(E) (0 when E = 0).
// compact: the windows with SNR > threshold (paper, section "Detection
//   rate") in window-id order, i.e. sorted by (scan, baseline, window
//   length, start): per-block counts, one exclusive scan, then an ordered
//   scatter (wave ballot ranks + per-wave offsets), so the list is
//   deterministic and the first max_out candidates are the ones kept.
#include "dev_common.h"
#include "kernels.h"

namespace fringe {

namespace {

__global__ void __launch_bounds__(256) finalize_kernel(const FinalizeArgs* __restrict__ tab,
                                                       int n_tab, int64_t n_windows) {
  const int64_t wa = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (wa >= n_windows) return;
  int e_lo = 0, e_hi = n_tab - 1;  // the entry owning window wa
  while (e_lo < e_hi) {
    const int mid = (e_lo + e_hi + 1) >> 1;
    if (tab[mid].win_begin <= wa) e_lo = mid; else e_hi = mid - 1;
  }
  const FinalizeArgs& a = tab[e_lo];
  const int64_t w = wa - a.win_begin;
  uint64_t key = 0;
  for (int kb = 0; kb < a.n_kb; ++kb) {
    const uint64_t k = a.part[static_cast<int64_t>(kb) * a.slab_windows + w];
    key = k > key ? k : key;
  }
  const int b = static_cast<int>(w / a.nwb);
  const int rem = static_cast<int>(w - static_cast<int64_t>(b) * a.nwb);
  int li = 0;
  while (li + 1 < a.lv.n && rem >= a.lvl_off[li + 1]) ++li;
  const int j = rem - a.lvl_off[li] + a.lvl_j0[li];
  const int t0 = j * a.lv.s[li];
  double energy = 0.0;
  uint32_t mask = 0;
  if (a.epart) {
    // delay-only: mean over the M_f delay bins of |G_0|^2 from the classes'
    // sums; the key is the power itself (rate bin 0)
    for (int kb = 0; kb < a.n_kb; ++kb)
      energy += a.epart[static_cast<int64_t>(kb) * a.slab_windows + w];
    energy /= a.M;
  } else {
    const float* eb = a.e + static_cast<int64_t>(b) * a.T + t0;
    for (int u = 0; u < a.lv.W[li]; ++u) energy += eb[u];
    // key = (rate key << 32) | (0xFFFFFFFF - k_f); rate key = power bits
    // with the low log2(M_t) bits replaced by M_t - 1 - k_t
    mask = static_cast<uint32_t>(a.pad_t * a.lv.W[li] - 1);
  }
  const uint32_t hi = static_cast<uint32_t>(key >> 32);
  const float p = __uint_as_float(hi & ~mask);
  const uint32_t k_t = mask - (hi & mask);
  const uint32_t k_f = 0xFFFFFFFFu - static_cast<uint32_t>(key);
  WindowRec r;
  r.flat = k_t * static_cast<uint32_t>(a.M) + k_f;
  const double amp = sqrt(static_cast<double>(p));
  if (energy > 0.0) {
    r.amp = static_cast<float>(amp);
    r.snr = static_cast<float>(amp / sqrt(energy));
  } else {  // all-zero window: peak (0, 0), amplitude and SNR 0
    r.amp = 0.f;
    r.snr = 0.f;
    r.flat = 0;
  }
  r.energy = static_cast<float>(energy);
  a.table[w] = r;
}

// Candidate record of window `w` from its table entry.
__device__ void decode_window(int64_t w, const WindowRec& rec, const ScanDev* scans, int n_scans,
                              const LevelTable& lv, fringe_candidate* out) {
  int lo = 0, hi = n_scans - 1;
  while (lo < hi) {  // last scan whose first id <= w
    const int mid = (lo + hi + 1) >> 1;
    if (scans[mid].win_off <= w) lo = mid; else hi = mid - 1;
  }
  const ScanDev& sc = scans[lo];
  const int64_t loc = w - sc.win_off;
  const int b = static_cast<int>(loc / sc.nwb);
  const int rem = static_cast<int>(loc - static_cast<int64_t>(b) * sc.nwb);
  int li = 0;
  while (li + 1 < lv.n && rem >= sc.lvl_off[li + 1]) ++li;
  const int j = rem - sc.lvl_off[li] + sc.lvl_j0[li];
  const int wl = lv.W[li];
  const int m_t = sc.pad_t * wl;
  const int k_t = static_cast<int>(rec.flat >> sc.log_mf);
  const int k_f = static_cast<int>(rec.flat & static_cast<uint32_t>(sc.M_f - 1));
  const int sk_f = k_f >= sc.M_f / 2 ? k_f - sc.M_f : k_f;
  const int sk_t = k_t >= m_t / 2 ? k_t - m_t : k_t;
  fringe_candidate c;
  c.scan = lo;
  c.baseline = b;
  c.window_ap = wl;
  c.t_start = static_cast<int32_t>(sc.t_origin + static_cast<int64_t>(j) * lv.s[li]);
  c.k_rate = k_t;
  c.k_delay = k_f;
  c.amp = rec.amp;
  c.snr = rec.snr;
  c.energy = rec.energy;
  c.reserved = 0;
  c.delay_s = static_cast<double>(sk_f) / (static_cast<double>(sc.M_f) * sc.df);
  c.rate_hz = static_cast<double>(sk_t) / (static_cast<double>(m_t) * sc.tap);
  *out = c;
}

constexpr int kThreads = 256;
constexpr int kRounds = kCompactBlock / kThreads;

__global__ void __launch_bounds__(kThreads) count_kernel(CompactArgs a) {
  __shared__ int wsum[kThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactBlock;
  int c = 0;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t w = base + r * kThreads + threadIdx.x;
    if (w < a.n_windows && a.table[w].snr > a.threshold) ++c;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < kThreads / 64; ++i) t += wsum[i];
    a.blk_counts[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts in one work group.
__global__ void __launch_bounds__(1024) scan_kernel(CompactArgs a) {
  __shared__ int64_t wtot[16];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < a.n_blocks; base += 1024) {
    const int64_t i = base + tid;
    const int64_t v = i < a.n_blocks ? a.blk_counts[i] : 0;
    int64_t incl = v;  // inclusive scan within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    int64_t before = carry;
    for (int k = 0; k < wid; ++k) before += wtot[k];
    if (i < a.n_blocks) a.blk_offsets[i] = before + incl - v;
    __syncthreads();
    if (tid == 0) {
      int64_t t = 0;
      for (int k = 0; k < 16; ++k) t += wtot[k];
      carry += t;
    }
    __syncthreads();
  }
  if (tid == 0) *a.total = carry;
}

__global__ void __launch_bounds__(kThreads) scatter_kernel(CompactArgs a) {
  __shared__ int wcnt[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactBlock;
  int64_t pos0 = a.blk_offsets[blockIdx.x];
  for (int r = 0; r < kRounds; ++r) {
    const int64_t w = base + r * kThreads + threadIdx.x;
    WindowRec rec{};
    bool flag = false;
    if (w < a.n_windows) {
      rec = a.table[w];
      flag = rec.snr > a.threshold;
    }
    const uint64_t mask = __ballot(flag);
    const int rank = __popcll(mask & __lanemask_lt());
    if (lane == 0) wcnt[wid] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < kThreads / 64; ++k) {
      if (k < wid) before += wcnt[k];
      total += wcnt[k];
    }
    const int64_t pos = pos0 + before + rank;
    if (flag && pos < a.max_out) decode_window(w, rec, a.scans, a.n_scans, a.lv, a.out + pos);
    pos0 += total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) gather_kernel(const WindowRec* table, const int64_t* ids,
                                                     int64_t n, fringe_candidate* out,
                                                     const ScanDev* scans, int n_scans,
                                                     LevelTable lv) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t w = ids[i];
  decode_window(w, table[w], scans, n_scans, lv, out + i);
}

}  // namespace

hipError_t launch_finalize(const FinalizeArgs* d_tab, int n_tab, int64_t n_windows,
                           hipStream_t st) {
  if (n_windows == 0 || n_tab == 0) return hipSuccess;
  const int64_t blocks = (n_windows + 255) / 256;
  hipLaunchKernelGGL(finalize_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     d_tab, n_tab, n_windows);
  return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs& a, hipStream_t st) {
  if (a.n_blocks > 0) {
    hipLaunchKernelGGL(count_kernel, dim3(static_cast<unsigned>(a.n_blocks)), dim3(kThreads), 0,
                       st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.n_blocks == 0) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(static_cast<unsigned>(a.n_blocks)), dim3(kThreads), 0,
                     st, a);
  return hipGetLastError();
}

hipError_t launch_gather(const WindowRec* table, const int64_t* ids, int64_t n,
                         fringe_candidate* out, const ScanDev* scans, int n_scans,
                         const LevelTable& lv, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, table,
                     ids, n, out, scans, n_scans, lv);
  return hipGetLastError();
}

}  // namespace fringe
