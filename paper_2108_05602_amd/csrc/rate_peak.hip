// Rate transform and grid peak: for every window of every length, the
// zero-padded DFT over the window's APs of each delay bin's spectrum,
//   G[k_t, k_f] = sum_{u<W} X_{t0+u}[k_f] exp(-2 pi i k_t u / M_t),
// followed by the peak of |G|^2 with lowest-flat-index tie-break.  The time
// sum is the paper's window combination (section "Code optimization",
// step 6, which keeps only k_t = 0); M_t = pad_t * W.
//
// Layout: one wavefront per work group; lane l owns delay bin
// k_f = 64 * kb + l of one baseline, so every HBM read of X is a coalesced
// 512-byte row segment.  A wave walks a chunk of APs (plus a halo of
// W_max - 1 APs for the windows that start in the chunk) in batches of kQ,
// keeping the bin's recent history in an LDS column (each lane only ever
// reads its own column, so no barriers are needed).  Every window whose
// last AP arrives in the batch is transformed in registers right away:
//   k_t = S p + r,  G[S p + r] = FFT_N( y_r )[p],
//   y_r[v] = w_{M_t}^{r v} sum_{h<H} x[v + N h] w_S^{r h},
// with N = M_t / S <= 16 sub-transforms (S = max(pad_t, M_t / 16),
// H = W / N), so a W = 128 window never needs more than 16 complex values
// in flight.  The lane's rate key goes through a 64-lane DPP max and one
// lane stores the bin-block's result (window_key.h).
//
// This kernel serves the windows longer than 64 APs (levels l0 and up);
// shorter ones go to the fused kernel (fused_search.h), which does its own
// delay transform and keeps the history in registers, also in plans that
// have long windows.
#include "kernels.h"
#include "window_key.h"

namespace fringe {

namespace {

constexpr int kQ = 8;  // APs per load batch

// One window of one lane's bin: samples from the lane's LDS column (copied
// to registers first for short windows), then the shared rate transform
// and peak key.
template <int L, int PT, bool DUMP>
__device__ __forceinline__ uint32_t window_key_lds(const float2* __restrict__ col,
                                                   float2* __restrict__ dump, int m_f) {
  constexpr int W = 1 << L;
  if constexpr (W <= 32) {
    float2 xr[W];
    static_for<0, W>([&](auto ui) {
      constexpr int u = decltype(ui)::value;
      xr[u] = col[u * kBinsPerWave];
    });
    return window_key<L, PT, DUMP>([&](auto ui) { return xr[decltype(ui)::value]; }, dump, m_f);
  } else {
    return window_key<L, PT, DUMP>(
        [&](auto ui) { return col[decltype(ui)::value * kBinsPerWave]; }, dump, m_f);
  }
}

// Only the lengths up to 2^LOGWMAX are compiled into a kernel, so a plan
// with short windows does not pay the registers of the long ones.
template <int PT, bool DUMP, int LOGWMAX, int L = 0>
__device__ __forceinline__ uint32_t window_key_dispatch(int logw, const float2* col,
                                                        float2* dump, int m_f) {
  if constexpr (L < LOGWMAX) {
    if (logw == L) return window_key_lds<L, PT, DUMP>(col, dump, m_f);
    return window_key_dispatch<PT, DUMP, LOGWMAX, L + 1>(logw, col, dump, m_f);
  } else {
    return window_key_lds<LOGWMAX, PT, DUMP>(col, dump, m_f);
  }
}

template <int PT, bool DUMP, int LOGWMAX>
__global__ void __launch_bounds__(64) rate_peak_kernel(RateArgs a) {
  extern __shared__ float2 hist[];  // [buf_slots][64]
  const int lane = threadIdx.x;
  const int item = blockIdx.x;
  const int kb = item % a.n_kb;
  const int rest = item / a.n_kb;
  const int chunk = rest % a.n_chunks;
  const int b = rest / a.n_chunks;
  const int kf = kb * kBinsPerWave + lane;
  const int T = a.T;
  const int M = a.M;
  const int own_lo = chunk * a.chunk;
  const int own_hi = min(T, own_lo + a.chunk);
  const int load_hi = min(T, own_hi + a.w_max - 1);
  const int keep = a.w_max - 1;
  const float2* __restrict__ xcol = a.X + static_cast<int64_t>(b) * T * M + kf;
  float2* mycol = hist + lane;

  int wp = 0, tbuf0 = own_lo, tb = own_lo;
  int nq = min(kQ, load_hi - tb);
  float2 pre[kQ];
  static_for<0, kQ>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    if (i < nq) pre[i] = xcol[static_cast<int64_t>(tb + i) * M];
  });
  while (tb < load_hi) {
    if (wp + nq > a.buf_slots) {  // keep the last W_max - 1 APs, drop the rest
      const int src = wp - keep;
      for (int i = 0; i < keep; ++i) mycol[i * kBinsPerWave] = mycol[(src + i) * kBinsPerWave];
      tbuf0 += src;
      wp = keep;
    }
    static_for<0, kQ>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      if (i < nq) mycol[(wp + i) * kBinsPerWave] = pre[i];
    });
    const int tn = tb + nq;
    const int nqn = min(kQ, load_hi - tn);
    static_for<0, kQ>([&](auto ii) {  // prefetch the next batch under the compute
      constexpr int i = decltype(ii)::value;
      if (i < nqn) pre[i] = xcol[static_cast<int64_t>(tn + i) * M];
    });
    for (int li = a.l0; li < a.lv.n; ++li) {
      const int W = a.lv.W[li];
      const int s = a.lv.s[li];
      const int lo = max(max(tb, a.t_emit) - W + 1, own_lo);
      const int hi = min(min(tb + nq - W, own_hi - 1), T - W);
      if (lo > hi) continue;
      for (int start = ((lo + s - 1) / s) * s; start <= hi; start += s) {
        const int j = start / s;
        float2* dump = nullptr;
        if constexpr (DUMP)
          dump = a.dump + a.dump_base + static_cast<int64_t>(b) * a.grid_per_bl + a.lvl_goff[li] +
                 static_cast<int64_t>(j - a.lvl_j0[li]) * (PT * W) * M + kf;
        const uint32_t key = window_key_dispatch<PT, DUMP, LOGWMAX>(
            a.lv.logW[li], mycol + (start - tbuf0) * kBinsPerWave, dump, M);
        const uint64_t pk = wave_peak(key, kb * kBinsPerWave, 1);
        if (lane == 0)
          a.part[static_cast<int64_t>(kb) * a.slab_windows + static_cast<int64_t>(b) * a.nwb +
                 a.lvl_off[li] + (j - a.lvl_j0[li])] = pk;
      }
    }
    wp += nq;
    tb = tn;
    nq = nqn;
  }
}

template <int PT, bool DUMP, int LOGWMAX>
hipError_t launch_t(const RateArgs& a, hipStream_t st) {
  const int64_t items = static_cast<int64_t>(a.nb) * a.n_chunks * a.n_kb;
  if (items == 0) return hipSuccess;
  if (items > 0x7FFFFFFF) return hipErrorInvalidValue;
  const size_t lds = static_cast<size_t>(a.buf_slots) * kBinsPerWave * sizeof(float2);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&rate_peak_kernel<PT, DUMP, LOGWMAX>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((rate_peak_kernel<PT, DUMP, LOGWMAX>), dim3(static_cast<unsigned>(items)), dim3(64),
                     lds, st, a);
  return hipGetLastError();
}

}  // namespace

int rate_buffer_slots(int w_max) { return w_max - 1 + 2 * kQ; }

// Plans with windows of at most kFusedMaxWindow APs go to the fused kernel.
template <int PT, bool DUMP>
hipError_t launch_w(const RateArgs& a, hipStream_t st) {
  if (a.w_max <= kFusedMaxWindow) return hipErrorInvalidValue;
  return launch_t<PT, DUMP, 7>(a, st);
}

hipError_t launch_rate_peak(const RateArgs& a, hipStream_t st) {
  const bool dump = a.dump != nullptr;
  if (a.pad_t == 1) return dump ? launch_w<1, true>(a, st) : launch_w<1, false>(a, st);
  if (a.pad_t == 2) return dump ? launch_w<2, true>(a, st) : launch_w<2, false>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace fringe
