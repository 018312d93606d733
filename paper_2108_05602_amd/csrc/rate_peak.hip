// Rate transform and grid peak: for every window of every length, the
// zero-padded DFT over the window's APs of each delay bin's spectrum,
//   G[k_t, k_f] = sum_{u<W} X_{t0+u}[k_f] exp(-2 pi i k_t u / M_t),
// followed by the peak of |G|^2 with lowest-flat-index tie-break.  The time
// sum is the paper's window combination (section "Code optimization",
// step 6, which keeps only k_t = 0); M_t = pad_t * W.
//
// Layout: lane l owns delay bin k_f = 64 * kb + l of one baseline, so every
// HBM read of X is a coalesced 512-byte row segment.  This kernel serves the
// windows longer than 64 APs (levels l0 and up), and with at most 128 APs
// per window those are the W = 128 windows, stride 64; shorter ones go to the
// fused kernel (fused_search.h), which does its own delay transform and keeps
// the history in registers, also in plans that have long windows.
//
// A work group of kWaves waves walks a chunk of APs (plus a halo of 127 APs
// for the windows that start in the chunk) in batches of kQ APs, each wave
// loading kQ / kWaves of them, into an LDS ring of 128 slots per bin (AP t in
// slot t mod 128).  Windows start at multiples of 64 and the chunk at a
// multiple of kQ, so a window ends on the last AP of a batch: its 128 APs are
// exactly the ring's contents, and the next batch overwrites only APs that
// no later window needs.  The waves share each window's transform: wave w
// computes the sub-transforms r = w, w + kWaves, ...
//   k_t = S p + r,  G[S p + r] = FFT_N( y_r )[p],
//   y_r[v] = w_{M_t}^{r v} sum_{h<H} x[v + N h] w_S^{r h},
// (N = 16, S = M_t / 16, H = 8), each wave's 64-lane DPP max gives its
// partial peak (window_key.h), and one lane stores the maximum of the
// kWaves partials.  Two barriers per window (one before its transform, so
// every wave's APs are in the ring; one after, so none is overwritten while
// read), none for the batches in between.
#include "kernels.h"
#include "window_key.h"

namespace fringe {

namespace {

constexpr int kQ = 32;                // APs per load batch (16 or 32: 13 % faster than 8 or 64)
constexpr int kWaves = 8;             // waves per work group
constexpr int kQW = kQ / kWaves;      // APs each wave loads per batch
constexpr int kRing = kMaxWindowAp;   // ring slots per bin (the window length)
constexpr int kLogRing = 7;
static_assert(kRing == 1 << kLogRing, "ring of one window");
static_assert(kQ % kWaves == 0 && (kRing / 2) % kQ == 0, "batches tile the stride");
// A sample of the ring as an LDS word (volatile accesses keep the generic
// address space unless it is named).
typedef __attribute__((address_space(3))) volatile uint64_t LdsU64;

template <int PT, bool DUMP>
// Two work groups per CU (the ring takes 64 KB of LDS): four waves per SIMD,
// registers capped to fit; the grid-dump variant (tests) keeps two, so as not
// to spill.
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(DUMP ? 2 : 4)))
rate_peak_kernel(RateArgs a) {
  extern __shared__ float2 ring[];  // [kRing][64], then kWaves uint64 partials
  uint64_t* wave_pk = reinterpret_cast<uint64_t*>(ring + kRing * kBinsPerWave);
  const int lane = threadIdx.x & (kBinsPerWave - 1);
  // the wave index, uniform in the wave (a scalar): the sub-transforms it
  // selects then read their twiddles with scalar loads
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kBinsPerWave);
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
  const int load_hi = min(T, own_hi + kRing - 1);
  const float2* __restrict__ xcol = a.X + static_cast<int64_t>(b) * T * M + kf;
  float2* mycol = ring + lane;

  int tb = own_lo;
  int nq = min(kQ, load_hi - tb);
  float2 pre[kQW];
  static_for<0, kQW>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int q = wv * kQW + i;
    if (q < nq) pre[i] = xcol[static_cast<int64_t>(tb + q) * M];
  });
  while (tb < load_hi) {
    static_for<0, kQW>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int q = wv * kQW + i;
      if (q < nq) mycol[((tb + q) & (kRing - 1)) * kBinsPerWave] = pre[i];
    });
    const int tn = tb + nq;
    const int nqn = min(kQ, load_hi - tn);
    static_for<0, kQW>([&](auto ii) {  // prefetch the next batch under the compute
      constexpr int i = decltype(ii)::value;
      const int q = wv * kQW + i;
      if (q < nqn) pre[i] = xcol[static_cast<int64_t>(tn + q) * M];
    });
    for (int li = a.l0; li < a.lv.n; ++li) {
      const int W = a.lv.W[li];  // = kRing (checked at launch)
      const int s = a.lv.s[li];
      const int lo = max(max(tb, a.t_emit) - W + 1, own_lo);
      const int hi = min(min(tb + nq - W, own_hi - 1), T - W);
      if (lo > hi) continue;
      for (int start = ((lo + s - 1) / s) * s; start <= hi; start += s) {
        __syncthreads();  // the window's APs, loaded by every wave, are in the ring
        const int j = start / s;
        float2* dump = nullptr;
        if constexpr (DUMP)
          dump = a.dump + a.dump_base + static_cast<int64_t>(b) * a.grid_per_bl + a.lvl_goff[li] +
                 static_cast<int64_t>(j - a.lvl_j0[li]) * (PT * kRing) * M + kf;
        // AP start + u sits in slot (start + u) mod kRing, start mod kRing
        // being 0 or kRing / 2.  The reads are volatile: every sub-transform
        // reads the window again from the ring rather than the compiler
        // hoisting all 128 samples into registers.
        const int off = (start & (kRing - 1)) * kBinsPerWave;
        const LdsU64* vcol = (const LdsU64*)(mycol);
        auto sample = [&](auto ui) {
          constexpr int u = decltype(ui)::value;
          const uint64_t v = u < kRing / 2 ? vcol[u * kBinsPerWave + off]
                                           : vcol[u * kBinsPerWave - off];
          return make_float2(__uint_as_float(static_cast<uint32_t>(v)),
                             __uint_as_float(static_cast<uint32_t>(v >> 32)));
        };
        // S = 2 kWaves sub-transforms (pad_time 2): wave wv takes the pair
        // r = wv, wv + kWaves in one pass; else one or none each
        uint32_t key;
        if constexpr (RateShape<kLogRing, PT>::S == 2 * kWaves)
          key = window_key_pair<kLogRing, PT, DUMP, true>(sample, dump, M, wv);
        else
          key = window_key<kLogRing, PT, DUMP, true>(sample, dump, M, wv, kWaves);
        const uint64_t pk = wave_peak(key, kb * kBinsPerWave, 1);
        if (lane == 0) wave_pk[wv] = pk;
        __syncthreads();  // every wave's partial is in, and the ring may be refilled
        if (threadIdx.x == 0) {
          uint64_t m = wave_pk[0];
          static_for<1, kWaves>([&](auto wi) {
            const uint64_t o = wave_pk[decltype(wi)::value];
            m = o > m ? o : m;
          });
          a.part[static_cast<int64_t>(kb) * a.slab_windows + static_cast<int64_t>(b) * a.nwb +
                 a.lvl_off[li] + (j - a.lvl_j0[li])] = m;
        }
      }
    }
    tb = tn;
    nq = nqn;
  }
}

template <int PT, bool DUMP>
hipError_t launch_t(const RateArgs& a, hipStream_t st) {
  const int64_t items = static_cast<int64_t>(a.nb) * a.n_chunks * a.n_kb;
  if (items == 0) return hipSuccess;
  if (items > 0x7FFFFFFF) return hipErrorInvalidValue;
  const size_t lds = static_cast<size_t>(kRing) * kBinsPerWave * sizeof(float2) +
                     kWaves * sizeof(uint64_t);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&rate_peak_kernel<PT, DUMP>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((rate_peak_kernel<PT, DUMP>), dim3(static_cast<unsigned>(items)),
                     dim3(64 * kWaves), lds, st, a);
  return hipGetLastError();
}

}  // namespace

int rate_buffer_slots(int /*w_max*/) { return kRing; }

// The kernel's ring and batches assume what the plan guarantees: every
// level it searches is W = 128 with stride 64, chunks start at multiples
// of 64 APs, and the bins split into whole 64-bin blocks.
template <int PT, bool DUMP>
hipError_t launch_w(const RateArgs& a, hipStream_t st) {
  if (a.w_max != kRing || a.chunk % (kRing / 2) != 0 || a.M != a.n_kb * kBinsPerWave ||
      a.l0 < 0 || a.l0 >= a.lv.n)
    return hipErrorInvalidValue;
  for (int li = a.l0; li < a.lv.n; ++li)
    if (a.lv.W[li] != kRing || a.lv.s[li] != kRing / 2) return hipErrorInvalidValue;
  return launch_t<PT, DUMP>(a, st);
}

hipError_t launch_rate_peak(const RateArgs& a, hipStream_t st) {
  const bool dump = a.dump != nullptr;
  if (a.pad_t == 1) return dump ? launch_w<1, true>(a, st) : launch_w<1, false>(a, st);
  if (a.pad_t == 2) return dump ? launch_w<2, true>(a, st) : launch_w<2, false>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace fringe
