// Delay transform: for every AP of every baseline, the zero-padded DFT
// over the concatenated IF x channel axis (paper, section "Code
// optimization", step 5; padding factor of section "Fringe fitting"):
//   X_t[k] = sum_{f<F} x_t[f] exp(-2 pi i k f / M),  M = pad_f * F,
// plus the AP energy e_t = sum_f |x_t[f]|^2 that the window SNR divides by
// (x multiplied first by the slab's calibration gains when it has them).
//
// Up to M = 1024 one wavefront per work group transforms NAP = 1024 / M
// APs at a time; above, M / 1024 waves share one AP (one radix-16
// butterfly per thread and pass, the group's LDS one transform), so the
// 2048- and 4096-point transforms keep three waves per SIMD instead of one
// wave holding 64 points per lane.  Self-sorting (Stockham) FFT: radix-16
// passes, then one radix-2/4/8 pass if log2(M) is not a multiple of 4.  The first pass
// reads the visibilities straight from HBM (coalesced, the zero half /
// three quarters of the padded input never loaded or multiplied), middle
// passes go through LDS, and the last pass writes X to HBM in natural order.
#include "dev_common.h"
#include "kernels.h"

namespace fringe {

namespace {

// DIF FFT of N points whose inputs beyond the first NZ are zero: stages
// whose upper half is all zero only copy and twiddle the lower half.
template <int N, int NZ, int LEN, int BLK, int J>
__device__ __forceinline__ void pruned_stage_bf(float2* v) {
  if constexpr (J < NZ) {
    v[BLK + J + LEN / 2] = twiddle_mul<LEN, J>(v[BLK + J]);
    pruned_stage_bf<N, NZ, LEN, BLK, J + 1>(v);
  }
}

template <int N, int NZ, int LEN, int BLK>
__device__ __forceinline__ void pruned_stage(float2* v) {
  if constexpr (BLK < N) {
    pruned_stage_bf<N, NZ, LEN, BLK, 0>(v);
    pruned_stage<N, NZ, LEN, BLK + LEN>(v);
  }
}

template <int N, int NZ, int LEN = N>
__device__ __forceinline__ void fft_dif_pruned(float2* v) {
  if constexpr (LEN >= 2) {
    if constexpr (LEN / 2 >= NZ) {
      pruned_stage<N, NZ, LEN, 0>(v);
      fft_dif_pruned<N, NZ, LEN / 2>(v);
    } else {
      fft_dif<N, LEN>(v);
    }
  }
}

constexpr int first_radix(int log_m) { return log_m >= 4 ? 16 : (1 << log_m); }

// One Stockham pass over NAP transforms of M points held in `lds`
// (or, for the first pass, read from `xin`; for the last, written to `xout`).
// Pass p has radix R and NS = product of the earlier radices:
//   v[r] = in[j + r M/R] * w_{NS R}^{(j mod NS) r},  V = DFT_R(v),
//   out[(j / NS) NS R + (j mod NS) + k NS] = V[k].
// LDS slot of element i of the group's transforms: one float2 of padding
// after every 16, so that a pass's strided writes (16 or 256 elements apart
// across threads) spread over the banks instead of landing on two of them.
__device__ __forceinline__ int lds_slot(int i) { return i + (i >> 4); }
constexpr int lds_slots(int n) { return n + n / 16; }

// The first pass's inputs: the NZ nonzero samples of each of the thread's
// butterflies (the rest of the padded input is zero), calibrated.
template <int M, int NAP, int R, int PF, int NT>
struct FirstInputs {
  static constexpr int BPL = NAP * M / R / NT;
  static constexpr int NZ = R / PF > 0 ? R / PF : 1;
  float2 x[BPL][NZ];
};

template <int M, int NAP, int R, int PF, int NT>
__device__ __forceinline__ void load_first(FirstInputs<M, NAP, R, PF, NT>& in,
                                           const float2* __restrict__ xin, int lane,
                                           int n_valid_ap, int F,
                                           const float2* __restrict__ gains,
                                           const int32_t* __restrict__ shifts,
                                           const float2* __restrict__ xbl, int t_first, int T,
                                           const float2* __restrict__ xbl2, int halo) {
  using In = FirstInputs<M, NAP, R, PF, NT>;
  constexpr int SPAN = M / R;
#pragma unroll
  for (int i = 0; i < In::BPL; ++i) {
    const int jj = lane + NT * i;
    const int a = jj / SPAN;
    const int j = jj % SPAN;
    const bool ok = a < n_valid_ap;
#pragma unroll
    for (int r = 0; r < In::NZ; ++r) {
      const int idx = j + r * SPAN;
      float2 x = make_float2(0.f, 0.f);
      if (ok && idx < F) {
        if (shifts) {  // dedispersion: channel idx from AP t + d, 0 past the data
          const int row = t_first + a + min(max(shifts[idx], 0), T);
          if (row < T) x = xbl[static_cast<int64_t>(row) * F + idx];  // T: the rows held
        } else if (xbl2) {  // a streamed chunk read in place: rows from halo on in xbl2
          const int row = t_first + a;
          const float2* src = row < halo ? xbl + static_cast<int64_t>(row) * F
                                         : xbl2 + static_cast<int64_t>(row - halo) * F;
          x = src[idx];
        } else {
          x = xin[static_cast<int64_t>(a) * F + idx];
        }
        if (gains) x = c_mul(x, gains[idx]);  // calibration
      }
      in.x[i][r] = x;
    }
  }
}

// NT threads (one to four waves) share the NAP transforms of a work group.
// The first pass takes its inputs from `pre` (loaded ahead by load_first).
template <int M, int NAP, int R, int NS, int PF, bool FIRST, bool LAST, int NT>
__device__ __forceinline__ void stockham_pass(float2* lds, float2* __restrict__ xout,
                                              const float2* __restrict__ tw, int lane,
                                              int n_valid_ap, float* esum,
                                              const FirstInputs<M, NAP, R, PF, NT>* pre) {
  constexpr int NBF = NAP * M / R;   // butterflies in this pass
  constexpr int BPL = NBF / NT;      // per thread
  static_assert(BPL >= 1 && NBF % NT == 0, "pass does not fill the work group");
  constexpr int SPAN = M / R;        // butterflies per transform
  constexpr int NZ = FIRST ? (R / PF > 0 ? R / PF : 1) : R;
  float2 v[BPL][R];
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int jj = lane + NT * i;
    const int a = jj / SPAN;
    const int j = jj % SPAN;
    if constexpr (FIRST) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r < NZ) {
          v[i][r] = pre->x[i][r];
          *esum += c_norm(v[i][r]);
        } else {
          v[i][r] = make_float2(0.f, 0.f);
        }
      }
    } else {
      const int jm = j % NS;
      // SPAN is a multiple of 16, so the padding of element base + r SPAN
      // is the base's plus r SPAN / 16: one slot computation per butterfly
      static_assert(SPAN % 16 == 0, "LDS padding assumes 16-element spans");
      const int sb = lds_slot(a * M + j);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = lds[sb + r * (SPAN + SPAN / 16)];
        if (r > 0) x = c_mul(x, tw[(jm * r) * (M / (NS * R))]);
        v[i][r] = x;
      }
    }
  }
  if constexpr (!FIRST) __syncthreads();  // every read of the pass before any write
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int jj = lane + NT * i;
    const int a = jj / SPAN;
    const int j = jj % SPAN;
    fft_dif_pruned<R, NZ>(v[i]);
    const int idxd = (j / NS) * NS * R + (j % NS);
    // element base + k NS: with NS = 1 the base is a multiple of 16 (R = 16)
    // and k < 16; with NS a multiple of 16 the padding grows by NS / 16 per k
    static_assert(LAST || (NS == 1 && R == 16) || NS % 16 == 0, "LDS padding");
    const int sb = lds_slot(a * M + idxd);
    constexpr int KSTEP = NS == 1 ? 1 : NS + NS / 16;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const float2 y = v[i][bitrev(k, ilog2(R))];
      if constexpr (LAST) {
        // streamed out (non-temporal): the spectra are read back by another
        // kernel long after this one's caches have turned over
        typedef float F2 __attribute__((ext_vector_type(2)));
        if (a < n_valid_ap)
          __builtin_nontemporal_store(
              F2{y.x, y.y}, reinterpret_cast<F2*>(xout + static_cast<int64_t>(a) * M + idxd + k * NS));
      } else {
        lds[sb + k * KSTEP] = y;
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
}

// Passes after the first: radix 16 while at least 4 bits remain, then the rest.
template <int M, int NAP, int PF, int NS, int NT>
__device__ __forceinline__ void later_passes(float2* lds, float2* xout, const float2* tw,
                                             int lane, int n_valid_ap, int F) {
  if constexpr (NS < M) {
    constexpr int rem = ilog2(M / NS);
    constexpr int R = rem >= 4 ? 16 : (1 << rem);
    constexpr bool LAST = (NS * R == M);
    stockham_pass<M, NAP, R, NS, PF, false, LAST, NT>(lds, xout, tw, lane, n_valid_ap, nullptr,
                                                      nullptr);
    later_passes<M, NAP, PF, NS * R, NT>(lds, xout, tw, lane, n_valid_ap, F);
  }
}

// Threads of the work group: one wave up to M = 1024 (1024 / M transforms
// at a time), M / 1024 waves on one transform above, so that each thread
// holds one radix-16 butterfly per pass and the group's LDS is one transform.
constexpr int fft_threads(int log_m) { return log_m > 10 ? (1 << (log_m - 10)) * 64 : 64; }

template <int LOGM, int PF>
__global__ void __launch_bounds__(fft_threads(LOGM)) delay_fft_kernel(DelayArgs a) {
  constexpr int M = 1 << LOGM;
  constexpr int NAP = M >= 1024 ? 1 : 1024 / M;
  constexpr int NT = fft_threads(LOGM);
  constexpr int NW = NT / 64;
  constexpr int R0 = first_radix(LOGM);
  constexpr int GROUP = (M / R0) < 64 ? (M / R0) : 64;  // lanes per AP in the first pass
  extern __shared__ float2 lds[];
  float* lds_e = reinterpret_cast<float*>(lds + lds_slots(NAP * M));  // per-wave energy partials
  const int lane = threadIdx.x;
  const int groups_per_bl = (a.T + NAP - 1) / NAP;
  const int64_t n_groups = static_cast<int64_t>(a.nb) * groups_per_bl;
  const int F = a.F;
  constexpr bool ONE_PASS = (R0 == M);
  // the first pass's inputs of group g, loaded one group ahead so that the
  // loads are in flight while the group before is transformed
  using In = FirstInputs<M, NAP, R0, PF, NT>;
  auto load_group = [&](int64_t g, In& in) {
    const int b = static_cast<int>(g / groups_per_bl);
    const int t0 = static_cast<int>(g % groups_per_bl) * NAP;
    const int n_valid = min(NAP, a.T - t0);
    const float2* xin = a.vis + static_cast<int64_t>(b) * a.vis_stride + static_cast<int64_t>(t0) * F;
    const float2* gains = a.gains ? a.gains + static_cast<int64_t>(b) * F : nullptr;
    const float2* xbl = a.vis + static_cast<int64_t>(b) * a.vis_stride;
    const float2* xbl2 = a.vis2 ? a.vis2 + static_cast<int64_t>(b) * a.vis2_stride : nullptr;
    load_first<M, NAP, R0, PF, NT>(in, xin, lane, n_valid, F, gains, a.shifts, xbl, t0,
                                   a.T_rows, xbl2, a.halo);
  };
  In nxt;
  if (static_cast<int64_t>(blockIdx.x) < n_groups) load_group(blockIdx.x, nxt);
  for (int64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
    const In cur = nxt;
    if (g + gridDim.x < n_groups) load_group(g + gridDim.x, nxt);
    const int b = static_cast<int>(g / groups_per_bl);
    const int t0 = static_cast<int>(g % groups_per_bl) * NAP;
    const int n_valid = min(NAP, a.T - t0);
    const int64_t ap0 = static_cast<int64_t>(b) * a.T + t0;
    float2* xout = a.X + ap0 * M;
    float es = 0.f;
    stockham_pass<M, NAP, R0, 1, PF, true, ONE_PASS, NT>(lds, xout, a.tw, lane, n_valid, &es,
                                                         &cur);
    // AP energies: lanes of one AP form an aligned group of GROUP lanes
    // (with several waves on one AP, each wave's sum goes through LDS; the
    // first pass's closing barrier orders the previous AP's reads of it)
#pragma unroll
    for (int off = GROUP / 2; off >= 1; off >>= 1) es += __shfl_xor(es, off, 64);
    if constexpr (NW > 1) {
      if ((lane & 63) == 0) lds_e[lane >> 6] = es;
      __syncthreads();
      if (lane == 0) {
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += lds_e[w];
        a.e[ap0] = t;
      }
    } else if constexpr (NAP == 1) {
      if (lane == 0) a.e[ap0] = es;
    } else {
      const int ap = lane / GROUP;
      if ((lane % GROUP) == 0 && ap < n_valid) a.e[ap0 + ap] = es;
    }
    if constexpr (!ONE_PASS) later_passes<M, NAP, PF, R0, NT>(lds, xout, a.tw, lane, n_valid, F);
  }
}

template <int LOGM, int PF>
hipError_t launch_one(const DelayArgs& a, hipStream_t st) {
  constexpr int M = 1 << LOGM;
  constexpr int NAP = M >= 1024 ? 1 : 1024 / M;
  const int64_t groups = static_cast<int64_t>(a.nb) * ((a.T + NAP - 1) / NAP);
  if (groups == 0) return hipSuccess;
  const int grid = static_cast<int>(groups < 65536 ? groups : 65536);
  const size_t lds = static_cast<size_t>(lds_slots(NAP * M)) * sizeof(float2) + 16 * sizeof(float);
  hipLaunchKernelGGL((delay_fft_kernel<LOGM, PF>), dim3(grid), dim3(fft_threads(LOGM)), lds, st,
                     a);
  return hipGetLastError();
}

template <int PF>
hipError_t launch_pf(const DelayArgs& a, hipStream_t st) {
  switch (a.log_m) {
    case 6: return launch_one<6, PF>(a, st);
    case 7: return launch_one<7, PF>(a, st);
    case 8: return launch_one<8, PF>(a, st);
    case 9: return launch_one<9, PF>(a, st);
    case 10: return launch_one<10, PF>(a, st);
    case 11: return launch_one<11, PF>(a, st);
    case 12: return launch_one<12, PF>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_delay_fft(const DelayArgs& a, hipStream_t st) {
  switch (a.pad_f) {
    case 1: return launch_pf<1>(a, st);
    case 2: return launch_pf<2>(a, st);
    case 4: return launch_pf<4>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fringe
