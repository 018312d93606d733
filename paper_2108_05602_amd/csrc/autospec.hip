// Auto-spectrum amplitude normalisation (paper, section "Fringe fitting":
// each frequency point's amplitude divided by the auto-spectrum dispersions
// of the two stations, as in the Mk4 format of HOPS):
//
//   g[b][f] = g_in[b][f] * (abar_i^2[f] * abar_j^2[f])^(-1/4),
//   abar_i^2[f] = (1 / n_spectra) sum_k a_i[k][f]^2,
//
// for baseline b = (i, j), written as per-baseline, per-channel gains that
// fringe_set_gains folds into the search at no cost.  A product of zero (a
// station with no power in the channel) gives a zero gain: the channel is
// flagged on that baseline.
#include "dev_common.h"
#include "kernels.h"
#include "../../include/fringe_calib.h"

namespace fringe {
void set_last_error(const char* msg);
}

using namespace fringe;

namespace {

// One thread per (baseline, channel); the dispersions are accumulated in
// double over the spectra (reads of consecutive channels coalesce).
__global__ void __launch_bounds__(256)
autospec_gain_kernel(const float* __restrict__ autos, int n_st, int n_spec, int n_freq,
                     const int32_t* __restrict__ pairs, int n_bl,
                     const float2* __restrict__ g_in, float2* __restrict__ g_out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(n_bl) * n_freq) return;
  const int b = static_cast<int>(idx / n_freq);
  const int f = static_cast<int>(idx - static_cast<int64_t>(b) * n_freq);
  const int i = pairs[2 * b], j = pairs[2 * b + 1];
  double scale = 0.0;
  if (i >= 0 && i < n_st && j >= 0 && j < n_st) {
    double si = 0.0, sj = 0.0;
    const float* ai = autos + static_cast<int64_t>(i) * n_spec * n_freq + f;
    const float* aj = autos + static_cast<int64_t>(j) * n_spec * n_freq + f;
    for (int k = 0; k < n_spec; ++k) {
      const double x = ai[static_cast<int64_t>(k) * n_freq];
      const double y = aj[static_cast<int64_t>(k) * n_freq];
      si = fma(x, x, si);
      sj = fma(y, y, sj);
    }
    const double prod = (si / n_spec) * (sj / n_spec);
    if (prod > 0.0) scale = 1.0 / sqrt(sqrt(prod));
  }
  const float2 g = g_in ? g_in[idx] : make_float2(1.f, 0.f);
  g_out[idx] = make_float2(static_cast<float>(g.x * scale), static_cast<float>(g.y * scale));
}

int fail_msg(int code, const char* msg) {
  set_last_error(msg);
  return code;
}

}  // namespace

extern "C" int fringe_autospectrum_gains(const float* d_auto, int32_t n_stations,
                                         int32_t n_spectra, int32_t n_freq,
                                         const int32_t* d_pairs, int32_t n_baselines,
                                         const fringe_cf32* d_gains_in, fringe_cf32* d_gains_out,
                                         void* hip_stream) {
  if (!d_auto || !d_pairs || !d_gains_out)
    return fail_msg(FRINGE_E_INVALID, "fringe_autospectrum_gains: null pointer");
  if (n_stations < 1 || n_spectra < 1 || n_freq < 1 || n_baselines < 1)
    return fail_msg(FRINGE_E_INVALID, "fringe_autospectrum_gains: sizes must be >= 1");
  const int64_t n = int64_t(n_baselines) * n_freq;
  if (d_gains_in && static_cast<const void*>(d_gains_in) != static_cast<const void*>(d_gains_out)) {
    const char* a = reinterpret_cast<const char*>(d_gains_in);
    const char* o = reinterpret_cast<const char*>(d_gains_out);
    const int64_t bytes = n * int64_t(sizeof(fringe_cf32));
    if (a < o + bytes && o < a + bytes)
      return fail_msg(FRINGE_E_INVALID, "fringe_autospectrum_gains: gains_in and gains_out "
                                        "overlap without being the same array");
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF)
    return fail_msg(FRINGE_E_UNSUPPORTED, "fringe_autospectrum_gains: too many gains");
  hipLaunchKernelGGL(autospec_gain_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     d_auto, n_stations, n_spectra, n_freq, d_pairs, n_baselines,
                     reinterpret_cast<const float2*>(d_gains_in),
                     reinterpret_cast<float2*>(d_gains_out));
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail_msg(FRINGE_E_HIP, hipGetErrorString(he));
  return FRINGE_OK;
}
