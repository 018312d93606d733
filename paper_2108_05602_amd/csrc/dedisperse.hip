// Dedispersion as a pass of its own (paper, section "Code optimization",
// step 4): out[b][t][f] = in[b][t + d_f][f], 0 where t + d_f runs past the
// scan, d_f clamped to [0, n_ap] as in the search kernels.  A plan then
// searches the dedispersed cube without shifts.  Each AP row of the output
// is written whole (coalesced); its reads come from rows t .. t + max d_f,
// contiguous within each run of equal shifts, and each input line is
// fetched once per output row it feeds, where the in-kernel shifts make
// every one of a (baseline, chunk)'s delay-bin classes fetch it again.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_common.h"
#include "fringe.h"

namespace fringe {
void set_last_error(const char* msg);
}

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void dedisperse_kernel(const float2* __restrict__ in,
                                                              float2* __restrict__ out,
                                                              int64_t n_rows, int T, int F,
                                                              const int32_t* __restrict__ shifts) {
  // one thread per (row, channel) with the channel fastest; rows = b * T + t
  const int64_t total = n_rows * F;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += stride) {
    const int64_t row = e / F;
    const int f = static_cast<int>(e - row * F);
    const int t = static_cast<int>(row % T);
    const int d = min(max(shifts[f], 0), T);
    float2 v = make_float2(0.f, 0.f);
    if (t + d < T) v = in[e + static_cast<int64_t>(d) * F];
    out[e] = v;
  }
}

}  // namespace

extern "C" int fringe_dedisperse(const fringe_cf32* d_in, fringe_cf32* d_out, int32_t n_baselines,
                                 int32_t n_ap, int32_t n_freq, const int32_t* d_shifts,
                                 void* hip_stream) {
  if (!d_in || !d_out || !d_shifts || n_baselines < 1 || n_ap < 1 || n_freq < 1) {
    fringe::set_last_error("fringe_dedisperse: null pointer or a size below 1");
    return FRINGE_E_INVALID;
  }
  const int64_t bytes = int64_t(n_baselines) * n_ap * n_freq * int64_t(sizeof(fringe_cf32));
  const char* a = reinterpret_cast<const char*>(d_in);
  const char* b = reinterpret_cast<const char*>(d_out);
  if (a < b + bytes && b < a + bytes) {
    fringe::set_last_error("fringe_dedisperse: input and output overlap");
    return FRINGE_E_INVALID;
  }
  const int64_t n_rows = int64_t(n_baselines) * n_ap;
  const int64_t total = n_rows * n_freq;
  const int64_t want = (total + kThreads - 1) / kThreads;
  const uint32_t blocks = uint32_t(want < 16384 ? want : 16384);
  hipLaunchKernelGGL(dedisperse_kernel, dim3(blocks), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream),
                     reinterpret_cast<const float2*>(d_in), reinterpret_cast<float2*>(d_out),
                     n_rows, int(n_ap), int(n_freq), d_shifts);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fringe::set_last_error(hipGetErrorString(e));
    return FRINGE_E_HIP;
  }
  return FRINGE_OK;
}
