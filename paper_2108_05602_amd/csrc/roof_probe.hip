// Roof probes: an FP32 FMA loop and a plain HBM copy (not part of the
// search; the measurement reads the search against what they achieve).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_common.h"
#include "fringe_probe.h"

namespace fringe {
void set_last_error(const char* msg);
}

namespace {

constexpr int kProbeLanes = 256;
constexpr int kChains = 16;

__global__ __launch_bounds__(kProbeLanes) void fma_probe_kernel(float* __restrict__ out,
                                                                int iters, float a, float b) {
  const int lane = threadIdx.x;
  // operands in VGPRs: the accumulate form x += a * b (v_fmac_f32 with
  // vector sources), the form of the search kernels' FMAs
  const float av = fringe::in_vgpr(a), bv = fringe::in_vgpr(b);
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = 1.0f + 0.001f * float(lane + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(av, bv, x[c]);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[int64_t(blockIdx.x) * kProbeLanes + lane] = s;
}

__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4* __restrict__ src,
                                                         uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace

extern "C" {

int fringe_probe_fma(int64_t n_blocks, int32_t iters, float* d_out, double* flops,
                     void* hip_stream) {
  if (!d_out || !flops || n_blocks < 1 || n_blocks > INT32_MAX || iters < 1) {
    fringe::set_last_error("fringe_probe_fma: null pointer, n_blocks or iters out of range");
    return FRINGE_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // each chain grows by a * b = 1e-6 per step: finite for any iters
  hipLaunchKernelGGL(fma_probe_kernel, dim3(uint32_t(n_blocks)), dim3(kProbeLanes), 0, st,
                     d_out, int(iters), 0.001f, 0.001f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fringe::set_last_error(hipGetErrorString(e));
    return FRINGE_E_HIP;
  }
  *flops = 2.0 * kChains * double(iters) * kProbeLanes * double(n_blocks);
  return FRINGE_OK;
}

int fringe_probe_copy(const void* d_src, void* d_dst, int64_t bytes, void* hip_stream) {
  if (!d_src || !d_dst || bytes < 16 || bytes % 16 != 0 ||
      (reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) % 16 != 0) {
    fringe::set_last_error("fringe_probe_copy: null or misaligned pointer, or bytes not a "
                           "positive multiple of 16");
    return FRINGE_E_INVALID;
  }
  const int64_t n = bytes / 16;
  // 8 workgroups of 256 lanes per CU over 256 CUs; each lane strides the rest
  const int64_t want = (n + 255) / 256;
  const uint32_t blocks = uint32_t(want < 2048 ? want : 2048);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(copy_probe_kernel, dim3(blocks), dim3(256), 0, st,
                     static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fringe::set_last_error(hipGetErrorString(e));
    return FRINGE_E_HIP;
  }
  return FRINGE_OK;
}

}  // extern "C"
