// Device helpers shared by the fringe-search kernels: complex arithmetic on
// float2, unit roots evaluated at compile time, and a fully unrolled
// radix-2 decimation-in-frequency FFT on a register array.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fringe {

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Pointers read from descriptor tables are generic; these casts let the
// compiler use global (not flat) memory instructions for them.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}
// float2 is a class type whose copy constructor cannot bind a global-space
// reference, so complex samples go through the native two-float vector.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_global(const float2* p) {
  const f32x2_t v = *(const __attribute__((address_space(1))) f32x2_t*)(p);
  return make_float2(v.x, v.y);
}

// The same load at a byte offset (< 4 GiB) from a wave-uniform base, so the
// address is a scalar base plus a 32-bit vector offset (no 64-bit vector
// address arithmetic per load).
__device__ __forceinline__ float2 ld_global_off(const float2* base, uint32_t byte_off) {
  const auto* b = (const __attribute__((address_space(1))) char*)(base);
  const f32x2_t v = *(const __attribute__((address_space(1))) f32x2_t*)(b + byte_off);
  return make_float2(v.x, v.y);
}

// Raw buffer access to a wave-uniform region: a load is a per-lane 32-bit
// offset plus a scalar offset (both in bytes), with no vector address
// arithmetic.  Word 3 of the resource is the gfx9-family setting for
// untyped 32-bit-element access; the record limit is left at its maximum
// (callers keep offsets inside their data).
constexpr int kBufferWord3 = 0x00020000;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0), -1,
                                           kBufferWord3);
}

__device__ __forceinline__ float2 ld_buffer(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff),
                                                         static_cast<int>(soff), 0);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

// v held in a vector register: values the compiler would keep in scalar
// registers (wave-uniform) cost a slower issue when they are VALU operands.
__device__ __forceinline__ float in_vgpr(float v) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

// A wave-uniform value (held in a scalar register) copied to a vector
// register once, so that the FMAs reading it issue at the full rate, not at
// the half rate of a scalar operand.
__device__ __forceinline__ float uniform_in_vgpr(float v) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float c_norm(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// ------------------------------------------------ compile-time unit roots --
// exp(-2 pi i k / n) for n a power of two, from Taylor series on an octant-
// reduced angle (|phi| <= pi/4, 13 terms: far below double rounding).
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int m = 1; m < 14; ++m) {
    term *= -x2 / double((2 * m) * (2 * m + 1));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int m = 1; m < 14; ++m) {
    term *= -x2 / double((2 * m - 1) * (2 * m));
    sum += term;
  }
  return sum;
}

struct CxD { double re, im; };

constexpr CxD unit_root(long k, long n) {
  k %= n;
  if (k < 0) k += n;
  // theta = 2 pi k / n = (pi / 4) * (oct + rem / n)
  const long k8 = 8 * k;
  const long oct = k8 / n;
  const long rem = k8 - oct * n;
  double c = 0, s = 0;
  long quad = 0;
  if ((oct & 1) == 0) {
    const double phi = (kPi / 4) * double(rem) / double(n);
    c = taylor_cos(phi);
    s = taylor_sin(phi);
    quad = oct / 2;
  } else {  // theta = (oct + 1) pi / 4 - phi'
    const double phi = (kPi / 4) * double(n - rem) / double(n);
    c = taylor_cos(phi);
    s = -taylor_sin(phi);
    quad = (oct + 1) / 2;
  }
  double cr = c, sr = s;  // rotate by quad * 90 degrees
  switch (quad & 3) {
    case 1: cr = -s; sr = c; break;
    case 2: cr = -c; sr = -s; break;
    case 3: cr = s; sr = -c; break;
    default: break;
  }
  // exp(-i theta) = cos - i sin; canonical +0 for exact zeros
  return CxD{cr + 0.0, -sr + 0.0};
}

// d * exp(-2 pi i J / LEN), with the trivial angles done by moves.
template <int LEN, int J>
__device__ __forceinline__ float2 twiddle_mul(float2 d) {
  constexpr int j = ((J % LEN) + LEN) % LEN;
  if constexpr (j == 0) {
    return d;
  } else if constexpr (4 * j == LEN) {       // * (-i)
    return make_float2(d.y, -d.x);
  } else if constexpr (2 * j == LEN) {       // * (-1)
    return make_float2(-d.x, -d.y);
  } else if constexpr (4 * j == 3 * LEN) {   // * (+i)
    return make_float2(-d.y, d.x);
  } else {
    constexpr CxD w = unit_root(j, LEN);
    constexpr float wr = float(w.re), wi = float(w.im);
    return make_float2(fmaf(d.x, wr, -d.y * wi), fmaf(d.x, wi, d.y * wr));
  }
}

// -------------------------------------------------- register radix-2 FFT --
// In-place DIF on v[0..N): afterwards v[i] holds X[bitrev(i)], where
// X[k] = sum_n v_in[n] exp(-2 pi i k n / N).
template <int N, int LEN, int BLK, int J>
__device__ __forceinline__ void dif_butterflies(float2* v) {
  if constexpr (J < LEN / 2) {
    const float2 a = v[BLK + J];
    const float2 b = v[BLK + J + LEN / 2];
    v[BLK + J] = c_add(a, b);
    v[BLK + J + LEN / 2] = twiddle_mul<LEN, J>(c_sub(a, b));
    dif_butterflies<N, LEN, BLK, J + 1>(v);
  }
}

template <int N, int LEN, int BLK>
__device__ __forceinline__ void dif_blocks(float2* v) {
  if constexpr (BLK < N) {
    dif_butterflies<N, LEN, BLK, 0>(v);
    dif_blocks<N, LEN, BLK + LEN>(v);
  }
}

template <int N, int LEN = N>
__device__ __forceinline__ void fft_dif(float2* v) {
  if constexpr (LEN >= 2) {
    dif_blocks<N, LEN, 0>(v);
    fft_dif<N, LEN / 2>(v);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

}  // namespace fringe
