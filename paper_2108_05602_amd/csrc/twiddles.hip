// Unit roots exp(-2 pi i k / M) for every delay-transform size the library
// serves (M = 64 ... 4096), evaluated at compile time (dev_common.h's
// octant-reduced Taylor series in double, rounded to float) and resident in
// device memory as part of the code object: plans and the allocation-free
// search read them in place, with no upload.
#include "dev_common.h"
#include "kernels.h"

namespace fringe {


constexpr int kTwLogMin = 6, kTwLogMax = 12;
constexpr int kTwTotal = (1 << (kTwLogMax + 1)) - (1 << kTwLogMin);

struct TwAll {
  float2 v[kTwTotal];
  constexpr TwAll() : v() {
    for (int lm = kTwLogMin; lm <= kTwLogMax; ++lm) {
      const int m = 1 << lm;
      for (int k = 0; k < m; ++k) {
        const CxD w = unit_root(k, m);
        v[m - (1 << kTwLogMin) + k] = float2{float(w.re), float(w.im)};
      }
    }
  }
};

namespace {

constexpr int kMaxDevices = 64;
const float2* g_tw_base[kMaxDevices] = {};

}  // namespace

// External linkage: a device variable that no kernel of this file reads is
// kept in the code object (where the runtime finds it by name) only if it is
// externally visible (so not const: a const variable at namespace scope
// has internal linkage).
__device__ TwAll kTwAll{};

// Device address of the table for M points on the current device (the
// symbol's address, looked up once per device).
hipError_t twiddles_for(int m, const float2** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices || m < (1 << kTwLogMin) || m > (1 << kTwLogMax) ||
      (m & (m - 1)) != 0)
    return hipErrorInvalidValue;
  if (!g_tw_base[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(kTwAll));
    if (e != hipSuccess) return e;
    g_tw_base[dev] = static_cast<const float2*>(p);
  }
  *out = g_tw_base[dev] + (m - (1 << kTwLogMin));
  return hipSuccess;
}

}  // namespace fringe
