// Per-window rate transform and peak key, shared by the search kernels.
//
// For one lane's delay bin and one window of W APs x[0..W) it forms every
// rate bin of the M_t = PT * W point zero-padded DFT,
//   G[k_t] = sum_{u<W} x[u] exp(-2 pi i k_t u / M_t),
// as S interleaved sub-transforms of N = M_t / S <= 16 points,
//   G[S p + r] = FFT_N(y_r)[p],   y_r[v] = w_{M_t}^{r v} sum_{h<H} x[v + N h] w_S^{r h},
// (H = W / N), and reduces |G[k_t]|^2 over k_t to one 32-bit key
//   key = (bits(|G|^2) with the low log2(M_t) bits cleared) | (M_t - 1 - k_t).
// Keys order like (power, then lower rate bin): powers within 2^-(23 -
// log2 M_t) of each other (< 2e-5 relative) count as ties, which go to the
// lower bin, and the power the key carries is exact to that relative size.
// A window-wide peak over the 64 delay bins of a wave is then one unsigned
// max plus the lowest lane holding it (lanes are in ascending k_f order).
#pragma once

#include "dev_common.h"

namespace fringe {

template <int LOGW, int PT>
struct RateShape {
  static constexpr int W = 1 << LOGW;
  static constexpr int MT = PT * W;
  static constexpr int NMAX = 16;
  static constexpr int S = (MT / NMAX > PT) ? MT / NMAX : PT;
  static constexpr int N = MT / S > 0 ? MT / S : 1;
  static constexpr int H = W / N > 0 ? W / N : 1;
  static constexpr uint32_t MASK = static_cast<uint32_t>(MT - 1);
};

__device__ __forceinline__ uint32_t rate_key(float p, uint32_t mask, uint32_t kt) {
  return (__float_as_uint(p) & ~mask) | (mask - kt);
}

// exp(-2 pi i k / 256), k < 256, for the sub-transform loop of long windows
// (every M_t <= 256 and S <= 16 divides 256).
constexpr int kTwN = 256;
struct TwTable {
  float2 v[kTwN];
  constexpr TwTable() : v() {
    for (int k = 0; k < kTwN; ++k) {
      const CxD w = unit_root(k, kTwN);
      v[k] = float2{float(w.re), float(w.im)};
    }
  }
};
static __constant__ TwTable kTw256{};

// X(u) returns the window's u-th sample (compile-time u).  DUMP writes each
// G[k_t] to dump[k_t * dump_stride].  For long windows (S > 4) the key may
// cover only the sub-transforms r = r0, r0 + r_step, ... (the rate bins
// k_t = r mod S), so that several waves can share one window.  VTW: move
// those windows' twiddles (read into scalar registers) to vector registers
// before use: the 128-AP ring kernel measured faster so, the 64-AP windows
// of the fused kernel slower (the moves cost more than the scalar operands).
template <int LOGW, int PT, bool DUMP, bool VTW, typename XF>
__device__ __forceinline__ uint32_t window_key_pair(XF&& X, float2* __restrict__ dump,
                                                    int dump_stride, int r);

template <int LOGW, int PT, bool DUMP, bool VTW = false, bool PAIR = false, typename XF>
__device__ __forceinline__ uint32_t window_key(XF&& X, float2* __restrict__ dump,
                                               int dump_stride, int r0 = 0, int r_step = 1) {
  using Sh = RateShape<LOGW, PT>;
  constexpr int MT = Sh::MT, S = Sh::S, N = Sh::N, H = Sh::H;
  constexpr uint32_t MASK = Sh::MASK;
  if constexpr (Sh::W == 1) {
    // one AP: every rate bin equals x[0]; the lowest bin wins the tie
    const float2 x0 = X(std::integral_constant<int, 0>{});
    if constexpr (DUMP) {
      static_for<0, MT>([&](auto ki) {
        dump[static_cast<int64_t>(decltype(ki)::value) * dump_stride] = x0;
      });
    }
    return rate_key(c_norm(x0), MASK, 0);
  } else if constexpr (S > 4 && PAIR) {
    // long windows, their sub-transforms by pairs (r, r + S/2)
    uint32_t key = 0;
    for (int r = r0; r < S / 2; r += r_step) {
      const uint32_t k = window_key_pair<LOGW, PT, DUMP, VTW>(X, dump, dump_stride, r);
      key = k > key ? k : key;
    }
    return key;
  } else if constexpr (S > 4) {
    // long windows: the sub-transform index r runs at run time, its
    // twiddles w_S^{r h} and w_{M_t}^{r v} come from the uniform table
    uint32_t key = 0;
    for (int r = r0; r < S; r += r_step) {
      float2 y[N];
      if constexpr (VTW) {
        auto tw = [](int k) {
          const float2 w = kTw256.v[k & (kTwN - 1)];
          return make_float2(uniform_in_vgpr(w.x), uniform_in_vgpr(w.y));
        };
        float2 wh[H];
        static_for<1, H>([&](auto hi) {
          constexpr int h = decltype(hi)::value;
          wh[h] = tw((r * h) * (kTwN / S));
        });
        static_for<0, N>([&](auto vi) {
          constexpr int v = decltype(vi)::value;
          float2 acc = X(std::integral_constant<int, v>{});
          static_for<1, H>([&](auto hi) {
            constexpr int h = decltype(hi)::value;
            acc = c_add(acc, c_mul(X(std::integral_constant<int, v + N * h>{}), wh[h]));
          });
          if constexpr (v == 0) y[v] = acc;
          else y[v] = c_mul(acc, tw((r * v) * (kTwN / MT)));
        });
      } else {
        static_for<0, N>([&](auto vi) {
          constexpr int v = decltype(vi)::value;
          float2 acc = X(std::integral_constant<int, v>{});
          static_for<1, H>([&](auto hi) {
            constexpr int h = decltype(hi)::value;
            const float2 w = kTw256.v[((r * h) * (kTwN / S)) & (kTwN - 1)];
            acc = c_add(acc, c_mul(X(std::integral_constant<int, v + N * h>{}), w));
          });
          if constexpr (v == 0) y[v] = acc;
          else y[v] = c_mul(acc, kTw256.v[((r * v) * (kTwN / MT)) & (kTwN - 1)]);
        });
      }
      fft_dif<N>(y);
      static_for<0, N>([&](auto pi) {
        constexpr int p = decltype(pi)::value;
        const uint32_t kt = static_cast<uint32_t>(S * p + r);
        const float2 val = y[bitrev(p, ilog2(N))];
        const uint32_t k = rate_key(c_norm(val), MASK, kt);
        key = k > key ? k : key;
        if constexpr (DUMP) dump[static_cast<int64_t>(kt) * dump_stride] = val;
      });
    }
    return key;
  } else {
    uint32_t key = 0;
    static_for<0, S>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      float2 y[N];
      static_for<0, N>([&](auto vi) {
        constexpr int v = decltype(vi)::value;
        float2 acc = X(std::integral_constant<int, v>{});
        static_for<1, H>([&](auto hi) {
          constexpr int h = decltype(hi)::value;
          acc = c_add(acc, twiddle_mul<S, r * h>(X(std::integral_constant<int, v + N * h>{})));
        });
        y[v] = twiddle_mul<MT, r * v>(acc);
      });
      fft_dif<N>(y);
      static_for<0, N>([&](auto pi) {
        constexpr int p = decltype(pi)::value;
        constexpr uint32_t kt = static_cast<uint32_t>(S * p + r);
        const float2 val = y[bitrev(p, ilog2(N))];
        const uint32_t k = rate_key(c_norm(val), MASK, kt);
        key = k > key ? k : key;
        if constexpr (DUMP) dump[static_cast<int64_t>(kt) * dump_stride] = val;
      });
    });
    return key;
  }
}

// The sub-transforms r and r + S/2 of a long window together (S >= 8).  Since w_S^{(r + S/2) h} = (-1)^h w_S^{r h}, both
// come from the sums of the same twiddled samples over even and over odd h:
//   y_r[v]       = w_{M_t}^{r v}            (E[v] + O[v]),
//   y_{r+S/2}[v] = w_{M_t}^{r v} w_{2N}^{v} (E[v] - O[v]),
// so each sample is read and twiddled once for the pair.
template <int LOGW, int PT, bool DUMP, bool VTW, typename XF>
__device__ __forceinline__ uint32_t window_key_pair(XF&& X, float2* __restrict__ dump,
                                                    int dump_stride, int r) {
  using Sh = RateShape<LOGW, PT>;
  constexpr int MT = Sh::MT, S = Sh::S, N = Sh::N, H = Sh::H;
  constexpr uint32_t MASK = Sh::MASK;
  static_assert(S >= 8 && H >= 2, "pairs of a long window's sub-transforms");
  auto tw = [](int k) {
    const float2 w = kTw256.v[k & (kTwN - 1)];
    if constexpr (VTW) return make_float2(uniform_in_vgpr(w.x), uniform_in_vgpr(w.y));
    else return w;
  };
  float2 wh[H];
  static_for<1, H>([&](auto hi) {
    constexpr int h = decltype(hi)::value;
    wh[h] = tw((r * h) * (kTwN / S));
  });
  float2 ya[N], yb[N];
  static_for<0, N>([&](auto vi) {
    constexpr int v = decltype(vi)::value;
    float2 e = X(std::integral_constant<int, v>{});
    float2 o = make_float2(0.f, 0.f);
    static_for<1, H>([&](auto hi) {
      constexpr int h = decltype(hi)::value;
      const float2 t = c_mul(X(std::integral_constant<int, v + N * h>{}), wh[h]);
      if constexpr (h % 2 == 0) e = c_add(e, t);
      else o = c_add(o, t);
    });
    if constexpr (v == 0) {
      ya[v] = c_add(e, o);
      yb[v] = c_sub(e, o);
    } else {
      const float2 w = tw((r * v) * (kTwN / MT));
      ya[v] = c_mul(c_add(e, o), w);
      yb[v] = twiddle_mul<2 * N, v>(c_mul(c_sub(e, o), w));
    }
  });
  fft_dif<N>(ya);
  fft_dif<N>(yb);
  uint32_t key = 0;
  static_for<0, N>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    const uint32_t kta = static_cast<uint32_t>(S * p + r);
    const uint32_t ktb = kta + S / 2;
    const float2 va = ya[bitrev(p, ilog2(N))];
    const float2 vb = yb[bitrev(p, ilog2(N))];
    const uint32_t ka = rate_key(c_norm(va), MASK, kta);
    const uint32_t kb = rate_key(c_norm(vb), MASK, ktb);
    key = ka > key ? ka : key;
    key = kb > key ? kb : key;
    if constexpr (DUMP) {
      dump[static_cast<int64_t>(kta) * dump_stride] = va;
      dump[static_cast<int64_t>(ktb) * dump_stride] = vb;
    }
  });
  return key;
}

// ------------------------------------------------------ DPP reductions --
// Full-mask DPP moves with bound_ctrl set: every lane of the patterns used
// here has a source lane, and the form lets the compiler fold the move into
// the consuming max / add.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_mov_dpp(static_cast<int>(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// DPP move into the rows of ROW_MASK only; the other rows get 0, the
// identity of an unsigned max (which lets the move fold into the max).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_rows_u32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_rows_f32(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within 16
constexpr int kDppRor8 = 0x128;        // lane i <- (i + 8) mod 16 within 16
constexpr int kDppRowBcast15 = 0x142;  // row r <- lane 15 of row r - 1
constexpr int kDppRowBcast31 = 0x143;  // rows 2, 3 <- lane 31

// Max of v over the 64 lanes (uniform result): four DPP steps give every
// lane of a 16-lane row the row's maximum; two row broadcasts (lane 15 into
// rows 1 and 3, then lane 31 into rows 2 and 3) gather all four rows in
// lane 63.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_u32<kDppXor1>(v));
  v = max(v, dpp_u32<kDppXor2>(v));
  v = max(v, dpp_u32<kDppHalfMirror>(v));
  v = max(v, dpp_u32<kDppMirror>(v));
  v = max(v, dpp_rows_u32<kDppRowBcast15, 0xA>(v));
  v = max(v, dpp_rows_u32<kDppRowBcast31, 0xC>(v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Sum of v over the 64 lanes (uniform result), by the same steps as
// wave_max_u32.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f32<kDppXor1>(v);
  v += dpp_f32<kDppXor2>(v);
  v += dpp_f32<kDppHalfMirror>(v);
  v += dpp_f32<kDppMirror>(v);
  v += dpp_rows_f32<kDppRowBcast15, 0xA>(v);
  v += dpp_rows_f32<kDppRowBcast31, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Maxima and sums over the 64 lanes of N independent values (uniform
// results), by the steps of wave_max_u32 / wave_sum_dpp with the N
// reductions interleaved so that their dependent DPP chains overlap.
template <int N>
__device__ __forceinline__ void wave_max_u32_n(uint32_t (&v)[N]) {
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_u32<kDppXor1>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_u32<kDppXor2>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_u32<kDppHalfMirror>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_u32<kDppMirror>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_rows_u32<kDppRowBcast15, 0xA>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = max(v[k], dpp_rows_u32<kDppRowBcast31, 0xC>(v[k])); });
  static_for<0, N>([&](auto k) { v[k] = __builtin_amdgcn_readlane(v[k], 63); });
}

template <int N>
__device__ __forceinline__ void wave_sum_f32_n(float (&v)[N]) {
  static_for<0, N>([&](auto k) { v[k] += dpp_f32<kDppXor1>(v[k]); });
  static_for<0, N>([&](auto k) { v[k] += dpp_f32<kDppXor2>(v[k]); });
  static_for<0, N>([&](auto k) { v[k] += dpp_f32<kDppHalfMirror>(v[k]); });
  static_for<0, N>([&](auto k) { v[k] += dpp_f32<kDppMirror>(v[k]); });
  static_for<0, N>([&](auto k) { v[k] += dpp_rows_f32<kDppRowBcast15, 0xA>(v[k]); });
  static_for<0, N>([&](auto k) { v[k] += dpp_rows_f32<kDppRowBcast31, 0xC>(v[k]); });
  static_for<0, N>([&](auto k) {
    v[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[k]), 63));
  });
}

// The bin-block partial of a window whose 64-lane key maximum m is known:
//   (m << 32) | (0xFFFFFFFF - k_f),  k_f = kf_base + kf_step * (lowest lane
// holding m); kf_top = 0xFFFFFFFF - kf_base.
__device__ __forceinline__ uint64_t peak_partial(uint32_t key, uint32_t m, uint32_t kf_top,
                                                 int kf_step) {
  const uint64_t holders = __ballot(key == m);
  const int lane = __builtin_ctzll(holders);
  return (static_cast<uint64_t>(m) << 32) | (kf_top - static_cast<uint32_t>(kf_step * lane));
}

// The same partial when each lane offers its own bin: lo is the lane's
// 0xFFFFFFFF - k_f; the lowest lane holding the maximum gives its k_f.
__device__ __forceinline__ uint64_t peak_partial_at(uint32_t key, uint32_t m, uint32_t lo) {
  const uint64_t holders = __ballot(key == m);
  const int lane = __builtin_ctzll(holders);
  return (static_cast<uint64_t>(m) << 32) |
         static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lo), lane));
}

// Window key of a wave: the 64-lane max of the lanes' rate keys, and the
// lowest lane holding it.  Returned as the bin-block partial
//   (key << 32) | (0xFFFFFFFF - k_f)   with k_f = kf_base + kf_step * lane,
// whose unsigned max over blocks is the window's peak (lowest flat index
// among ties).
__device__ __forceinline__ uint64_t wave_peak(uint32_t key, int kf_base, int kf_step) {
  return peak_partial(key, wave_max_u32(key), 0xFFFFFFFFu - static_cast<uint32_t>(kf_base),
                      kf_step);
}

}  // namespace fringe
