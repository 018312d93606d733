// Fused fringe search for window lengths up to 64 APs: delay transform,
// rate transform and grid peak in one pass over the visibilities.
//
// Work item = (baseline b, time chunk, residue class c of the delay bins):
// the wave owns the 64 bins k_f = R m + c (R = M / 64), lane m holding bin
// R m + c.  Per AP t (paper, section "Code optimization", step 5):
//   z[f'] = w_M^{c f'} sum_h x_t[f' + 64 h] w_R^{c h}      (f' < 64)
//   X_t[R m + c] = sum_{f'} z[f'] w_64^{m f'}
// lane l loads and folds f = l (contiguous loads), one LDS permute moves the
// fold to lane bitrev6(f), then six radix-2 decimation-in-time stages
// across the wave (partners exchanged on the LDS crossbar: ds_swizzle and
// ds_bpermute, no LDS memory) leave X_t of lane m's bin in lane m (in the
// full search two APs at a time, their exchanges interleaved so that one
// crossbar latency serves both).  Each lane keeps the last W_max APs of its bin's
// spectrum in registers: the APs come in periods of P = W_max / 2 that are
// unrolled, so every window that ends in a period has compile-time register
// positions; after the period the newer half moves down.  Every window that
// ends at the AP is searched at once (window_key: rate transform + peak
// key) and reduced over the 64 bins with DPP (wave_peak); one lane stores
// the class's partial peak.  Waves of class 0 also store the AP energies.
// PT = 0 is the delay-only search of the paper's step 6: the window's APs
// are summed, the power of the sum is the key, and each class also stores
// its sum of that power over its 64 bins (for the mean over the delay axis).
//
// Block g runs on XCD g mod 8; the R classes of one (baseline, chunk) are
// given the same XCD and consecutive slots, so the chunk's visibilities are
// fetched from HBM once and served to the other classes from that XCD's L2.
#pragma once

#include "kernels.h"
#include "window_key.h"

namespace fringe {

namespace fused {

// Partner exchange across lanes lane ^ D on one float, on the LDS crossbar
// (it takes no VALU issue slot, a DPP move or permlane swap does):
// ds_swizzle in bit mode within 32 lanes for D <= 16, ds_bpermute from the
// precomputed byte address 4 * (lane ^ 32) for D = 32.
template <int D>
__device__ __forceinline__ float xchg(float v, int addr32) {
  if constexpr (D <= 16)
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (D << 10) | 0x1F));
  else
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr32, __float_as_int(v)));
}

// One DIT stage of half-span D on N independent values (N APs: their
// exchanges are issued together, so one crossbar latency serves all N).
// Lanes with bit D set ("b" lanes) first multiply their value by w (w = 1
// on "a" lanes); then a' = a + w b and b' = a - w b, i.e. new = s * own +
// partner with s = +1 on a lanes, -1 on b lanes.
template <int D, int N>
__device__ __forceinline__ void dit_stage(float2 (&v)[N], float2 w, float s, bool rot,
                                          int addr32) {
  float2 t[N], p[N];
#pragma unroll
  for (int n = 0; n < N; ++n)  // D = 2: the twiddle is 1 or -i (rot), applied by selects
    t[n] = (D == 1) ? v[n]
         : (D == 2) ? make_float2(rot ? v[n].y : v[n].x, rot ? -v[n].x : v[n].y)
                    : c_mul(v[n], w);
#pragma unroll
  for (int n = 0; n < N; ++n) p[n] = make_float2(xchg<D>(t[n].x, addr32), xchg<D>(t[n].y, addr32));
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = make_float2(fmaf(s, t[n].x, p[n].x), fmaf(s, t[n].y, p[n].y));
}

struct LaneConsts {
  float2 w[6];   // stage twiddles (index log2 D)
  float s[6];    // stage signs
  bool rot2;     // stage D = 2 twiddle is -i (b lane with bit 0 set)
  int addr32;    // 4 * (lane ^ 32), the D = 32 exchange's source
};

template <int N>
__device__ __forceinline__ void xlane_dit(float2 (&v)[N], const LaneConsts& k) {
  dit_stage<1>(v, k.w[0], k.s[0], false, k.addr32);
  dit_stage<2>(v, k.w[1], k.s[1], k.rot2, k.addr32);
  dit_stage<4>(v, k.w[2], k.s[2], false, k.addr32);
  dit_stage<8>(v, k.w[3], k.s[3], false, k.addr32);
  dit_stage<16>(v, k.w[4], k.s[4], false, k.addr32);
  dit_stage<32>(v, k.w[5], k.s[5], false, k.addr32);
}

constexpr int ilog2c(int v) { return v > 1 ? 1 + ilog2c(v / 2) : 0; }

// Windows ending at position i of a period of P APs: the length 2^L has
// one there when its first AP is still held (base >= 0) and its start is on
// the length's stride.
template <int P>
constexpr bool window_site(int i, int L) {
  const int w = 1 << L, s = w > 1 ? w / 2 : 1, base = P + i + 1 - w;
  return base >= 0 && ((i + 1 - w) % s + s) % s == 0;
}

template <int P, int LOGWMAX>
constexpr int window_sites(int i) {
  int n = 0;
  for (int L = 0; L <= LOGWMAX; ++L) n += window_site<P>(i, L) ? 1 : 0;
  return n;
}

// The length (log2) of the k-th window ending at position i.
template <int P, int LOGWMAX>
constexpr int site_level(int i, int k) {
  for (int L = 0; L <= LOGWMAX; ++L)
    if (window_site<P>(i, L) && k-- == 0) return L;
  return -1;
}

}  // namespace fused

// Two waves per SIMD at least: the 64-AP history with 16 folds sits just
// above the 256 registers of that occupancy, and holding it there costs a
// few rematerialisations, not spills.
//
// SRCX: the entry's data are delay spectra X[b][t][k_f] (M bins per AP,
// written by the delay-transform kernel with calibration and dedispersion
// applied), not visibilities: the wave of class c owns the contiguous bins
// 64 c + m and reads its 512-byte segment of each AP, and the kernel only
// does the rate transforms and peaks (AP energies come with the spectra).
//
// TWO (streaming plans): an entry's rows may lie in two buffers, the halo's
// in vis and the chunk's in vis2, where the caller holds the chunk; the
// buffer is chosen per AP.  Batch plans run the kernels without the choice.
template <int PT, int LOGWMAX, int HFMAX, bool DUMP, bool SRCX, bool TWO = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DUMP ? 1 : 2)))
fused_search_kernel(const FusedArgs* __restrict__ tab, int n_tab) {
  constexpr int WMAX = 1 << LOGWMAX;
  constexpr int P = WMAX / 2;          // APs per unrolled period
  constexpr int HS = 2 * P;            // history registers (complex)
  constexpr int PD = HFMAX > 4 ? 1 : 2;  // prefetch depth in APs
  // APs whose delay transforms run together (their crossbar exchanges
  // interleaved): the prefetched ones in the full search, where that hides
  // exchange latency behind the rate transforms; one at a time in the
  // delay-only search, which measured faster so (fewer live registers).
  constexpr int G = PT > 0 ? PD : 1;
  static_assert(P % PD == 0 && P % G == 0 && P >= 4, "period");
  // Delay-bin classes per wave: the delay-only search gives a wave NC
  // classes (4 on bands of up to 256 channels, else 2), c = cls + j R (j <
  // NC, R = ceil(M / 64 / NC) waves per (baseline, chunk)), so that an AP's
  // loads, the per-window bookkeeping and one 64-lane reduction per window
  // serve NC classes; lane m then holds the bins (M / 64) m + c.  Classes
  // c >= M / 64 (when NC does not divide M / 64) are ghosts: their fold
  // coefficients are zero, so their power is exactly 0, which never beats a
  // lower class (strictly greater replaces) and adds nothing to the sums.
  // One class per wave in the full search.
  constexpr int NC = (PT == 0 && !SRCX) ? delay_only_classes(HFMAX) : 1;
  // Two classes on a band with 8 or 16 folds (M / 64 = 2R there): their fold
  // twiddles differ by (-1)^h, so the LDS table holds one coefficient per h,
  // g_h w_R'^{cls h}, and the classes take the sums over even h plus and
  // minus the sums over odd h, times their w_M^{c l}.
  constexpr bool FACT2 = NC == 2 && HFMAX > 4;

  const int lane = threadIdx.x;
  // the entry (scan slab) that owns this block
  int lo = 0, hi = n_tab - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].block_off <= static_cast<int64_t>(blockIdx.x)) lo = mid; else hi = mid - 1;
  }
  const FusedArgs& a = tab[lo];
  const int g = static_cast<int>(static_cast<int64_t>(blockIdx.x) - a.block_off);
  const int R = a.R;
  const int cls = (g >> 3) % R;
  const int q = ((g >> 3) / R) * 8 + (g & 7);
  if (q >= a.n_pairs) return;
  const int b = q / a.n_chunks;
  const int chunk = q - b * a.n_chunks;
  const int T = a.T, F = a.F, M = a.M, hf = a.hf;
  // read here, outside every lane-dependent branch, so that it stays a
  // scalar: a copy in a vector register makes the buffer descriptor built
  // from it non-uniform, and every load then runs in a loop over lanes
  const int T_rows = __builtin_amdgcn_readfirstlane(a.T_rows);
  const int own_lo = chunk * a.chunk;
  const int own_hi = min(T, own_lo + a.chunk);
  const int t_end = min(T, own_hi + WMAX - 1);

  // lane constants
  const int fl = static_cast<int>(__builtin_bitreverse32(static_cast<uint32_t>(lane)) >> 26);
  const int rev_addr = fl * 4;  // ds_bpermute source lane bitrev6(lane), in bytes
  fused::LaneConsts kc;
  const float2* tw = a.tw;
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int d = 1 << st;
    const bool bl = (lane & d) != 0;
    kc.s[st] = bl ? -1.f : 1.f;
    const float2 w = ld_global(tw + (lane & (d - 1)) * (M / (2 * d)));
    kc.w[st] = bl ? w : make_float2(1.f, 0.f);
  }
  kc.rot2 = (lane & 2) != 0 && (lane & 1) != 0;
  kc.addr32 = (lane ^ 32) * 4;
  // Wide bands (more than 4 folds) keep the per-lane fold coefficients and,
  // with dedispersion, the shifted load offsets in LDS, read back per AP:
  // in registers they would push the kernel with a 64-AP history to one
  // wave per SIMD.  Narrow bands keep both in registers.
  constexpr bool TAB_LDS = HFMAX > 4;
  __shared__ f32x2_t s_gw[TAB_LDS ? (FACT2 ? 1 : NC) * HFMAX : 1][64];  // [class j][fold h] at j HFMAX + h
  __shared__ uint32_t s_off[TAB_LDS ? HFMAX : 1][64];
  typedef const volatile __attribute__((address_space(3))) f32x2_t* LdsGw;
  typedef const volatile __attribute__((address_space(3))) uint32_t* LdsOff;

  const float2* xb = a.vis + static_cast<int64_t>(b) * a.vis_stride;
  // Loads are unconditional and in bounds (the AP clamped to T - 1, lanes
  // past the band reading sample 0 or past the row, where the buffer's range
  // check returns zeros); what lies outside the data is zeroed where it is
  // used, so no load has to complete before later work issues.
  bool lane_in[HFMAX];
#pragma unroll
  for (int h = 0; h < HFMAX; ++h) lane_in[h] = h < hf && lane + 64 * h < F;
  const uint32_t lane8 = static_cast<uint32_t>(lane) * sizeof(float2);
  // (a baseline's data is < 4 GiB, checked at plan time)
  const uint32_t row_bytes = static_cast<uint32_t>(F) * sizeof(float2);
  // dedispersion: channel f of AP t is read from AP t + d_f.  The shift is
  // folded into the lane's offset, the AP is added to it (not given as the
  // scalar offset), and the buffer's record limit, the T_rows APs the data
  // hold (T, or more in a streaming plan, whose stage holds the lookahead
  // the shifts need), turns the reads past the data into zeros (with shifts
  // a baseline is < 1 GiB, so no offset wraps).  Without shifts every read
  // is in range.
  const bool has_s = a.shifts != nullptr;
  // byte offset of the lane's sample of fold h in an AP row (natural order:
  // each load is one contiguous segment)
  auto shifted_off = [&](int h) -> uint32_t {
    if (!lane_in[h]) return 0u;
    uint32_t o = lane8 + static_cast<uint32_t>(64 * sizeof(float2) * h);
    if (has_s)
      o += static_cast<uint32_t>(min(max(a.shifts[lane + 64 * h], 0), T_rows)) * row_bytes;
    return o;
  };
  uint32_t lane_off[TAB_LDS ? 1 : HFMAX];
#pragma unroll
  for (int h = 0; h < (TAB_LDS ? 1 : HFMAX); ++h) lane_off[h] = shifted_off(h);
  if constexpr (TAB_LDS) {
    if (has_s) {
#pragma unroll
      for (int h = 0; h < HFMAX; ++h) s_off[h][lane] = shifted_off(h);
    }
  }
  // A streamed chunk read where the caller holds it: the halo's rows [0,
  // halo) in vis, the chunk's rows from vis2 (never with shifts, so the row
  // is the AP's for every lane and the choice of buffer is wave-uniform).
  const bool two = TWO && a.vis2 != nullptr;
  const int halo = two ? __builtin_amdgcn_readfirstlane(a.halo) : T_rows;
  const auto vrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(xb), static_cast<short>(0),
      static_cast<int>(static_cast<uint32_t>(halo) * row_bytes), kBufferWord3);
  const auto vrs2 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(two ? a.vis2 + static_cast<int64_t>(b) * a.vis2_stride : xb),
      static_cast<short>(0),
      static_cast<int>(static_cast<uint32_t>(two ? T_rows - halo : 0) * row_bytes), kBufferWord3);
  auto load_ap = [&](int t, float2 (&dst)[HFMAX]) {
    int tr = min(t, T - 1);
    auto vrs_t = vrs;
    if constexpr (TWO) {
      if (tr >= halo) {
        vrs_t = vrs2;
        tr -= halo;
      }
    }
    const uint32_t toff = static_cast<uint32_t>(tr) * row_bytes;
    if constexpr (TAB_LDS) {
      if (has_s) {
        const LdsOff so = (LdsOff)(&s_off[0][lane]);
#pragma unroll
        for (int h = 0; h < HFMAX; ++h) dst[h] = ld_buffer(vrs_t, so[64 * h] + toff, 0);
      } else {
#pragma unroll
        for (int h = 0; h < HFMAX; ++h)
          dst[h] = ld_buffer(vrs_t, lane8 + toff, static_cast<uint32_t>(64 * sizeof(float2) * h));
      }
    } else {
#pragma unroll
      for (int h = 0; h < HFMAX; ++h) dst[h] = ld_buffer(vrs_t, lane_off[h] + toff, 0);
    }
  };
  const bool band_full = F == 64 * HFMAX;  // every lane in band for every fold
  // The fold's coefficients per lane l (f' = l) and h: the calibration gain
  // of channel l + 64 h (1 without gains), the fold twiddle w_R^{c h} and
  // the twiddle w_M^{c l} applied before the permute (the same value the
  // permute's destination lane would apply), so a calibrated AP costs what
  // an uncalibrated one does; |g|^2 scales the AP energies.  The gains'
  // buffer holds exactly the baseline's F gains, so lanes past the band read
  // zeros.
  const bool has_g = a.gains != nullptr;
  float2 wsrc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) wsrc[j] = ld_global(tw + (((cls + j * R) * lane) & (M - 1)));
  const auto grs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(has_g ? a.gains + static_cast<int64_t>(b) * F : a.gains),
      static_cast<short>(0), static_cast<int>(static_cast<uint32_t>(F) * sizeof(float2)),
      kBufferWord3);
  auto coef = [&](int j, int h) -> float2 {
    const int c = cls + j * R;
    if (NC > 1 && c >= (M >> 6)) return make_float2(0.f, 0.f);  // a ghost class
    const float2 w = ld_global(tw + (((c * h) * 64) & (M - 1)));  // w_R^{c h}
    const float2 ww = c_mul(make_float2(in_vgpr(w.x), in_vgpr(w.y)), wsrc[j]);
    if (!has_g) return ww;
    return c_mul(ld_buffer(grs, lane8 + 64 * sizeof(float2) * h, 0), ww);
  };
  // Four classes of a 4-fold band, factored: c = cls + jR and M / 64 = 4R
  // make w_R'^{c h} (R' = M / 64) = w_R'^{cls h} w_4^{j h}, so the four folds
  // are one multiply per h by fa[h] = g_h w_R'^{cls h}, a 4-point DFT over h
  // (S_j = sum_h u_h (-i)^{j h}: adds and swaps) and one multiply per class
  // by fb[j] = w_M^{c l}.  With M / 64 = 2R the second class is cls + R,
  // whose fold takes (-1)^h, the DFT's S_2 (fmid); ghost classes get fb = 0.
  constexpr bool FACT = NC == 4 && HFMAX == 4 && !TAB_LDS;
  float2 fa[FACT ? HFMAX : 1], fb[(FACT || FACT2) ? NC : 1];
  const bool fmid = (M >> 6) < 4 * R;
  float2 gw[FACT ? 1 : NC][TAB_LDS ? 1 : HFMAX];
  float gn[TAB_LDS ? 1 : HFMAX];
  if constexpr (FACT) {
#pragma unroll
    for (int h = 0; h < HFMAX; ++h) {
      const float2 w = ld_global(tw + (((cls * h) * 64) & (M - 1)));  // w_R'^{cls h}
      float2 v = make_float2(in_vgpr(w.x), in_vgpr(w.y));
      if (has_g) v = c_mul(ld_buffer(grs, lane8 + 64 * sizeof(float2) * h, 0), v);
      fa[h] = v;
    }
#pragma unroll
    for (int j = 0; j < NC; ++j)
      fb[j] = cls + j * R < (M >> 6) ? wsrc[j] : make_float2(0.f, 0.f);
  } else if constexpr (FACT2) {
#pragma unroll
    for (int h = 0; h < HFMAX; ++h) {
      const float2 w = ld_global(tw + (((cls * h) * 64) & (M - 1)));  // w_R'^{cls h}
      float2 v = make_float2(in_vgpr(w.x), in_vgpr(w.y));
      if (has_g) v = c_mul(ld_buffer(grs, lane8 + 64 * sizeof(float2) * h, 0), v);
      s_gw[h][lane] = f32x2_t{v.x, v.y};
    }
#pragma unroll
    for (int j = 0; j < NC; ++j)
      fb[j] = cls + j * R < (M >> 6) ? wsrc[j] : make_float2(0.f, 0.f);
  } else if constexpr (TAB_LDS) {
#pragma unroll
    for (int h = 0; h < HFMAX; ++h) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float2 c = coef(j, h);
        s_gw[j * HFMAX + h][lane] = f32x2_t{c.x, c.y};
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < HFMAX; ++h) {
#pragma unroll
      for (int j = 0; j < NC; ++j) gw[j][h] = coef(j, h);
      gn[h] = has_g ? c_norm(ld_buffer(grs, lane8 + 64 * sizeof(float2) * h, 0)) : 1.f;
    }
  }
  // coefficient h of this lane (from LDS: |g|^2 = |coefficient|^2 up to
  // rounding, the twiddles having unit modulus)
  auto coef_of = [&](int j, int h) -> float2 {
    if constexpr (TAB_LDS) {
      const f32x2_t v = ((LdsGw)(&s_gw[j * HFMAX][lane]))[64 * h];
      return make_float2(v.x, v.y);
    } else {
      return gw[j][h];
    }
  };
  auto sample = [&](float2 x, int h, bool t_in) {
    const bool ok = t_in && lane_in[h];
    return make_float2(ok ? x.x : 0.f, ok ? x.y : 0.f);
  };

  float2 pre[SRCX ? 1 : PD][HFMAX];
  if constexpr (!SRCX) {
    static_for<0, PD>([&](auto di) {
      constexpr int d = decltype(di)::value;
      load_ap(own_lo + d, pre[d]);
    });
  }
  // spectra in: this class's 64 bins of AP t, PDX APs prefetched (8 measured
  // 1 % faster than 4 on the 1,024-channel spectra)
  constexpr int PDX = P >= 16 ? 8 : 4;
  static_assert(!SRCX || P % PDX == 0, "period");
  const uint32_t xrow = static_cast<uint32_t>(M) * sizeof(float2);
  const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(xb), static_cast<short>(0),
      static_cast<int>(static_cast<uint32_t>(T) * xrow), kBufferWord3);
  auto load_x = [&](int t) {
    return ld_buffer(xrs, lane8 + static_cast<uint32_t>(min(t, T - 1)) * xrow,
                     static_cast<uint32_t>(cls) * 64 * sizeof(float2));
  };
  float2 prex[SRCX ? PDX : 1];
  if constexpr (SRCX) {
#pragma unroll
    for (int d = 0; d < PDX; ++d) prex[d] = load_x(own_lo + d);
  }
  // full search: the last 2P APs of this lane's bin.  Delay-only search:
  // instead, per length 2^L the coherent sums of the windows that ended in
  // the last 2P APs (sum[L][P + i] for a window ending at position i of the
  // period), each window being the sum of its two halves; only the few
  // sums a later window still needs stay live in registers.
  float2 hist[HS];
  float2 sum[NC][LOGWMAX + 1][HS];
#pragma unroll
  for (int k = 0; k < HS; ++k) {
    hist[k] = make_float2(0.f, 0.f);
#pragma unroll
    for (int L = 0; L <= LOGWMAX; ++L)
#pragma unroll
      for (int j = 0; j < NC; ++j) sum[j][L][k] = make_float2(0.f, 0.f);
  }

  const auto eb = gptr(a.e + static_cast<int64_t>(b) * T);
  // per window length 2^L: searched or not, and the part index of the
  // window with start index j is pidx[L] + j (fields read once, before the
  // loop, so they live in scalar registers)
  const auto part = gptr(a.part + static_cast<int64_t>(cls) * a.slab_windows +
                         static_cast<int64_t>(b) * a.nwb);
  const auto epart = gptr(PT == 0 ? a.epart + static_cast<int64_t>(cls) * a.slab_windows +
                                        static_cast<int64_t>(b) * a.nwb
                                  : a.epart);
  const int t_emit = a.t_emit;
  const uint32_t own_n = static_cast<uint32_t>(own_hi - own_lo);
  // bin of lane m: R m + c (visibilities in, bins interleaved over the
  // classes by the cross-lane transform) or 64 c + m (spectra in)
  const int kf_step = SRCX ? 1 : (NC > 1 ? (M >> 6) : R);
  const int my_bin = SRCX ? 64 * cls + lane : cls + kf_step * lane;
  const uint32_t kf_top = 0xFFFFFFFFu - static_cast<uint32_t>(SRCX ? 64 * cls : cls);
  // NC classes: 0xFFFFFFFF - k_f of this lane's bin of class j
  uint32_t lo_j[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j)
    lo_j[j] = kf_top - static_cast<uint32_t>(kf_step * lane) - static_cast<uint32_t>(j * R);
  int pidx[LOGWMAX + 1];
  bool on[LOGWMAX + 1];
  int64_t gidx[LOGWMAX + 1];
#pragma unroll
  for (int L = 0; L <= LOGWMAX; ++L) {
    const int lvl = a.lvl_of_log[L];
    on[L] = lvl >= 0;
    pidx[L] = lvl >= 0 ? a.lvl_off[lvl] - a.lvl_j0[lvl] : 0;
    gidx[L] = 0;
    if constexpr (DUMP) {
      if (lvl >= 0)
        gidx[L] = a.dump_base + static_cast<int64_t>(b) * a.grid_per_bl + a.lvl_goff[lvl] -
                  static_cast<int64_t>(a.lvl_j0[lvl]) * (PT << L) * M + my_bin;
    }
  }

  for (int p0 = own_lo; p0 < t_end; p0 += P) {
    // this period's store bases per length: a window with start p0 + d
    // (d a multiple of its stride s) has index pidx + p0 / s + d / s, so its
    // slot is pb[L][d / s], a constant offset from a base set once here
    // (p0 is a multiple of every stride).  The base index is signed: with a
    // streaming plan pidx < 0, and a period's base may lie before the
    // buffer while the windows it reports (d > 0) lie inside it.
    std::remove_const_t<decltype(part)> pb[LOGWMAX + 1];
    std::remove_const_t<decltype(epart)> epb[LOGWMAX + 1];
    static_for<0, LOGWMAX + 1>([&](auto li) {
      constexpr int L = decltype(li)::value;
      constexpr int LS = L > 0 ? L - 1 : 0;
      const int64_t o = static_cast<int64_t>(pidx[L]) + (p0 >> LS);
      pb[L] = part + o;
      if constexpr (PT == 0) epb[L] = epart + o;
    });
    static_for<0, P>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int t = p0 + i;
      // delay transform of APs t .. t + G - 1 for this class (transformed
      // together at the first of them): fold, then across the wave.
      // Samples outside the data (past the scan's end, lanes past a band
      // narrower than the fold) are zeroed on a uniform branch, so APs with
      // none spend nothing on it.
      if constexpr (SRCX) {
        float2 z = prex[i % PDX];
        if (t >= T) z = make_float2(0.f, 0.f);
        prex[i % PDX] = load_x(t + PDX);
        if constexpr (PT > 0) hist[P + i] = z;
        else sum[0][0][P + i] = z;
      } else if constexpr (i % G == 0) {
        float2 z[G * NC];  // AP t + e, class cls + j R at z[e NC + j]
        static_for<0, G>([&](auto di) {
          constexpr int e = decltype(di)::value;
          constexpr int fs = (i + e) % PD;  // prefetch slot of AP t + e
          const int te = t + e;
          if (!(band_full && te < T)) {
            const bool t_in = te < T;
#pragma unroll
            for (int h = 0; h < HFMAX; ++h) pre[fs][h] = sample(pre[fs][h], h, t_in);
          }
          if constexpr (FACT) {
            float2 u[HFMAX];
#pragma unroll
            for (int h = 0; h < HFMAX; ++h) u[h] = c_mul(pre[fs][h], fa[h]);
            const float2 a0 = c_add(u[0], u[2]), a1 = c_sub(u[0], u[2]);
            const float2 b0 = c_add(u[1], u[3]), b1 = c_sub(u[1], u[3]);
            const float2 mb1 = make_float2(b1.y, -b1.x);  // -i b1
            const float2 s0 = c_add(a0, b0), s2 = c_sub(a0, b0);
            const float2 s1 = c_add(a1, mb1), s3 = c_sub(a1, mb1);
            z[e * NC + 0] = c_mul(s0, fb[0]);
            z[e * NC + 1] = c_mul(fmid ? s2 : s1, fb[1]);
            z[e * NC + 2] = c_mul(s2, fb[2]);
            z[e * NC + 3] = c_mul(s3, fb[3]);
          } else if constexpr (FACT2) {
            float2 ev = c_mul(pre[fs][0], coef_of(0, 0)), od = make_float2(0.f, 0.f);
#pragma unroll
            for (int h = 1; h < HFMAX; ++h) {
              const float2 u = c_mul(pre[fs][h], coef_of(0, h));
              if (h % 2 == 0) ev = c_add(ev, u);
              else od = c_add(od, u);
            }
            z[e * NC + 0] = c_mul(c_add(ev, od), fb[0]);
            z[e * NC + 1] = c_mul(c_sub(ev, od), fb[1]);
          } else {
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              float2& zz = z[e * NC + j];
              zz = c_mul(pre[fs][0], coef_of(j, 0));
#pragma unroll
              for (int h = 1; h < HFMAX; ++h) zz = c_add(zz, c_mul(pre[fs][h], coef_of(j, h)));
            }
          }
          if (PT > 0 && cls == 0) {  // AP energies: one class per (baseline, chunk) stores them
            float es = 0.f;
#pragma unroll
            for (int h = 0; h < HFMAX; ++h) {
              float gh;
              if constexpr (TAB_LDS) gh = has_g ? c_norm(coef_of(0, h)) : 1.f;
              else gh = gn[h];
              es = fmaf(gh, c_norm(pre[fs][h]), es);
            }
            const float en = wave_sum_dpp(es);
            if (lane == 0 && te < own_hi) eb[te] = en;
          }
          load_ap(te + PD, pre[fs]);
          // lane l folded f = l; the transform wants f' = bitrev6(l) in lane l
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            float2& zz = z[e * NC + j];
            zz = make_float2(
                __int_as_float(__builtin_amdgcn_ds_bpermute(rev_addr, __float_as_int(zz.x))),
                __int_as_float(__builtin_amdgcn_ds_bpermute(rev_addr, __float_as_int(zz.y))));
          }
        });
        fused::xlane_dit(z, kc);
        static_for<0, G>([&](auto di) {
          constexpr int e = decltype(di)::value;
          if constexpr (PT > 0) {
            hist[P + i + e] = z[e];
          } else {
#pragma unroll
            for (int j = 0; j < NC; ++j) sum[j][0][P + i + e] = z[e * NC + j];
          }
        });
      }

      // every window that ends at AP t (and is reported: within the data,
      // at or after the first AP the call reports, starting in this chunk)
      const bool t_ok = t < T && t >= t_emit;
      if constexpr (PT == 0) {
        // delay-only: each window's APs summed coherently; the power of the
        // sum in this lane's bin is its key, and the class's power sum goes
        // to the mean over the delay axis.  The window (s, 2^L) is the sum of
        // (s, 2^(L-1)), which ended 2^(L-1) APs ago, and (s + 2^(L-1),
        // 2^(L-1)), which ends here (every length is summed, searched or
        // not, as the next one's halves).  The windows ending here are
        // reduced together (independent DPP chains interleaved).  With NC
        // classes a lane first takes the strongest of its NC bins (the lowest
        // class on ties: the lower bin) and sums their powers.
        static_for<1, LOGWMAX + 1>([&](auto li) {
          constexpr int L = decltype(li)::value;
          if constexpr (fused::window_site<P>(i, L)) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
              sum[j][L][P + i] =
                  c_add(sum[j][L - 1][P + i - (1 << (L - 1))], sum[j][L - 1][P + i]);
          }
        });
        constexpr int NS = fused::window_sites<P, LOGWMAX>(i);
        uint32_t key[NS], mx[NS], lo[NS];
        float ps[NS];
        static_for<0, NS>([&](auto ki) {
          constexpr int k = decltype(ki)::value;
          constexpr int L = fused::site_level<P, LOGWMAX>(i, k);
          ps[k] = c_norm(sum[0][L][P + i]);
          key[k] = __float_as_uint(ps[k]);
          if constexpr (NC > 1) {
            lo[k] = lo_j[0];
#pragma unroll
            for (int j = 1; j < NC; ++j) {
              const float pj = c_norm(sum[j][L][P + i]);
              ps[k] += pj;
              const uint32_t kj = __float_as_uint(pj);
              const bool up = kj > key[k];
              key[k] = up ? kj : key[k];
              lo[k] = up ? lo_j[j] : lo[k];
            }
          }
          mx[k] = key[k];
        });
        wave_max_u32_n(mx);
        wave_sum_f32_n(ps);
        static_for<0, NS>([&](auto ki) {
          constexpr int k = decltype(ki)::value;
          constexpr int L = fused::site_level<P, LOGWMAX>(i, k);
          constexpr int W = 1 << L;
          constexpr int s = W > 1 ? W / 2 : 1;
          constexpr int d = (i + 1 - W) / s;  // start - p0, in strides
          const int start = t + 1 - W;
          if (on[L] && t_ok && static_cast<uint32_t>(start - own_lo) < own_n) {
            uint64_t pk;
            if constexpr (NC > 1) pk = peak_partial_at(key[k], mx[k], lo[k]);
            else pk = peak_partial(key[k], mx[k], kf_top, kf_step);
            if (lane == 0) {
              pb[L][d] = pk;
              epb[L][d] = ps[k];
            }
          }
        });
      } else {
        static_for<0, LOGWMAX + 1>([&](auto li) {
          constexpr int L = decltype(li)::value;
          constexpr int W = 1 << L;
          constexpr int s = W > 1 ? W / 2 : 1;
          constexpr int base = P + i + 1 - W;  // register of the window's first AP
          if constexpr (fused::window_site<P>(i, L)) {
            constexpr int d = (i + 1 - W) / s;  // start - p0, in strides
            const int start = t + 1 - W;
            if (on[L] && t_ok && static_cast<uint32_t>(start - own_lo) < own_n) {
              float2* dump = nullptr;
              if constexpr (DUMP) {
                const uint32_t j = static_cast<uint32_t>(start) >> fused::ilog2c(s);
                dump = a.dump + gidx[L] + static_cast<int64_t>(j) * (PT * W) * M;
              }
              // from spectra (registers to spare at two waves per SIMD): the
              // 64-AP windows' sub-transforms by pairs
              const uint32_t key = window_key<L, PT, DUMP, false, SRCX>(
                  [&](auto ui) { return hist[base + decltype(ui)::value]; }, dump, M);
              const uint64_t pk = peak_partial(key, wave_max_u32(key), kf_top, kf_step);
              if (lane == 0) pb[L][d] = pk;
            }
          }
        });
      }
    });
#pragma unroll
    for (int k = 0; k < P; ++k) {
      hist[k] = hist[P + k];
#pragma unroll
      for (int L = 0; L <= LOGWMAX; ++L)
#pragma unroll
        for (int j = 0; j < NC; ++j) sum[j][L][k] = sum[j][L][P + k];
    }
  }
}

// Launches the instantiation, or with occ set, stores the work groups (one
// wave each) it keeps resident per CU and launches nothing.
template <int PT, int LOGWMAX, int HFMAX, bool DUMP, bool SRCX = false, bool TWO = false>
hipError_t launch_fused_t(const FusedArgs* tab, int n_tab, int64_t blocks, hipStream_t st,
                          int* occ) {
  if (occ)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        occ,
        reinterpret_cast<const void*>(&fused_search_kernel<PT, LOGWMAX, HFMAX, DUMP, SRCX, TWO>),
        64, 0);
  if (blocks == 0 || n_tab == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fused_search_kernel<PT, LOGWMAX, HFMAX, DUMP, SRCX, TWO>),
                     dim3(static_cast<unsigned>(blocks)), dim3(64), 0, st, tab, n_tab);
  return hipGetLastError();
}

}  // namespace fringe
