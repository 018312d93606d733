// Consumers of the candidate list, on the host: matching candidate windows
// into single pulses (per baseline across window lengths, then across
// baselines) and the delay-only localization of Eq. (2).
//
// Both matching levels form groups anchored at their strongest member:
// repeatedly the strongest remaining item and every remaining item whose AP
// span shares an AP with the anchor's.  Items are visited once in strength
// order (an item removed by an earlier group is skipped), and the members
// of a group are found among the items sorted by first AP: those starting
// in [anchor start - longest span + 1, anchor end), so each group costs a
// binary search plus the items in reach of its anchor.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <utility>
#include <vector>

#include "fringe_match.h"

namespace fringe {
void set_last_error(const char* msg);
}

namespace {

int fail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  fringe::set_last_error(buf);
  return code;
}

// A pulse on one baseline: the group's span, its size, and the index of its
// representative (anchor) candidate.
struct BaselinePulse {
  int32_t scan, baseline, t_lo, t_hi, n_windows, n_lengths;
  int64_t rep;
};

// Window strength: higher SNR, then the shorter window, then the earlier
// start (then the lower input index, for duplicate records).
bool stronger(const fringe_candidate* c, int64_t a, int64_t b) {
  const fringe_candidate &x = c[a], &y = c[b];
  if (x.snr != y.snr) return x.snr > y.snr;
  if (x.window_ap != y.window_ap) return x.window_ap < y.window_ap;
  if (x.t_start != y.t_start) return x.t_start < y.t_start;
  return a < b;
}

int32_t count_distinct(std::vector<int32_t>& v) {
  std::sort(v.begin(), v.end());
  return int32_t(std::unique(v.begin(), v.end()) - v.begin());
}

// Anchored groups over items [0, n) with spans span(i) = [lo, hi), visited
// in the order `by_strength`.  Calls emit(anchor, members) for every group,
// in the order found.
template <class Span, class Emit>
void anchored_groups(int64_t n, const std::vector<int64_t>& by_strength, Span span, Emit emit) {
  std::vector<int64_t> by_start(by_strength);
  std::sort(by_start.begin(), by_start.end(), [&](int64_t a, int64_t b) {
    int64_t la = span(a).first, lb = span(b).first;
    return la != lb ? la < lb : a < b;
  });
  std::vector<int64_t> starts(n);
  int64_t longest = 1;
  for (int64_t k = 0; k < n; ++k) {
    starts[k] = span(by_start[k]).first;
    longest = std::max(longest, span(by_start[k]).second - span(by_start[k]).first);
  }
  std::vector<char> removed(size_t(n), 0);  // indexed by item
  std::vector<int64_t> members;
  for (int64_t anchor : by_strength) {
    if (removed[anchor]) continue;
    auto [s0, e0] = span(anchor);
    members.clear();
    int64_t k = std::lower_bound(starts.begin(), starts.end(), s0 - longest + 1) - starts.begin();
    for (; k < n && starts[k] < e0; ++k) {
      int64_t it = by_start[k];
      if (!removed[it] && span(it).second > s0) {
        removed[it] = 1;
        members.push_back(it);
      }
    }
    emit(anchor, members);
  }
}

std::vector<BaselinePulse> baseline_pulses(const fringe_candidate* c, int64_t n,
                                           int32_t min_windows) {
  // candidates grouped by (scan, baseline), each group in strength order
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [c](int64_t a, int64_t b) {
    if (c[a].scan != c[b].scan) return c[a].scan < c[b].scan;
    if (c[a].baseline != c[b].baseline) return c[a].baseline < c[b].baseline;
    return stronger(c, a, b);
  });
  std::vector<BaselinePulse> out;
  std::vector<int32_t> lengths;
  std::vector<int64_t> local;
  int64_t i = 0;
  while (i < n) {
    int64_t j = i + 1;
    while (j < n && c[idx[j]].scan == c[idx[i]].scan && c[idx[j]].baseline == c[idx[i]].baseline)
      ++j;
    const int64_t* gi = idx.data() + i;  // the run's candidates, strongest first
    local.resize(j - i);
    for (int64_t k = 0; k < j - i; ++k) local[k] = k;
    auto span = [c, gi](int64_t k) {
      const fringe_candidate& w = c[gi[k]];
      return std::pair<int64_t, int64_t>(w.t_start, int64_t(w.t_start) + w.window_ap);
    };
    anchored_groups(j - i, local, span, [&](int64_t anchor, const std::vector<int64_t>& mem) {
      lengths.clear();
      int64_t lo = INT64_MAX, hi = INT64_MIN;
      for (int64_t k : mem) {
        lengths.push_back(c[gi[k]].window_ap);
        lo = std::min(lo, span(k).first);
        hi = std::max(hi, span(k).second);
      }
      int32_t n_len = count_distinct(lengths);
      if (n_len >= min_windows)
        out.push_back({c[gi[anchor]].scan, c[gi[anchor]].baseline, int32_t(lo), int32_t(hi),
                       int32_t(mem.size()), n_len, gi[anchor]});
    });
    i = j;
  }
  return out;
}

void fill_row(fringe_pulse& r, const BaselinePulse& p, const fringe_candidate& w, int32_t pulse) {
  r.scan = p.scan;
  r.pulse = pulse;
  r.baseline = p.baseline;
  r.window_ap = w.window_ap;
  r.t_start = w.t_start;
  r.k_rate = w.k_rate;
  r.k_delay = w.k_delay;
  r.t_lo = p.t_lo;
  r.t_hi = p.t_hi;
  r.n_windows = p.n_windows;
  r.n_lengths = p.n_lengths;
  r.amp = w.amp;
  r.snr = w.snr;
  r.reserved = 0;
  r.delay_s = w.delay_s;
  r.rate_hz = w.rate_hz;
}

bool finite_all(const double* v, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Least squares for two unknowns by a Gram-Schmidt QR of the n x 2 design
// [a | d] (the second column orthogonalised twice), over every row but
// `skip` (skip = -1 keeps them all).  Returns false when the second column
// is, to rounding, a multiple of the first (or either is zero).
bool lsq2(const double* y, const double* a, const double* d, int32_t n, int32_t skip,
          double* x, double* rms) {
  double r11 = 0;
  for (int32_t i = 0; i < n; ++i)
    if (i != skip) r11 += a[i] * a[i];
  r11 = std::sqrt(r11);
  double na2 = 0;
  for (int32_t i = 0; i < n; ++i)
    if (i != skip) na2 += d[i] * d[i];
  na2 = std::sqrt(na2);
  if (!(r11 > 0) || !(na2 > 0)) return false;
  std::vector<double> v(n, 0.0);
  double r12 = 0;
  for (int32_t i = 0; i < n; ++i)
    if (i != skip) r12 += a[i] / r11 * d[i];
  for (int32_t i = 0; i < n; ++i) v[i] = (i == skip) ? 0.0 : d[i] - r12 * a[i] / r11;
  double c = 0;
  for (int32_t i = 0; i < n; ++i) c += a[i] / r11 * v[i];
  for (int32_t i = 0; i < n; ++i)
    if (i != skip) v[i] -= c * a[i] / r11;
  r12 += c;
  double r22 = 0;
  for (int32_t i = 0; i < n; ++i) r22 += v[i] * v[i];
  r22 = std::sqrt(r22);
  if (!(r22 > 1e-12 * na2)) return false;
  double qy1 = 0, qy2 = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (i == skip) continue;
    qy1 += a[i] / r11 * y[i];
    qy2 += v[i] / r22 * y[i];
  }
  x[1] = qy2 / r22;
  x[0] = (qy1 - r12 * x[1]) / r11;
  double ss = 0;
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (i == skip) continue;
    double e = y[i] - a[i] * x[0] - d[i] * x[1];
    ss += e * e;
    ++m;
  }
  *rms = std::sqrt(ss / m);
  return true;
}

}  // namespace

extern "C" {

int fringe_match(const fringe_candidate* candidates, int64_t n, const fringe_match_params* params,
                 fringe_pulse* out, int64_t capacity, int64_t* n_rows, int64_t* n_pulses) {
  if (!params || !n_rows || !n_pulses || n < 0 || capacity < 0 || (n > 0 && !candidates) ||
      (capacity > 0 && !out))
    return fail(FRINGE_E_INVALID, "fringe_match: null pointer or negative size");
  if (params->min_windows < 1 || params->min_baselines < 1)
    return fail(FRINGE_E_INVALID, "fringe_match: min_windows %d and min_baselines %d must be >= 1",
                params->min_windows, params->min_baselines);
  for (int64_t i = 0; i < n; ++i) {
    const fringe_candidate& w = candidates[i];
    if (w.window_ap < 1 || w.t_start < 0 || int64_t(w.t_start) + w.window_ap > INT32_MAX ||
        !std::isfinite(w.snr))
      return fail(FRINGE_E_INVALID,
                  "fringe_match: candidate %lld has window_ap %d, t_start %d, snr %g",
                  (long long)i, w.window_ap, w.t_start, double(w.snr));
  }
  std::vector<BaselinePulse> bp = baseline_pulses(candidates, n, params->min_windows);
  // Pulse strength: that of its representative window, then the lower
  // baseline.
  auto pulse_stronger = [candidates, &bp](int64_t a, int64_t b) {
    const fringe_candidate &x = candidates[bp[a].rep], &y = candidates[bp[b].rep];
    if (x.snr != y.snr) return x.snr > y.snr;
    if (x.window_ap != y.window_ap) return x.window_ap < y.window_ap;
    if (x.t_start != y.t_start) return x.t_start < y.t_start;
    return bp[a].baseline < bp[b].baseline;
  };
  // single pulses of every scan: (scan, first AP, order found, members)
  struct Group {
    int32_t scan;
    int64_t t_lo, found;
    std::vector<int64_t> members;
  };
  std::vector<Group> found;
  std::vector<int64_t> order(bp.size());
  for (size_t k = 0; k < bp.size(); ++k) order[k] = int64_t(k);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return bp[a].scan != bp[b].scan ? bp[a].scan < bp[b].scan : pulse_stronger(a, b);
  });
  std::vector<int32_t> bl;
  std::vector<int64_t> local;
  size_t i = 0;
  while (i < order.size()) {
    size_t j = i + 1;
    while (j < order.size() && bp[order[j]].scan == bp[order[i]].scan) ++j;
    const int64_t* gi = order.data() + i;
    local.resize(j - i);
    for (size_t k = 0; k < j - i; ++k) local[k] = int64_t(k);
    auto span = [&bp, gi](int64_t k) {
      return std::pair<int64_t, int64_t>(bp[gi[k]].t_lo, bp[gi[k]].t_hi);
    };
    int64_t n_found = 0;
    anchored_groups(int64_t(j - i), local, span, [&](int64_t, const std::vector<int64_t>& mem) {
      bl.clear();
      int64_t lo = INT64_MAX;
      for (int64_t k : mem) {
        bl.push_back(bp[gi[k]].baseline);
        lo = std::min(lo, span(k).first);
      }
      if (count_distinct(bl) >= params->min_baselines) {
        Group g{bp[gi[mem[0]]].scan, lo, n_found, {}};
        for (int64_t k : mem) g.members.push_back(gi[k]);
        found.push_back(std::move(g));
      }
      ++n_found;
    });
    i = j;
  }
  std::sort(found.begin(), found.end(), [](const Group& x, const Group& y) {
    if (x.scan != y.scan) return x.scan < y.scan;
    return x.t_lo != y.t_lo ? x.t_lo < y.t_lo : x.found < y.found;
  });
  int64_t rows = 0, pulses = 0;
  for (Group& g : found) {
    // one row per baseline: its strongest pulse, rows in baseline order
    std::sort(g.members.begin(), g.members.end(), [&](int64_t a, int64_t b) {
      if (bp[a].baseline != bp[b].baseline) return bp[a].baseline < bp[b].baseline;
      return pulse_stronger(a, b);
    });
    for (size_t k = 0; k < g.members.size(); ++k) {
      const BaselinePulse& p = bp[g.members[k]];
      if (k > 0 && p.baseline == bp[g.members[k - 1]].baseline) continue;
      if (rows < capacity) fill_row(out[rows], p, candidates[p.rep], int32_t(pulses));
      ++rows;
    }
    ++pulses;
  }
  *n_rows = rows;
  *n_pulses = pulses;
  if (rows > capacity)
    return fail(FRINGE_E_CAPACITY, "fringe_match: %lld rows, capacity %lld", (long long)rows,
                (long long)capacity);
  return FRINGE_OK;
}

int fringe_localize(const double* tau, const double* dtau_dra, const double* dtau_ddec,
                    int32_t n, double* sol, double* rms, double* loo, double* loo_rms) {
  if (!tau || !dtau_dra || !dtau_ddec || !sol || !rms)
    return fail(FRINGE_E_INVALID, "fringe_localize: null pointer");
  if (n < 2) return fail(FRINGE_E_INVALID, "fringe_localize: %d baselines, need >= 2", n);
  if (!finite_all(tau, n) || !finite_all(dtau_dra, n) || !finite_all(dtau_ddec, n))
    return fail(FRINGE_E_INVALID, "fringe_localize: non-finite input");
  if (!lsq2(tau, dtau_dra, dtau_ddec, n, -1, sol, rms))
    return fail(FRINGE_E_INVALID, "fringe_localize: the partials do not fix both offsets");
  if (loo && loo_rms && n >= 3) {
    for (int32_t i = 0; i < n; ++i) {
      if (!lsq2(tau, dtau_dra, dtau_ddec, n, i, loo + 2 * i, loo_rms + i)) {
        loo[2 * i] = loo[2 * i + 1] = NAN;
        loo_rms[i] = NAN;
      }
    }
  }
  return FRINGE_OK;
}

int fringe_delay_partials(const double* b_xyz, int32_t n, double gast, double ra, double dec,
                          double* dtau_dra, double* dtau_ddec) {
  if (n < 0 || (n > 0 && (!b_xyz || !dtau_dra || !dtau_ddec)))
    return fail(FRINGE_E_INVALID, "fringe_delay_partials: null pointer or n < 0");
  const double c = 299792458.0;
  double h = gast - ra;
  double cd = std::cos(dec), sd = std::sin(dec), ch = std::cos(h), sh = std::sin(h);
  // derivatives of s = (cos dec cos h, -cos dec sin h, sin dec), dh/dra = -1
  const double sa[3] = {cd * sh, cd * ch, 0.0};
  const double sdd[3] = {-sd * ch, sd * sh, cd};
  for (int32_t i = 0; i < n; ++i) {
    const double* b = b_xyz + 3 * int64_t(i);
    dtau_dra[i] = -(b[0] * sa[0] + b[1] * sa[1] + b[2] * sa[2]) / c;
    dtau_ddec[i] = -(b[0] * sdd[0] + b[1] * sdd[1] + b[2] * sdd[2]) / c;
  }
  return FRINGE_OK;
}

}  // extern "C"
