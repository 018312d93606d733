// Host driver for tests/test_match_sanitized.py: exercises the candidate
// consumers of libfringe (fringe_match, fringe_localize,
// fringe_delay_partials) on seeded random inputs, built together with their
// source under AddressSanitizer and UndefinedBehaviorSanitizer, and checks
// the documented invariants of their outputs.  Prints "ok" and exits 0.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "fringe_match.h"

namespace fringe {
std::string g_msg;
void set_last_error(const char* msg) { g_msg = msg; }
}  // namespace fringe

#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                         \
    }                                                                       \
  } while (0)

static std::vector<fringe_candidate> random_list(std::mt19937_64& rng, int n) {
  std::vector<fringe_candidate> v(static_cast<size_t>(n));
  const int lens[6] = {1, 2, 4, 8, 16, 32};
  for (auto& c : v) {
    c = fringe_candidate{};
    c.scan = int32_t(rng() % 3);
    c.baseline = int32_t(rng() % 12);
    c.window_ap = lens[rng() % 6];
    const int s = c.window_ap > 1 ? c.window_ap / 2 : 1;
    c.t_start = int32_t((rng() % 400) / s * s);
    c.snr = float(4.5 + 0.25 * double(rng() % 40));
    c.amp = c.snr * 3.0f;
    c.delay_s = 1e-9 * double(rng() % 100);
  }
  return v;
}

int main() {
  std::mt19937_64 rng(12345);
  for (int it = 0; it < 200; ++it) {
    const int n = int(rng() % 600);
    std::vector<fringe_candidate> c = random_list(rng, n);
    fringe_match_params prm{int32_t(1 + rng() % 3), int32_t(1 + rng() % 6)};
    int64_t rows = -1, pulses = -1;
    int rc = fringe_match(n ? c.data() : nullptr, n, &prm, nullptr, 0, &rows, &pulses);
    CHECK(rc == FRINGE_OK || rc == FRINGE_E_CAPACITY);
    CHECK(rows >= 0 && pulses >= 0 && pulses <= rows);
    std::vector<fringe_pulse> out(size_t(rows) + 1);
    rc = fringe_match(n ? c.data() : nullptr, n, &prm, out.data(), rows, &rows, &pulses);
    CHECK(rc == FRINGE_OK);
    // invariants: (pulse, baseline) strictly increasing; every pulse has at
    // least min_baselines rows; every row's window lies in its span and the
    // span's pulse has enough distinct lengths
    std::vector<int> per_pulse(size_t(pulses), 0);
    for (int64_t r = 0; r < rows; ++r) {
      const fringe_pulse& p = out[size_t(r)];
      CHECK(p.pulse >= 0 && p.pulse < pulses);
      if (r > 0) {
        const fringe_pulse& q = out[size_t(r - 1)];
        CHECK(q.pulse < p.pulse || (q.pulse == p.pulse && q.baseline < p.baseline));
        CHECK(q.scan <= p.scan);
      }
      CHECK(p.t_lo <= p.t_start && p.t_start + p.window_ap <= p.t_hi);
      CHECK(p.n_lengths >= prm.min_windows && p.n_windows >= p.n_lengths);
      per_pulse[size_t(p.pulse)]++;
    }
    for (int k : per_pulse) CHECK(k >= prm.min_baselines);
    // a too-small buffer: the first rows, the exact counts, and an error
    if (rows > 1) {
      std::vector<fringe_pulse> small(1);
      int64_t r2 = 0, p2 = 0;
      CHECK(fringe_match(c.data(), n, &prm, small.data(), 1, &r2, &p2) == FRINGE_E_CAPACITY);
      CHECK(r2 == rows && p2 == pulses && small[0].pulse == out[0].pulse &&
            small[0].baseline == out[0].baseline);
    }
  }
  // invalid inputs are rejected
  {
    std::vector<fringe_candidate> c(1);
    c[0] = fringe_candidate{};
    c[0].window_ap = 0;
    fringe_match_params prm{2, 5};
    int64_t rows, pulses;
    CHECK(fringe_match(c.data(), 1, &prm, nullptr, 0, &rows, &pulses) == FRINGE_E_INVALID);
    c[0].window_ap = 4;
    c[0].t_start = INT32_MAX - 1;
    CHECK(fringe_match(c.data(), 1, &prm, nullptr, 0, &rows, &pulses) == FRINGE_E_INVALID);
    CHECK(fringe_match(c.data(), -1, &prm, nullptr, 0, &rows, &pulses) == FRINGE_E_INVALID);
    CHECK(fringe_match(c.data(), 1, nullptr, nullptr, 0, &rows, &pulses) == FRINGE_E_INVALID);
  }
  // localization: exact recovery, leave-one-out rows, degenerate subsets
  std::normal_distribution<double> g(0.0, 1e-4);
  for (int it = 0; it < 200; ++it) {
    const int n = 2 + int(rng() % 40);
    std::vector<double> a(static_cast<size_t>(n)), d(static_cast<size_t>(n)), tau(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
      a[size_t(i)] = g(rng);
      d[size_t(i)] = g(rng);
      tau[size_t(i)] = 2e-6 * a[size_t(i)] - 1e-6 * d[size_t(i)];
    }
    double sol[2], rms;
    std::vector<double> loo(static_cast<size_t>(2 * n)), loo_rms(static_cast<size_t>(n));
    CHECK(fringe_localize(tau.data(), a.data(), d.data(), n, sol, &rms, loo.data(),
                          loo_rms.data()) == FRINGE_OK);
    CHECK(std::fabs(sol[0] - 2e-6) < 1e-12 && std::fabs(sol[1] + 1e-6) < 1e-12);
    if (n >= 3)
      for (int i = 0; i < n; ++i)
        CHECK(std::isnan(loo[size_t(2 * i)]) || std::fabs(loo[size_t(2 * i)] - 2e-6) < 1e-9);
  }
  {
    double a[3] = {1e-4, 2e-4, 3e-4}, d[3] = {2e-4, 4e-4, 6e-4}, tau[3] = {0, 0, 0};
    double sol[2], rms;
    CHECK(fringe_localize(tau, a, d, 3, sol, &rms, nullptr, nullptr) == FRINGE_E_INVALID);
    CHECK(fringe_localize(tau, a, d, 1, sol, &rms, nullptr, nullptr) == FRINGE_E_INVALID);
  }
  {
    std::vector<double> b(3 * 45), da(45), dd(45);
    for (auto& x : b) x = g(rng) * 3e10;
    CHECK(fringe_delay_partials(b.data(), 45, 1.0, 0.5, 0.3, da.data(), dd.data()) == FRINGE_OK);
    for (int i = 0; i < 45; ++i) CHECK(std::isfinite(da[size_t(i)]) && std::isfinite(dd[size_t(i)]));
    CHECK(fringe_delay_partials(nullptr, 0, 0, 0, 0, nullptr, nullptr) == FRINGE_OK);
    CHECK(fringe_delay_partials(b.data(), -1, 0, 0, 0, da.data(), dd.data()) == FRINGE_E_INVALID);
  }
  std::printf("ok\n");
  return 0;
}
