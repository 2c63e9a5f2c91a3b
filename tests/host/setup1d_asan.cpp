// Host-only driver of the univariate setup (knot checks, Gauss rule, B-spline
// tables, M, K and the generalised eigendecomposition) for a build with the
// address and undefined-behaviour sanitizers: degrees 1..6, uniform,
// jittered and repeated-knot vectors, sizes that take the threaded
// eigenvector update, and the error paths.  Exit status 0 when every result
// is finite and U^T M U = I holds to 1e-9; the sanitizers abort on the first
// memory or UB error.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

namespace igafd {
void set_error(const std::string&) {}
}  // namespace igafd

static std::vector<double> open_knots(int E, int p, double jitter, unsigned seed, int mult_mid) {
  std::vector<double> k(p + 1, 0.0), h(E);
  unsigned s = seed;
  double tot = 0.0;
  for (int e = 0; e < E; ++e) {
    s = s * 1664525u + 1013904223u;
    h[e] = 1.0 + jitter * ((s >> 8) / 16777216.0 * 2.0 - 1.0);
    tot += h[e];
  }
  double acc = 0.0;
  for (int e = 0; e + 1 < E; ++e) {
    acc += h[e];
    const int m = (mult_mid > 1 && e == E / 2) ? mult_mid : 1;
    for (int r = 0; r < m; ++r) k.push_back(acc / tot);
  }
  for (int r = 0; r <= p; ++r) k.push_back(1.0);
  return k;
}

static bool check(const igafd::Dir1D& d) {
  const int n = d.n;
  std::vector<double> MU((size_t)n * n, 0.0);  // M U
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double m = d.M[(size_t)i * n + j];
      if (m != 0.0)
        for (int b = 0; b < n; ++b) MU[(size_t)i * n + b] += m * d.U[(size_t)j * n + b];
    }
  double worst = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double s = 0.0;  // (U^T M U)_ab
      for (int i = 0; i < n; ++i) s += d.U[(size_t)i * n + a] * MU[(size_t)i * n + b];
      const double e = std::fabs(s - (a == b ? 1.0 : 0.0));
      if (!(e <= worst)) worst = e;
    }
  for (double v : d.lam)
    if (!std::isfinite(v) || v <= 0.0) return false;
  return worst <= 1e-9;
}

int main() {
  int bad = 0;
  for (int p = 1; p <= 6; ++p)
    for (int variant = 0; variant < 3; ++variant) {
      const int E = variant == 2 ? 300 : 17 + 3 * p;
      const auto k = open_knots(E, p, variant == 0 ? 0.0 : 0.3, 7u + p, variant == 1 ? p : 1);
      igafd::Dir1D d;
      const igafd_status st = igafd::build_direction(p, p + 1, (int)k.size(), k.data(), &d);
      if (st != IGAFD_OK || !check(d)) {
        std::printf("FAIL p=%d variant=%d status=%d\n", p, variant, (int)st);
        ++bad;
      }
    }
  // error paths: too short, not open, decreasing, multiplicity above p
  const std::vector<std::vector<double>> wrong = {
      {0, 0, 1, 1}, {0.1, 0, 0, 0.5, 1, 1, 1}, {0, 0, 0, 0.7, 0.3, 1, 1, 1}, {0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1}};
  for (const auto& k : wrong) {
    igafd::Dir1D d;
    if (igafd::build_direction(2, 3, (int)k.size(), k.data(), &d) == IGAFD_OK) {
      std::printf("FAIL: invalid knot vector accepted\n");
      ++bad;
    }
  }
  std::printf("%s\n", bad ? "FAILED" : "OK");
  return bad ? 1 : 0;
}
