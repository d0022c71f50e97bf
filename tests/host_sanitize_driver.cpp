// Exercises the library's host numerics (Leja points, divided differences of
// phi_1 and phi_2, the dense exponential) over a spread of arguments, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  Exits non-zero on a failed check.
#include <cmath>
#include <cstdio>
#include <vector>

#include "host_numerics.h"

using namespace erem;

static int failures = 0;

static void check(bool ok, const char* what, double a, double b) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s (%.17g, %.17g)\n", what, a, b);
    ++failures;
  }
}

int main() {
  std::vector<double> xi;
  check(!leja_points(-1, xi), "leja_points(-1) refused", -1, 0);
  check(!leja_points(kMaxLeja + 1, xi), "leja_points(max + 1) refused", kMaxLeja + 1, 0);
  check(leja_points(0, xi) && xi.empty(), "leja_points(0) empty", 0, xi.size());
  for (int n : {1, 2, 7, 65, 258}) {
    check(leja_points(n, xi) && static_cast<int>(xi.size()) == n, "leja_points size", n, xi.size());
    for (double x : xi) check(x >= -2.0 && x <= 2.0, "Leja point in [-2, 2]", x, n);
  }
  leja_points(258, xi);
  for (int ell = 1; ell <= 2; ++ell)
    for (double hc : {-200.0, -30.0, -1.0, -1e-9, 0.0})
      for (double hg : {1e-6, 0.5, 8.0, 40.0})
        for (int n : {1, 2, 9, 65, 258}) {
          std::vector<double> out(n), out_ws(n), work(divided_differences_work(ell, n));
          phi_divided_differences(ell, hc, hg, xi.data(), n, out.data());
          phi_divided_differences_ws(ell, hc, hg, xi.data(), n, out_ws.data(), work.data());
          for (int k = 0; k < n; ++k) {
            check(std::isfinite(out[k]), "finite divided difference", hc, hg);
            check(out[k] == out_ws[k], "workspace variant equal", out[k], out_ws[k]);
          }
          // the zeroth divided difference is phi_ell at the first node
          const double z = hc + hg * xi[0];
          const double ref = ell == 1 ? (z == 0.0 ? 1.0 : std::expm1(z) / z) : phi2_scalar(z);
          check(std::fabs(out[0] - ref) <= 1e-13 * std::fabs(ref) + 1e-300, "d_0 = phi(z_0)", out[0], ref);
        }
  std::vector<double> d1(40), d1b(40);
  phi1_divided_differences(-5.0, 2.0, xi.data(), 40, d1.data());
  phi_divided_differences(1, -5.0, 2.0, xi.data(), 40, d1b.data());
  for (int k = 0; k < 40; ++k) check(d1[k] == d1b[k], "phi1 entry point", d1[k], d1b[k]);
  for (double z : {-700.0, -20.0, -1.0, -1e-3, 0.0, 1e-3, 0.5, 3.0}) {
    const double p2 = phi2_scalar(z);
    check(std::isfinite(p2) && p2 > 0.0, "phi2 positive", z, p2);
  }
  for (int n : {1, 2, 5, 12}) {
    std::vector<double> A(n * n), E(n * n);
    for (int i = 0; i < n * n; ++i) A[i] = std::sin(1.0 + i) * (i % (n + 1) == 0 ? -3.0 : 0.4);
    dense_expm(n, A.data(), E.data());
    for (double e : E) check(std::isfinite(e), "finite exponential", n, e);
    if (n == 1) check(std::fabs(E[0] - std::exp(A[0])) <= 1e-14 * std::exp(A[0]), "exp of 1 x 1", E[0], std::exp(A[0]));
  }
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("host numerics: all checks passed\n");
  return failures ? 1 : 0;
}
