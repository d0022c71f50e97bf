// Host-side numerics: real Leja points, Newton divided differences of phi1,
// small dense exponential.  Plain C++17, FP64.
#include "host_numerics.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>

namespace erem {

namespace {

std::mutex g_leja_mutex;
std::vector<double> g_leja;  // memoised sequence

// log prod_k |x - p_k|
double log_node_poly(double x, const std::vector<double>& p) {
  double s = 0.0;
  for (double pk : p) s += std::log(std::fabs(x - pk));
  return s;
}

// Maximiser of log prod |x - p_k| on the open gap (a, b) between adjacent
// nodes.  The function is strictly concave there (second derivative
// -sum 1/(x - p_k)^2), its derivative falls from +inf to -inf, so a
// bracketed Newton iteration on the derivative converges to the unique root.
double gap_argmax(double a, double b, const std::vector<double>& p) {
  double lo = a, hi = b, x = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double g = 0.0, gp = 0.0;
    for (double pk : p) {
      const double t = 1.0 / (x - pk);
      g += t;
      gp -= t * t;
    }
    if (g > 0.0) lo = x; else hi = x;
    double xn = x - g / gp;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const double tol = 4.0 * std::numeric_limits<double>::epsilon() * std::max(1.0, std::fabs(x));
    if (std::fabs(xn - x) <= tol || hi - lo <= tol) return xn;
    x = xn;
  }
  return x;
}

void extend_leja(int n) {
  if (g_leja.empty()) g_leja.push_back(2.0);          // xi_0 = beta (right end)
  if (n > 1 && g_leja.size() == 1) g_leja.push_back(-2.0);  // farthest point from 2
  while (static_cast<int>(g_leja.size()) < n) {
    std::vector<double> s = g_leja;
    std::sort(s.begin(), s.end());
    double best_x = 0.0, best_v = -std::numeric_limits<double>::infinity();
    for (size_t k = 0; k + 1 < s.size(); ++k) {
      const double x = gap_argmax(s[k], s[k + 1], g_leja);
      const double v = log_node_poly(x, g_leja);
      // Gaps are scanned left to right; a value equal to the best within
      // rounding (a tie, e.g. the symmetric pair +-2/sqrt(3)) takes the
      // larger point.
      const double tie = std::isfinite(best_v) ? 1e-12 * std::max(1.0, std::fabs(best_v)) : 0.0;
      if (v > best_v + tie) {
        best_v = v;
        best_x = x;
      } else if (std::fabs(v - best_v) <= tie && x > best_x) {
        best_v = std::max(v, best_v);
        best_x = x;
      }
    }
    g_leja.push_back(best_x);
  }
}

// Lower-triangular (row-major, n x n) product C = A * B.
// Row i of C is the combination of rows k <= i of B with weights A[i][k], so
// the inner loop runs along contiguous rows (it vectorises).
void tri_mul(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i) {
    double* c = C + static_cast<size_t>(i) * n;
    for (int j = 0; j < n; ++j) c[j] = 0.0;
    for (int k = 0; k <= i; ++k) {
      const double a = A[static_cast<size_t>(i) * n + k];
      const double* b = B + static_cast<size_t>(k) * n;
      for (int j = 0; j <= k; ++j) c[j] += a * b[j];
    }
  }
}

}  // namespace

bool leja_points(int n, std::vector<double>& out) {
  if (n < 0 || n > kMaxLeja) return false;
  std::lock_guard<std::mutex> lock(g_leja_mutex);
  if (static_cast<int>(g_leja.size()) < n) extend_leja(n);
  out.assign(g_leja.begin(), g_leja.begin() + n);
  return true;
}

size_t divided_differences_work(int ell, int n) {
  const size_t M = static_cast<size_t>(n) + ell;
  return 2 * M + 2 * M * M;
}

void phi_divided_differences_ws(int ell, double hc, double hg, const double* xi, int n, double* out, double* work) {
  // Augmented lower-bidiagonal matrix of order M = n + ell:
  //   diag = (0 (ell times), hc + hg xi_0, ..., hc + hg xi_{n-1}),
  //   subdiag = (1 (ell times), hg, ..., hg).
  // Its exponential's first column is (1, 1, .., 1/(ell-1)!, phi_ell(L) e_1)
  // with L = hc I + hg Lhat: the first ell unknowns of y' = A y, y(0) = e_1,
  // are s^j / j!, which feed the last block as the forcing s^(ell-1)/(ell-1)!
  // e_1, whose response at s = 1 is phi_ell(L) e_1 by the integral
  // definition of phi_ell.  phi_ell(L) e_1 holds the divided differences of
  // phi_ell(hc + hg xi).
  const int M = n + ell;
  double* dg = work;
  double* sd = work + M;
  for (int k = 0; k < M; ++k) dg[k] = sd[k] = 0.0;
  for (int k = 0; k < n; ++k) dg[k + ell] = hc + hg * xi[k];
  for (int k = 1; k <= ell && k < M; ++k) sd[k] = 1.0;  // A[k][k-1]
  for (int k = ell + 1; k < M; ++k) sd[k] = hg;
  double nrm = 0.0;                        // 1-norm: max column sum
  for (int j = 0; j < M; ++j) {
    const double c = std::fabs(dg[j]) + (j + 1 < M ? std::fabs(sd[j + 1]) : 0.0);
    nrm = std::max(nrm, c);
  }
  int s = 0;
  if (nrm > 0.5) {
    // s = ceil(log2(nrm / 0.5)) exactly: nrm / 0.5 = f 2^e with f in [1/2, 1)
    int e = 0;
    const double f = std::frexp(nrm / 0.5, &e);
    s = f == 0.5 ? e - 1 : e;
  }
  const double scale = std::ldexp(1.0, -s);
  for (int k = 0; k < M; ++k) { dg[k] *= scale; sd[k] *= scale; }

  // Taylor series of degree 20 by Horner's rule, E <- I + X E / k, where X is
  // bidiagonal so X E costs O(M^2).
  const int degree = 20;
  const size_t MM = static_cast<size_t>(M) * M;
  double* E = work + 2 * M;
  double* T = E + MM;
  for (size_t i = 0; i < MM; ++i) E[i] = T[i] = 0.0;
  for (int i = 0; i < M; ++i) E[i * M + i] = 1.0;
  for (int k = degree; k >= 1; --k) {
    const double inv = 1.0 / k;
    for (int i = 0; i < M; ++i) {
      double* t = T + static_cast<size_t>(i) * M;
      const double* e = E + static_cast<size_t>(i) * M;
      const double di = dg[i];
      if (i == 0) {
        t[0] = di * e[0] * inv;
      } else {
        const double* ep = e - M;  // row i - 1 (zero at column i)
        const double si = sd[i];
        for (int j = 0; j <= i; ++j) t[j] = (di * e[j] + si * ep[j]) * inv;
      }
      t[i] += 1.0;
    }
    std::swap(E, T);
  }
  // Squaring: the last square only needs the first column.
  for (int q = 0; q < s; ++q) {
    if (q + 1 == s) {
      for (int i = 0; i < M; ++i) {
        double acc = 0.0;
        for (int k = 0; k <= i; ++k) acc += E[i * M + k] * E[k * M + 0];
        T[i * M + 0] = acc;
      }
      for (int i = 0; i < M; ++i) E[i * M + 0] = T[i * M + 0];
    } else {
      tri_mul(M, E, E, T);
      std::swap(E, T);
    }
  }
  for (int k = 0; k < n; ++k) out[k] = E[(k + ell) * M + 0];
}

void phi_divided_differences(int ell, double hc, double hg, const double* xi, int n, double* out) {
  std::vector<double> work(divided_differences_work(ell, n));
  phi_divided_differences_ws(ell, hc, hg, xi, n, out, work.data());
}

void phi1_divided_differences(double hc, double hg, const double* xi, int n, double* out) {
  phi_divided_differences(1, hc, hg, xi, n, out);
}

double phi2_scalar(double z) {
  if (std::fabs(z) < 1.0) {
    // sum_{k>=0} z^k / (k+2)!: terms fall by |z| / (k+3) each
    double acc = 0.0, term = 0.5;
    for (int k = 0; k < 25; ++k) {
      acc += term;
      term *= z / (k + 3);
    }
    return acc;
  }
  return (std::expm1(z) - z) / (z * z);
}

void dense_expm(int n, const double* A, double* E) {
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += std::fabs(A[i * n + j]);
    nrm = std::max(nrm, c);
  }
  int s = 0;
  if (nrm > 0.5) s = static_cast<int>(std::ceil(std::log2(nrm / 0.5)));
  const double scale = std::ldexp(1.0, -s);
  std::vector<double> X(static_cast<size_t>(n) * n), P(X.size()), Q(X.size());
  for (size_t i = 0; i < X.size(); ++i) X[i] = A[i] * scale;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) P[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int k = 20; k >= 1; --k) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int l = 0; l < n; ++l) acc += X[i * n + l] * P[l * n + j];
        Q[i * n + j] = acc / k + (i == j ? 1.0 : 0.0);
      }
    std::swap(P, Q);
  }
  for (int q = 0; q < s; ++q) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int l = 0; l < n; ++l) acc += P[i * n + l] * P[l * n + j];
        Q[i * n + j] = acc;
      }
    std::swap(P, Q);
  }
  for (size_t i = 0; i < P.size(); ++i) E[i] = P[i];
}

}  // namespace erem
