// Host-side small dense numerics of the EREM library (no device code).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace erem {

// First n real Leja points of [-2, 2] (Sec. 4.2, Eq. lejaa).  Thread-safe,
// memoised; n <= kMaxLeja.
constexpr int kMaxLeja = 1025;
bool leja_points(int n, std::vector<double>& out);

// Divided differences of g(xi) = phi1(hc + hg xi) at xi[0..n-1] (Sec. 4.2):
// first column of phi1(hc I + hg L), L lower bidiagonal (diag xi, subdiag 1),
// read off exp([[0, 0], [e_1, hc I + hg L]]).
void phi1_divided_differences(double hc, double hg, const double* xi, int n, double* out);

// The same for g(xi) = phi_ell(hc + hg xi), ell = 1 or 2 (phi_2 of the
// non-autonomous step, Sec. 3.2.3): first column of phi_ell(hc I + hg L),
// read off the exponential of the bidiagonal matrix augmented by ell rows.
void phi_divided_differences(int ell, double hc, double hg, const double* xi, int n, double* out);
// The same on a caller's workspace of divided_differences_work(ell, n)
// doubles (no allocation).
size_t divided_differences_work(int ell, int n);
void phi_divided_differences_ws(int ell, double hc, double hg, const double* xi, int n, double* out, double* work);

// phi2(z) = (e^z - 1 - z) / z^2 (Sec. 3.2.3), by its series for |z| < 1.
double phi2_scalar(double z);

// Dense exponential of an n x n row-major matrix by Taylor scaling-and-squaring.
void dense_expm(int n, const double* A, double* E);

}  // namespace erem
