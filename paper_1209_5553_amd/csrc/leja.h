// Device Newton-Leja evaluation: launchers (leja.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kLejaRing = 16;       // terms whose block partials are kept
#ifndef EREM_LEJA_TILE_ROWS
#define EREM_LEJA_TILE_ROWS 8
#endif
constexpr int kLejaTileRows = EREM_LEJA_TILE_ROWS;  // rows of the multi-term tile (64 wide)
#ifndef EREM_LEJA_THREAD_ROWS
#define EREM_LEJA_THREAD_ROWS 8
#endif
constexpr int kLejaThreadRows = EREM_LEJA_THREAD_ROWS;  // thread rows of its block (64 wide)
constexpr int kCheckThreads = 1024;  // workgroup of the stop-test kernel
constexpr int kCheckEvery = 4;      // terms between stop tests

int leja_num_blocks(const Dims& d);

hipError_t launch_leja_reset(LejaState* st, int nslots, int nterms, hipStream_t s);
template <class V>
hipError_t launch_leja_init(const Dims& d, const LejaCoef* cf, const double* v, V* q0, V* p,
                            double* part, hipStream_t s);
template <class V>
hipError_t launch_leja_term(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout,
                            V* p, const LejaState* st, double* part, int k, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Terms k .. k + nterms - 1 in one launch (2D grids only, nterms 2 or 4):
// the last q to qout, p updated, every term's partial sums in its ring slot.
template <class V>
hipError_t launch_leja_terms(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout,
                             V* p, const LejaState* st, double* part, int k, int nterms, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_leja_check(const Dims& d, const LejaCoef* cf, LejaState* st, const double* part,
                             int k1, int k2, hipStream_t s);
// u = (first ? 0 : u) + delta p (+ zt when zt is not null)
template <class V>
hipError_t launch_substep_update(const Dims& d, double* u, const V* p, double delta, int first,
                                 hipStream_t s, const double* zt = nullptr);
hipError_t launch_cast_f32(const double* a, float* b, long long n, hipStream_t s);

// Coefficients of one Newton-Leja phi1 evaluation formed on the device from
// the assembly's reduction slots, so that the evaluation can be enqueued
// before the host has read the interval.  The kernel folds the slots into
// the Gershgorin interval [alpha, beta] and the largest |T|, forms
// scal = tol_a + tol_r max|T|, and, when the interval is finite and not
// degenerate and its substep count ceil(h (beta - alpha) / rho) (at least 1,
// at most smax) equals the count s the evaluation was enqueued with, fills
// cf for substeps of delta = h / s: the divided differences of
// phi1(delta (c + gamma xi)) (Sec. 4.2; the augmented bidiagonal
// exponential by Taylor scaling and squaring, as on the host), the shifts
// c / gamma + xi_{k-1} and the stop-test factors |delta d_k| / (sqrt(N) scal).
// Otherwise it marks the s stop states as stopped, so that the evaluation's
// term launches return at entry, and the host, which reads the same slots
// afterwards, evaluates again with the interval it has read.
struct LejaCoefArgs {
  const AsmReduce* red;
  int n;            // coefficients d_0 .. d_{n-1}, 1 <= n <= kCoefMaxN
  int s, smax;      // substeps enqueued; cap of the substep count
  double h, rho;    // step; widest substep interval (rho <= 0: one substep)
  double tol_a, tol_r, thresh, rootN;
  const double* xi;  // device copy of the Leja points (n values)
  DdCache* cache;
  LejaCoef* cf;
  LejaState* st;
};
constexpr int kCoefThreads = 256;
// Most coefficients the kernel forms: the augmented matrix (order n + 1 <=
// 32) and its square stay in LDS.  Past that its dependent phases (20 Taylor
// steps and up to 8 squarings) take longer than the host round trip they
// replace.
constexpr int kCoefMaxN = 31;
hipError_t launch_leja_coef(const LejaCoefArgs& a, hipStream_t s);

}  // namespace erem
