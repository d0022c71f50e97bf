// Shifted linear solves (sigma I - J) x = b for the Rosenbrock-type and
// theta-Euler steps (Sec. 3.2.1-3.2.3): BiCGSTAB with Jacobi (diagonal)
// right preconditioning on the stencil of J, scalars resident on the device.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

// Scalars of the BiCGSTAB iteration.  Its inner products are kept as
// partial sums, one per 64 x 4 cell band (the blocks of cell_grid), in a ring
// of four iterations; every consumer adds a product's partials in band order
// (wave_part_sum), so results do not depend on the order in which blocks
// ran.  The arrays live in one allocation of bicg_parts_words(nb) doubles.
struct BicgState {
  int done;       // 1 once converged (or broken down)
  int it_done;    // iteration at which the test passed
  int breakdown;  // rho = 0, omega = 0 or a non-finite scalar
  int nb;         // partial slots per inner product
  double tol2;    // rtol^2
  double* bb_sl;  // [nb] ||b||^2
  double* rho;    // [4][nb] (rhat, r_it)
  double* rr;     // [4][nb] (r_it, r_it)
  double* rv;     // [4][nb] (rhat, v_it)
  double* ts;     // [4][nb] (t_it, s_it)
  double* tt;     // [4][nb] (t_it, t_it)
};
inline size_t bicg_parts_words(int nb) { return static_cast<size_t>(21) * nb; }
inline void bicg_bind_parts(BicgState* st, double* parts, int nb) {
  st->nb = nb;
  st->bb_sl = parts;
  st->rho = parts + nb;
  st->rr = parts + 5 * static_cast<size_t>(nb);
  st->rv = parts + 9 * static_cast<size_t>(nb);
  st->ts = parts + 13 * static_cast<size_t>(nb);
  st->tt = parts + 17 * static_cast<size_t>(nb);
}

// Vectors of one solve (N values each, device).
struct BicgBufs {
  double *r, *rhat, *p[2], *v[2], *s, *t;
};

hipError_t launch_bicg_reset(BicgState* st, double tol2, hipStream_t s);
// r = rhat = b, x = 0, ||b||^2, (rhat, r_0), (r_0, r_0)
hipError_t launch_bicg_start(const Dims& d, const double* b, double* x, const BicgBufs& B, BicgState* st,
                             hipStream_t s);
// One iteration `it` (three kernels); with events, kernel-level timing of
// each (e[0..5]).
hipError_t launch_bicg_iteration(const Dims& d, double sigma, const double* coef, double* x,
                                 const BicgBufs& B, BicgState* st, int it, hipStream_t s,
                                 const hipEvent_t* e = nullptr);
// out = sum_{m < n} w[m] in[m] (elementwise; out may alias in[0])
struct LinComb {
  const double* in[4];
  double w[4];
  int n;
};
hipError_t launch_lincomb(const Dims& d, double* out, const LinComb& lc, hipStream_t s);

}  // namespace erem
