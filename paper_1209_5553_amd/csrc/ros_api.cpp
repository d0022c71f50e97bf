// C ABI of the comparison schemes (Sec. 3.2.1-3.2.3): the shifted solve
// (sigma I - J) x = b, the Rosenbrock-type steps ROSM(1), ROSM(1/2),
// ROS2(1) and ROS3p (Eq. ROS, Eq. ROSMh, Tables ros2 and ros3) and the
// theta-Euler step with Newton's method (Eq. temscheme).  Every linear
// system goes through one BiCGSTAB (rosenbrock.hip).
#include "erem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "ctx.h"
#include "device.h"
#include "rosenbrock.h"

using namespace erem;
using namespace erem_internal;

namespace {

// Stage coefficients of Eq. ROSMh (only j < i is used; the tables' c_ii =
// 1/gamma belong to the diagonal and do not enter the stage equations).
struct RosScheme {
  int stages;
  double gamma;
  double a[3][3];
  double c[3][3];
  double b[3];
  double gam[3];    // gamma_i of the D_t f term
  double alpha[3];  // stage times t_n + alpha_i h
};

// ROSM(gamma) is the one-stage method (I/(tau gamma) - J) k = f,
// y+ = y + k / gamma (Eq. ROS).
// ROSM(gamma) with a time-dependent right-hand side carries gamma tau D_t f
// (Eq. ROSf).
const RosScheme kSchemes[4] = {
    {1, 1.0, {{0.0}}, {{0.0}}, {1.0}, {1.0}, {0.0}},
    {1, 0.5, {{0.0}}, {{0.0}}, {2.0}, {0.5}, {0.0}},
    // Table ros2: ROS2(1)
    {2, 1.707106781186547,
     {{0.0}, {5.857864376269050e-01}},
     {{0.0}, {1.171572875253810e+00}},
     {8.786796564403575e-01, 2.928932188134525e-01},
     {1.707106781186547, -1.707106781186547},
     {0.0, 1.0}},
    // Table ros3: ROS3p
    {3, 7.886751345948129e-01,
     {{0.0}, {1.267949192431123}, {1.267949192431123, 0.0}},
     {{0.0}, {1.607695154586736}, {3.464101615137755, 1.732050807568877}},
     {2.0, 5.773502691896258e-01, 4.226497308103742e-01},
     {7.886751345948129e-01, -2.113248654051871e-01, -1.077350269189626},
     {0.0, 1.0, 1.0}},
};

// Boundary data of a non-autonomous Rosenbrock step: the boundary
// temperatures at the stage times t_n + alpha_i h and their rates at t_n.
struct StageBc {
  double Tl[3], Tr[3];
  double dTl, dTr;
};

int ensure_bicg(erem_ctx* c) {
  if (c->bicg) return EREM_OK;
  const size_t n = c->d.N;
  int rc = EREM_OK;
  double** v[] = {&c->bc_r, &c->bc_rhat, &c->bc_p0, &c->bc_p1, &c->bc_v0, &c->bc_v1, &c->bc_s, &c->bc_t,
                  &c->rs_k0, &c->rs_k1, &c->rs_k2, &c->rs_y, &c->rs_g, &c->rs_rhs};
  for (double** b : v) rc |= dev_alloc(c, b, n);
  rc |= dev_alloc(c, &c->rs_coef, n * ndir(c));
  const int nb = cell_bands(c->d);
  rc |= dev_alloc(c, &c->bicg_parts, bicg_parts_words(nb));
  rc |= dev_alloc(c, &c->bicg, 1);
  if (rc) return EREM_ENOMEM;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_bicg), sizeof(BicgState), hipHostMallocDefault) != hipSuccess)
    return fail(c, EREM_ENOMEM, "hipHostMalloc failed");
  // the state's pointers into the partial slots, set once
  BicgState init{};
  bicg_bind_parts(&init, c->bicg_parts, nb);
  HIP_TRY(c, hipMemcpy(c->bicg, &init, sizeof(BicgState), hipMemcpyHostToDevice));
  return EREM_OK;
}

BicgBufs bufs(erem_ctx* c) { return BicgBufs{c->bc_r, c->bc_rhat, {c->bc_p0, c->bc_p1}, {c->bc_v0, c->bc_v1}, c->bc_s, c->bc_t}; }

// (sigma I - J) x = b with the context's stencil, from x = 0, to
// ||r|| <= rtol ||b|| (recursive residual).  Iterations after convergence
// still launch and return at entry: the host polls after the previous
// solve's count + 1 iterations, then every four.
int bicg_solve(erem_ctx* c, double sigma, const double* b, double* x, double rtol, int max_iter, int* iters) {
  const Dims& d = c->d;
  const BicgBufs B = bufs(c);
  HIP_TRY(c, launch_bicg_reset(c->bicg, rtol * rtol, c->stream));
  HIP_TRY(c, launch_bicg_start(d, b, x, B, c->bicg, c->stream));
  const int first = c->bicg_last > 0 ? c->bicg_last + 1 : 8;
  const int chunk = 4;
  if (c->prof) {
    const int rc = ensure_events(c, 6 * static_cast<size_t>(std::max(first, chunk)));
    if (rc) return rc;
  }
  int it = 0;
  while (it < max_iter) {
    const int n = std::min(it == 0 ? first : chunk, max_iter - it);
    const int it0 = it;
    for (int j = 0; j < n; ++j, ++it) {
      const bool timed = c->prof && it % c->prof == 0;
      HIP_TRY(c, launch_bicg_iteration(d, sigma, c->coef, x, B, c->bicg, it, c->stream,
                                       timed ? &c->ev[6 * j] : nullptr));
    }
    HIP_TRY(c, hipMemcpyAsync(c->h_bicg, c->bicg, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const bool done = c->h_bicg->done != 0;
    const int last = done ? c->h_bicg->it_done : it;  // iterations that did work
    if (c->prof) {
      for (int j = 0; j < n; ++j) {
        const int k = it0 + j;
        if (k % c->prof != 0 || k >= last) continue;
        c->t_bicg += elapsed_ms(c->ev[6 * j], c->ev[6 * j + 1]) + elapsed_ms(c->ev[6 * j + 2], c->ev[6 * j + 3]) +
                     elapsed_ms(c->ev[6 * j + 4], c->ev[6 * j + 5]);
        c->n_bicg += 1;
      }
    }
    if (done) {
      if (c->h_bicg->breakdown) return fail(c, EREM_ENOCONV, "BiCGSTAB broke down");
      *iters = c->h_bicg->it_done;
      c->bicg_last = *iters;
      return EREM_OK;
    }
  }
  return fail(c, EREM_ENOCONV, "BiCGSTAB did not reach the tolerance within max_iter iterations");
}

int lincomb(erem_ctx* c, double* out, std::initializer_list<std::pair<const double*, double>> terms) {
  LinComb lc{};
  int n = 0;
  for (const auto& t : terms) {
    lc.in[n] = t.first;
    lc.w[n] = t.second;
    ++n;
  }
  lc.n = n;
  HIP_TRY(c, launch_lincomb(c->d, out, lc, c->stream));
  return EREM_OK;
}

int scheme_checks(erem_ctx* c, double h, const double* d_T, double rtol) {
  if (!d_T) return fail(c, EREM_EINVAL, "T is NULL");
  if (!(h > 0) || !std::isfinite(h)) return fail(c, EREM_EINVAL, "h must be > 0");
  if (!(rtol > 0) || !(rtol < 1)) return fail(c, EREM_EINVAL, "linear tolerance must be in (0, 1)");
  return EREM_OK;
}

int ros_step(erem_ctx* c, double h, int32_t scheme, double* d_T, double lin_rtol, erem_stats* stats,
             const StageBc* bc) {
  int rc = scheme_checks(c, h, d_T, lin_rtol);
  if (rc) return rc;
  if (scheme < EREM_ROSM_1 || scheme > EREM_ROS3P) return fail(c, EREM_EINVAL, "unknown Rosenbrock scheme");
  const RosScheme& S = kSchemes[scheme];
  if (bc) {
    for (int i = 0; i < S.stages; ++i)
      if (!std::isfinite(bc->Tl[i]) || !std::isfinite(bc->Tr[i]))
        return fail(c, EREM_EINVAL, "stage boundary temperatures must be finite");
    if (!std::isfinite(bc->dTl) || !std::isfinite(bc->dTr)) return fail(c, EREM_EINVAL, "rates must be finite");
  }
  rc = ensure_bicg(c);
  if (rc) return rc;
  if (bc && !c->gt) {
    rc = dev_alloc(c, &c->gt, c->d.N);
    if (!rc) rc = dev_alloc(c, &c->zt, c->d.N);
    if (rc) return EREM_ENOMEM;
  }
  if (bc) { c->ph.T_left = bc->Tl[0]; c->ph.T_right = bc->Tr[0]; }
  rc = erem_form_jacobian(c, d_T);  // J_n and G(T^n, t_n)
  if (rc) return rc;
  const Dims& d = c->d;
  // D_t f(T^n, t_n): the boundary vector with the rates, over V C
  if (bc) HIP_TRY(c, launch_time_rate(d, c->ph, c->poro, c->fx, d_T, bc->dTl, bc->dTr, c->gt, c->stream));
  const double sigma = 1.0 / (h * S.gamma);
  double* k[3] = {c->rs_k0, c->rs_k1, c->rs_k2};
  int total = 0;
  for (int i = 0; i < S.stages; ++i) {
    const double* rhs = c->F;
    const double wt = bc ? h * S.gam[i] : 0.0;  // weight of D_t f
    if (i == 0 && bc) {
      rc = lincomb(c, c->rs_rhs, {{c->F, 1.0}, {c->gt, wt}});
      if (rc) return rc;
      rhs = c->rs_rhs;
    } else if (i > 0) {
      // Y = T + sum_j a_ij k_j, then G(Y, t_n + alpha_i h) (the scratch
      // stencil keeps J_n)
      if (i == 1) rc = lincomb(c, c->rs_y, {{d_T, 1.0}, {k[0], S.a[1][0]}});
      else rc = lincomb(c, c->rs_y, {{d_T, 1.0}, {k[0], S.a[2][0]}, {k[1], S.a[2][1]}});
      if (rc) return rc;
      if (bc) { c->ph.T_left = bc->Tl[i]; c->ph.T_right = bc->Tr[i]; }
      HIP_TRY(c, launch_reset_reduce(c->red, c->stream));
      HIP_TRY(c, launch_assemble(d, c->ph, c->poro, c->fx, c->fy, c->fz, c->rs_y, c->rs_coef, c->rs_g, c->red,
                                 c->stream));
      // rhs = G(Y) - sum_j (c_ij / h) k_j (+ h gamma_i D_t f)
      if (i == 1) {
        if (bc) rc = lincomb(c, c->rs_rhs, {{c->rs_g, 1.0}, {k[0], -S.c[1][0] / h}, {c->gt, wt}});
        else rc = lincomb(c, c->rs_rhs, {{c->rs_g, 1.0}, {k[0], -S.c[1][0] / h}});
      } else {
        if (bc)
          rc = lincomb(c, c->rs_rhs, {{c->rs_g, 1.0}, {k[0], -S.c[2][0] / h}, {k[1], -S.c[2][1] / h}, {c->gt, wt}});
        else rc = lincomb(c, c->rs_rhs, {{c->rs_g, 1.0}, {k[0], -S.c[2][0] / h}, {k[1], -S.c[2][1] / h}});
      }
      if (rc) return rc;
      rhs = c->rs_rhs;
    }
    int it = 0;
    rc = bicg_solve(c, sigma, rhs, k[i], lin_rtol, 10000, &it);
    if (bc) { c->ph.T_left = bc->Tl[0]; c->ph.T_right = bc->Tr[0]; }
    if (rc) return rc;
    total += it;
  }
  if (S.stages == 1) rc = lincomb(c, d_T, {{d_T, 1.0}, {k[0], S.b[0]}});
  else if (S.stages == 2) rc = lincomb(c, d_T, {{d_T, 1.0}, {k[0], S.b[0]}, {k[1], S.b[1]}});
  else rc = lincomb(c, d_T, {{d_T, 1.0}, {k[0], S.b[0]}, {k[1], S.b[1]}, {k[2], S.b[2]}});
  if (rc) return rc;
  if (stats) {
    *stats = erem_stats{};
    stats->substeps = S.stages;
    stats->iterations = total;
  }
  return EREM_OK;
}

}  // namespace

extern "C" {

int erem_shifted_solve(erem_ctx* c, double sigma, const double* d_b, double* d_x, double rtol, int32_t max_iter,
                       erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  if (!c->jac_set) return fail(c, EREM_EINVAL, "erem_form_jacobian (or erem_set_jacobian) must come first");
  if (c->op_pressure) return fail(c, EREM_EINVAL, kHoldsPressure);
  if (!d_b || !d_x || d_b == d_x) return fail(c, EREM_EINVAL, "b and x must be distinct non-NULL");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(c, EREM_EINVAL, "sigma must be > 0");
  if (!(rtol > 0) || !(rtol < 1)) return fail(c, EREM_EINVAL, "rtol must be in (0, 1)");
  if (max_iter < 1) return fail(c, EREM_EINVAL, "max_iter must be >= 1");
  int rc = ensure_bicg(c);
  if (rc) return rc;
  int iters = 0;
  rc = bicg_solve(c, sigma, d_b, d_x, rtol, max_iter, &iters);
  if (stats) {
    *stats = erem_stats{};
    stats->iterations = iters;
  }
  return rc;
}

int erem_step_rosenbrock(erem_ctx* c, double h, int32_t scheme, double* d_T, double lin_rtol,
                         erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  return ros_step(c, h, scheme, d_T, lin_rtol, stats, nullptr);
}

int erem_step_rosenbrock_nonautonomous(erem_ctx* c, double h, int32_t scheme, const double* T_left_stage,
                                       const double* T_right_stage, double dT_left_dt, double dT_right_dt,
                                       double* d_T, double lin_rtol, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  if (!T_left_stage || !T_right_stage) return fail(c, EREM_EINVAL, "stage boundary arrays are NULL");
  if (scheme < EREM_ROSM_1 || scheme > EREM_ROS3P) return fail(c, EREM_EINVAL, "unknown Rosenbrock scheme");
  StageBc bc{};
  for (int i = 0; i < kSchemes[scheme].stages; ++i) {
    bc.Tl[i] = T_left_stage[i];
    bc.Tr[i] = T_right_stage[i];
  }
  bc.dTl = dT_left_dt;
  bc.dTr = dT_right_dt;
  return ros_step(c, h, scheme, d_T, lin_rtol, stats, &bc);
}

int erem_step_theta(erem_ctx* c, double h, double theta, double* d_T, double newton_rtol, double lin_rtol,
                    int32_t max_newton, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = scheme_checks(c, h, d_T, lin_rtol);
  if (rc) return rc;
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(c, EREM_EINVAL, "theta must be in [0, 1]");
  if (!(newton_rtol > 0) || max_newton < 1) return fail(c, EREM_EINVAL, "Newton tolerance and iterations must be > 0");
  rc = ensure_bicg(c);
  if (rc) return rc;
  rc = erem_form_jacobian(c, d_T);  // G(T^n) (and J at X_0 = T^n)
  if (rc) return rc;
  rc = read_reduce(c);
  if (rc) return rc;
  const double xscale = std::max(c->tmax, 1e-300);
  if (theta == 0.0) {  // explicit Euler
    rc = lincomb(c, d_T, {{d_T, 1.0}, {c->F, h}});
    if (stats) { *stats = erem_stats{}; }
    return rc;
  }
  double* g0 = c->rs_k0;  // G(T^n)
  double* X = c->rs_k1;   // Newton iterate
  double* dX = c->rs_k2;  // Newton update
  rc = lincomb(c, g0, {{c->F, 1.0}});
  if (!rc) rc = lincomb(c, X, {{d_T, 1.0}});
  if (rc) return rc;
  const double sigma = 1.0 / (h * theta);
  int total = 0, newton = 0;
  bool conv = false;
  for (newton = 1; newton <= max_newton; ++newton) {
    if (newton > 1) {
      rc = erem_form_jacobian(c, X);  // J(X_k), G(X_k)
      if (rc) return rc;
    }
    // (I - h theta J) dX = -F(X)  <=>  (sigma I - J) dX = -F(X) / (h theta),
    // -F(X)/(h theta) = -sigma X + G(X) + ((1 - theta)/theta) G(T^n) + sigma T^n
    rc = lincomb(c, c->rs_rhs, {{X, -sigma}, {c->F, 1.0}, {g0, (1.0 - theta) / theta}, {d_T, sigma}});
    if (rc) return rc;
    int it = 0;
    rc = bicg_solve(c, sigma, c->rs_rhs, dX, lin_rtol, 10000, &it);
    if (rc) return rc;
    total += it;
    rc = lincomb(c, X, {{X, 1.0}, {dX, 1.0}});
    if (rc) return rc;
    HIP_TRY(c, launch_absmax(c->d, dX, c->red, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->h_red, c->red, sizeof(AsmReduce), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double dmax = slot_max(c->h_red->vmax);
    if (!std::isfinite(dmax)) return fail(c, EREM_ENONFINITE, "non-finite Newton update");
    if (dmax <= newton_rtol * xscale) {
      conv = true;
      break;
    }
  }
  if (!conv) return fail(c, EREM_ENOCONV, "theta-Euler Newton iteration did not converge");
  rc = lincomb(c, d_T, {{X, 1.0}});
  if (rc) return rc;
  if (stats) {
    *stats = erem_stats{};
    stats->substeps = newton;
    stats->iterations = total;
  }
  return EREM_OK;
}

}  // extern "C"
