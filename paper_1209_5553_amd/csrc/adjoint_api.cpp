// C ABI of the sequential coupled step with a tape of its discrete choices
// and of its adjoint (erem_coupled_step, erem_coupled_step_adjoint).
//
// The step (Sec. 3.2.2): transmissibilities and steady pressure at T^n, face
// fluxes, J and G at T^n, then T^{n+1} = T^n + u_s with the Newton-Leja
// substeps u_{j+1} = u_j + delta sum_k d_k q_k, q_0 = G + J u_j (Sec. 4.2,
// Eq. newt).  A tape fixes the interval [alpha, beta] (so c, gamma, the
// divided differences and the shifts), the substep count and each
// substep's degree; the adjoint differentiates the step with these fixed.
#include "erem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.h"
#include "ctx.h"
#include "device.h"
#include "leja.h"

using namespace erem;
using namespace erem_internal;

namespace {

constexpr int kPressureMaxIter = 200000;

int tape_check(erem_ctx* c, const erem_tape* t, const erem_opts* o) {
  if (t->substeps < 1 || t->substeps > EREM_TAPE_MAX_SUBSTEPS)
    return fail(c, EREM_EINVAL, "tape substeps must be in [1, 256]");
  for (int j = 0; j < t->substeps; ++j)
    if (t->m[j] < 1 || t->m[j] > o->m_max) return fail(c, EREM_EINVAL, "tape degree outside [1, m_max]");
  if (!std::isfinite(t->alpha) || !std::isfinite(t->beta) || !(t->beta > t->alpha))
    return fail(c, EREM_EINVAL, "tape interval must satisfy alpha < beta");
  return EREM_OK;
}

int max_degree(const erem_tape* t) {
  int K = 0;
  for (int j = 0; j < t->substeps; ++j) K = std::max(K, static_cast<int>(t->m[j]));
  return K;
}

// Leja coefficients of the tape's interval for substeps of length delta
// (divided differences of phi1 on the scaled interval, shifts c/gamma + xi).
int upload_coef(erem_ctx* c, const erem_tape* t, double delta, int K) {
  const double cc = 0.5 * (t->alpha + t->beta);
  const double gg = 0.25 * (t->beta - t->alpha);
  const std::vector<double>& dv = divided_differences(c, delta * cc, delta * gg, K + 1);
  LejaCoef* hc = c->h_cf;
  hc->inv_g = 1.0 / gg;
  hc->thresh = 0.0;
  for (int k = 0; k <= K; ++k) {
    hc->dk[k] = dv[k];
    hc->shift[k] = (k > 0) ? cc / gg + c->xi[k - 1] : 0.0;
    hc->estf[k] = 0.0;
  }
  const size_t bytes = offsetof(LejaCoef, shift) + 3 * sizeof(double) * (kMaxTerms + 1);
  HIP_TRY(c, hipMemcpyAsync(c->cf, hc, bytes, hipMemcpyHostToDevice, c->stream));
  // one never-checked stop state: every term launch runs
  HIP_TRY(c, launch_leja_reset(c->states, 1, K, c->stream));
  return EREM_OK;
}

// Iterate store: substep j keeps q_k for k = 0, S, 2S, ... <= m_j.
struct Slots {
  std::vector<size_t> off;
  size_t total = 0;
  int S = 1;
};

Slots slot_layout(const erem_tape* t, int S) {
  Slots L;
  L.S = S;
  L.off.resize(t->substeps);
  for (int j = 0; j < t->substeps; ++j) {
    L.off[j] = L.total;
    L.total += static_cast<size_t>(t->m[j] / S) + 1;
  }
  return L;
}

double* slot(erem_ctx* c, const Slots& L, int j, int a) {
  return c->adj_q + (L.off[j] + static_cast<size_t>(a)) * static_cast<size_t>(c->d.N);
}

int grow(erem_ctx* c, double** p, size_t* cap, size_t n) {
  if (*cap >= n) return EREM_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (dev_alloc(c, p, n)) return EREM_ENOMEM;
  *cap = n;
  return EREM_OK;
}

int ensure_adjoint(erem_ctx* c, const Slots& L, int s) {
  const size_t N = c->d.N;
  if (!c->adj_block) {
    // sa, sb, jbar(5), wbar, ubar, rbar, dbar, abar(4), pbar, lam, pscr: 18 N; + faces
    const size_t words = 18 * N + c->nfx + c->nfy;
    if (dev_alloc(c, &c->adj_block, words)) return EREM_ENOMEM;
    double* p = c->adj_block;
    auto take = [&](size_t n) { double* r = p; p += n; return r; };
    c->adj_sa = take(N);
    c->adj_sb = take(N);
    c->adj_jbar = take(5 * N);
    c->adj_wbar = take(N);
    c->adj_ubar = take(N);
    c->adj_rbar = take(N);
    c->adj_dbar = take(N);
    c->adj_abar = take(4 * N);
    c->adj_pbar = take(N);
    c->adj_lam = take(N);
    c->adj_pscr = take(N);
    c->adj_fxbar = take(c->nfx);
    c->adj_fybar = take(c->nfy);
  }
  if (grow(c, &c->adj_q, &c->adj_q_cap, L.total * N)) return EREM_ENOMEM;
  if (grow(c, &c->adj_u, &c->adj_u_cap, static_cast<size_t>(s) * N)) return EREM_ENOMEM;
  if (L.S > 1 && grow(c, &c->adj_seg, &c->adj_seg_cap, static_cast<size_t>(L.S) * N)) return EREM_ENOMEM;
  return EREM_OK;
}

// c->u <- sum of the tape's substeps applied to G = c->F (the step's
// increment).  With a store, q_k (k a multiple of S) of every substep goes
// to the iterate store and u_j (j >= 1) to adj_u.
int replay(erem_ctx* c, double h, const erem_tape* t, const Slots* store) {
  const Dims& d = c->d;
  const int s = t->substeps;
  const double delta = h / s;
  int rc = upload_coef(c, t, delta, max_degree(t));
  if (rc) return rc;
  const size_t N = d.N;
  for (int j = 0; j < s; ++j) {
    const double* src = c->F;
    if (j > 0) {
      HIP_TRY(c, launch_stencil_axpy(d, c->coef, c->F, c->u, c->w, c->stream));
      src = c->w;
      if (store)
        HIP_TRY(c, hipMemcpyAsync(c->adj_u + j * N, c->u, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
    }
    double* cur = store ? slot(c, *store, j, 0) : c->qa;
    HIP_TRY(c, launch_leja_init<double>(d, c->cf, src, cur, c->pacc, c->part, c->stream));
    for (int k = 1; k <= t->m[j]; ++k) {
      double* nxt = (store && k % store->S == 0) ? slot(c, *store, j, k / store->S) : (cur == c->qa ? c->qb : c->qa);
      HIP_TRY(c, launch_leja_term<double>(d, c->cf, c->coef, cur, nxt, c->pacc, c->states, c->part, k, c->stream));
      cur = nxt;
    }
    HIP_TRY(c, launch_substep_update<double>(d, c->u, c->pacc, delta, j == 0 ? 1 : 0, c->stream));
  }
  return EREM_OK;
}

int common_checks(erem_ctx* c, double h, const double* d_T, double p_rtol, const erem_opts* o) {
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (c->d.dim != 2) return fail(c, EREM_EINVAL, "the coupled step and its adjoint support 2D grids");
  if (!d_T) return fail(c, EREM_EINVAL, "T is NULL");
  if (!(h > 0) || !std::isfinite(h)) return fail(c, EREM_EINVAL, "h must be > 0");
  if (!(p_rtol > 0)) return fail(c, EREM_EINVAL, "p_rtol must be > 0");
  return EREM_OK;
}

// Transmissibilities, pressure (zero initial guess) and fluxes at T.
int pressure_at(erem_ctx* c, const double* d_T, double p_rtol, int* iters) {
  int rc = erem_assemble_transmissibilities(c, d_T);
  if (rc) return rc;
  erem_stats pst{};
  rc = erem_solve_pressure(c, p_rtol, kPressureMaxIter, 0, nullptr, &pst);
  if (iters) *iters = pst.iterations;
  return rc;
}

}  // namespace

extern "C" {

int erem_coupled_step(erem_ctx* c, double h, double* d_T, double p_rtol, const erem_opts* o,
                      const erem_tape* tape_in, erem_tape* tape_out, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = common_checks(c, h, d_T, p_rtol, o);
  if (rc) return rc;
  if ((tape_in || tape_out) && (o->method != EREM_METHOD_LEJA || o->precision != EREM_PREC_FP64))
    return fail(c, EREM_EINVAL, "tapes record the FP64 Leja method");
  if (tape_in && (rc = tape_check(c, tape_in, o))) return rc;
  int piters = 0;
  if ((rc = pressure_at(c, d_T, p_rtol, &piters))) return rc;
  if (!tape_in) {
    erem_stats st{};
    if ((rc = erem_step(c, h, d_T, o, &st))) return rc;
    st.iterations = piters;
    if (stats) *stats = st;
    if (tape_out) {
      std::memset(tape_out, 0, sizeof(*tape_out));
      if (c->applied.size() > static_cast<size_t>(EREM_TAPE_MAX_SUBSTEPS))
        return fail(c, EREM_EINVAL, "the step used more substeps than a tape holds");
      tape_out->substeps = static_cast<int32_t>(c->applied.size());
      for (size_t j = 0; j < c->applied.size(); ++j) tape_out->m[j] = c->applied[j];
      tape_out->alpha = c->alpha;
      tape_out->beta = c->beta;
    }
    return EREM_OK;
  }
  if ((rc = erem_form_jacobian(c, d_T))) return rc;
  if ((rc = replay(c, h, tape_in, nullptr))) return rc;
  HIP_TRY(c, launch_axpby(c->d, d_T, 1.0, c->u, 1.0, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (tape_out && tape_out != tape_in) std::memcpy(tape_out, tape_in, sizeof(*tape_out));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    for (int j = 0; j < tape_in->substeps; ++j) stats->m_total += tape_in->m[j];
    stats->substeps = tape_in->substeps;
    stats->iterations = piters;
    stats->alpha = tape_in->alpha;
    stats->beta = tape_in->beta;
  }
  return EREM_OK;
}

int erem_coupled_step_adjoint(erem_ctx* c, double h, const double* d_T, double p_rtol, const erem_opts* o,
                              const erem_tape* tape, int32_t ckpt_stride, double* d_Tbar, double* d_logk_bar,
                              erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = common_checks(c, h, d_T, p_rtol, o);
  if (rc) return rc;
  if (o->method != EREM_METHOD_LEJA || o->precision != EREM_PREC_FP64)
    return fail(c, EREM_EINVAL, "the adjoint runs the FP64 Leja method");
  if (!tape) return fail(c, EREM_EINVAL, "tape is NULL");
  if ((rc = tape_check(c, tape, o))) return rc;
  if (ckpt_stride < 1) return fail(c, EREM_EINVAL, "ckpt_stride must be >= 1");
  if (!d_Tbar || !d_logk_bar || d_Tbar == d_T || d_logk_bar == d_T || d_logk_bar == d_Tbar)
    return fail(c, EREM_EINVAL, "Tbar and logk_bar must be distinct non-NULL arrays");
  const Dims& d = c->d;
  const size_t N = d.N;
  int piters = 0;
  if ((rc = pressure_at(c, d_T, p_rtol, &piters))) return rc;
  if ((rc = erem_form_jacobian(c, d_T))) return rc;
  const Slots L = slot_layout(tape, ckpt_stride);
  const int s = tape->substeps;
  if ((rc = ensure_adjoint(c, L, s))) return rc;
  if ((rc = replay(c, h, tape, &L))) return rc;
  // reverse sweep over the substeps (last first)
  const double delta = h / s;
  const std::vector<double> dk(c->h_cf->dk, c->h_cf->dk + max_degree(tape) + 1);
  const std::vector<double> shift(c->h_cf->shift, c->h_cf->shift + max_degree(tape) + 1);
  const double inv_g = c->h_cf->inv_g;
  HIP_TRY(c, hipMemcpyAsync(c->adj_ubar, d_Tbar, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->adj_jbar, 0, sizeof(double) * 5 * N, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->adj_wbar, 0, sizeof(double) * N, c->stream));
  const int S = ckpt_stride;
  for (int j = s - 1; j >= 0; --j) {
    const int m = tape->m[j];
    double* sin = c->adj_sa;
    double* sout = c->adj_sb;
    if (c->prof && (rc = ensure_events(c, 2 * static_cast<size_t>(m)))) return rc;
    HIP_TRY(c, launch_adj_scale(d, c->adj_ubar, delta * dk[m], sin, c->stream));
    int seg = -1;  // segment of recomputed iterates held in adj_seg
    for (int k = m; k >= 1; --k) {
      const int kk = k - 1;
      const double* q;
      if (kk % S == 0) {
        q = slot(c, L, j, kk / S);
      } else {
        const int a = kk / S;
        if (seg != a) {
          // q_{aS+1} .. q_{min(aS+S-1, m-1)} from the stored q_{aS}
          const double* cur = slot(c, L, j, a);
          const int top = std::min(a * S + S - 1, m - 1);
          for (int kidx = a * S + 1; kidx <= top; ++kidx) {
            double* nxt = c->adj_seg + static_cast<size_t>(kidx - a * S) * N;
            HIP_TRY(c, launch_leja_term<double>(d, c->cf, c->coef, cur, nxt, c->adj_pscr, c->states, c->part, kidx,
                                                c->stream));
            cur = nxt;
          }
          seg = a;
        }
        q = c->adj_seg + static_cast<size_t>(kk - a * S) * N;
      }
      const bool timed = c->prof && k % c->prof == 0;
      HIP_TRY(c, launch_adj_rev_term(d, c->coef, sin, q, c->adj_ubar, delta * dk[kk], inv_g, shift[k], c->adj_jbar,
                                     sout, c->stream, timed ? c->ev[2 * (m - k)] : nullptr,
                                     timed ? c->ev[2 * (m - k) + 1] : nullptr));
      std::swap(sin, sout);
    }
    if (c->prof) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      for (int k = m; k >= 1; --k) {
        if (k % c->prof != 0) continue;
        c->t_adj += elapsed_ms(c->ev[2 * (m - k)], c->ev[2 * (m - k) + 1]);
        ++c->n_adj;
      }
    }
    HIP_TRY(c, launch_adj_substep(d, c->coef, sin, j > 0 ? c->adj_u + j * N : nullptr, c->adj_wbar, c->adj_ubar,
                                  c->adj_jbar, c->stream));
  }
  // G, J -> T, face fluxes -> pressure, transmissibilities -> log K, T
  HIP_TRY(c, launch_adj_heat_cell(d, c->ph, c->poro, c->fx, c->fy, d_T, c->adj_jbar, c->adj_wbar, d_Tbar,
                                  c->adj_rbar, c->adj_dbar, c->adj_abar, c->stream));
  HIP_TRY(c, launch_adj_heat_face(d, c->ph, c->fx, c->fy, c->adj_rbar, c->adj_dbar, c->adj_abar, d_Tbar,
                                  c->adj_fxbar, c->adj_fybar, c->stream));
  HIP_TRY(c, launch_adj_flux_p(d, c->tx, c->ty, c->adj_fxbar, c->adj_fybar, c->adj_pbar, c->stream));
  int aiters = 0;
  // the FP64 residual of the adjoint system cannot certify much below 1e-13;
  // 1e-12 leaves the gradient accurate far beyond what it is used for
  if ((rc = spd_solve(c, c->adj_pbar, c->adj_lam, std::max(p_rtol, 1e-12), kPressureMaxIter, &aiters))) return rc;
  HIP_TRY(c, launch_adj_trans(d, c->ph, c->logk, d_T, c->pres, c->pres_lo, c->adj_fxbar, c->adj_fybar, c->adj_lam,
                              d_Tbar, d_logk_bar, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    for (int j = 0; j < s; ++j) stats->m_total += tape->m[j];
    stats->substeps = s;
    stats->iterations = piters + aiters;
    stats->alpha = tape->alpha;
    stats->beta = tape->beta;
  }
  return EREM_OK;
}

}  // extern "C"
