// C ABI of the EREM library: context, assembly, pressure, phi1 and the step.
//
// Host control follows the paper's algorithm (Sec. 4.2): Gershgorin interval
// of J, Leja points on [-2, 2], divided differences of phi1 on the scaled
// interval, Newton recurrence with the scaled-norm stop test, and splitting
// of the step when the degree would be too large.  All per-cell work runs in
// the kernels of kernels.hip; the host only moves scalars.
#include "erem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "adjoint.h"
#include "ctx.h"
#include "device.h"
#include "host_numerics.h"
#include "krylov.h"
#include "leja.h"
#include "mg.h"

using namespace erem;

namespace erem_internal {

int fail(erem_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

// Make sure the event pool holds at least n events (profiling only).
int ensure_events(erem_ctx* c, size_t n) {
  while (c->ev.size() < n) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  return EREM_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? static_cast<double>(ms) : 0.0;
}

constexpr int kProfSubsteps = 8;  // profiled substeps per evaluation

int check_opts(erem_ctx* c, const erem_opts* o) {
  if (!o) return fail(c, EREM_EINVAL, "opts is NULL");
  if (o->method != EREM_METHOD_LEJA && o->method != EREM_METHOD_KRYLOV)
    return fail(c, EREM_EINVAL, "unknown method");
  if (o->precision != EREM_PREC_FP64 && o->precision != EREM_PREC_MIXED)
    return fail(c, EREM_EINVAL, "unknown precision");
  if (!(o->tol_a >= 0.0) || !(o->tol_r >= 0.0) || (o->tol_a == 0.0 && o->tol_r == 0.0))
    return fail(c, EREM_EINVAL, "tolerances must be >= 0 and not both 0");
  if (o->m_max < 5 || o->m_max > kMaxTerms) return fail(c, EREM_EINVAL, "m_max must be in [5, 1024]");
  if (o->max_substeps < 1 || o->max_substeps > 4096) return fail(c, EREM_EINVAL, "max_substeps must be in [1, 4096]");
  if (o->p_order < 0 || o->p_order > 12) return fail(c, EREM_EINVAL, "p_order must be in [0, 12]");
  if (o->chunk < 0) return fail(c, EREM_EINVAL, "chunk must be >= 0");
  return EREM_OK;
}


void free_all(erem_ctx* c) {
  double** bufs[] = {&c->logk, &c->poro, &c->tx, &c->ty, &c->tz, &c->fx, &c->fy, &c->fz,
                     &c->coef, &c->F, &c->qa, &c->qb, &c->pacc, &c->u, &c->w, &c->pres,
                     &c->pr, &c->pr2, &c->pw, &c->ps0, &c->ps1, &c->pz, &c->pp0, &c->pp1, &c->pq, &c->pdiag,
                     &c->pres_lo, &c->pdelta, &c->prhs, &c->part, &c->gt, &c->zt,
                     &c->bc_r, &c->bc_rhat, &c->bc_p0, &c->bc_p1, &c->bc_v0, &c->bc_v1, &c->bc_s, &c->bc_t,
                     &c->rs_k0, &c->rs_k1, &c->rs_k2, &c->rs_y, &c->rs_g, &c->rs_rhs, &c->rs_coef,
                     &c->xi_dev};
  for (double** b : bufs)
    if (*b) { (void)hipFree(*b); *b = nullptr; }
  if (c->ddc) (void)hipFree(c->ddc);
  c->ddc = nullptr;
  if (c->cf) (void)hipFree(c->cf);
  if (c->states) (void)hipFree(c->states);
  if (c->red) (void)hipFree(c->red);
  if (c->pcg) (void)hipFree(c->pcg);
  if (c->bicg) (void)hipFree(c->bicg);
  if (c->h_bicg) (void)hipHostFree(c->h_bicg);
  if (c->bicg_parts) (void)hipFree(c->bicg_parts);
  c->bicg = nullptr;
  c->h_bicg = nullptr;
  c->bicg_parts = nullptr;
  if (c->h_cf) (void)hipHostFree(c->h_cf);
  if (c->h_states) (void)hipHostFree(c->h_states);
  if (c->h_red) (void)hipHostFree(c->h_red);
  if (c->h_pcg) (void)hipHostFree(c->h_pcg);
  if (c->pcg_parts) (void)hipFree(c->pcg_parts);
  if (c->pres_prev) (void)hipFree(c->pres_prev);
  c->pres_prev = nullptr;
  c->pres_prev_set = false;
  if (c->h_pcg_parts) (void)hipHostFree(c->h_pcg_parts);
  c->pcg_parts = nullptr;
  c->h_pcg_parts = nullptr;
  float** fbufs[] = {&c->coef32, &c->qa32, &c->qb32, &c->p32};
  for (float** b : fbufs)
    if (*b) { (void)hipFree(*b); *b = nullptr; }
  double** kbufs[] = {&c->kV, &c->kw, &c->kH, &c->kbeta, &c->kc, &c->kg, &c->kpart};
  for (double** b : kbufs)
    if (*b) { (void)hipFree(*b); *b = nullptr; }
  double** abufs[] = {&c->adj_q, &c->adj_u, &c->adj_seg, &c->adj_block};
  for (double** b : abufs)
    if (*b) { (void)hipFree(*b); *b = nullptr; }
  c->adj_q_cap = c->adj_u_cap = c->adj_seg_cap = 0;
  c->cf = nullptr; c->states = nullptr; c->red = nullptr; c->pcg = nullptr;
  c->h_cf = nullptr; c->h_states = nullptr; c->h_red = nullptr; c->h_pcg = nullptr;
}

int ndir(const erem_ctx* c) { return c->d.dim == 3 ? 7 : 5; }

void free_mg(erem_ctx* c) {
  for (double* b : c->mg_bufs) (void)hipFree(b);
  c->mg_bufs.clear();
}

// LDS layout of the coarse solve over levels lc..lb: per smoothed level the
// faces (z faces only in 3D), the diagonal, three vectors and 1/diagonal; on
// the bottom level two vectors and the partial products; then the bottom
// inverse.  Fills the offsets when `a` is
// given and returns the number of words.
size_t mg_lds_layout(const MgHierarchy& h, int lc, MgCoarseArgs* a) {
  size_t w = 0;
  for (int l = lc; l <= h.lb; ++l) {
    const MgLevelDev& L = h.lev[l];
    const size_t n = static_cast<size_t>(L.nx) * L.ny * L.nz;
    int* off = a ? a->off[l - lc] : nullptr;
    if (l < h.lb) {
      const size_t nfx = static_cast<size_t>(L.nx + 1) * L.ny * L.nz;
      const size_t nfy = static_cast<size_t>(L.nx) * (L.ny + 1) * L.nz;
      const size_t nfz = L.nz > 1 ? static_cast<size_t>(L.nx) * L.ny * (L.nz + 1) : 0;
      const size_t sizes[8] = {nfx, nfy, nfz, n, n, n, n, n};
      for (int k = 0; k < 8; ++k) {
        if (off) off[k] = static_cast<int>(w);
        w += sizes[k];
      }
    } else {
      // bottom: B, E, the partial products of the dense solve (one row of
      // nb per wavefront of the workgroup), then the inverse
      if (off) {
        for (int k = 0; k < 8; ++k) off[k] = 0;
        off[4] = static_cast<int>(w);
        off[5] = static_cast<int>(w + n);
        off[6] = static_cast<int>(w + 2 * n);
      }
      w += 2 * n + static_cast<size_t>(kMgLdsCells / 64) * n;
      if (a) a->inv_off = static_cast<int>(w);
      w += n * n;
    }
  }
  return w;
}

// Aggregation hierarchy down to one cell; level 0 aliases the context's
// face arrays and diagonal.
int build_mg(erem_ctx* c) {
  MgHierarchy& h = c->mg;
  int nx = c->d.nx, ny = c->d.ny, nz = c->d.nz;
  int l = 0;
  for (;;) {
    if (l >= kMgMaxLevels) return fail(c, EREM_EINVAL, "grid too large for the multigrid hierarchy");
    MgLevelDev& L = h.lev[l];
    L.nx = nx; L.ny = ny; L.nz = nz;
    const size_t n = static_cast<size_t>(nx) * ny * nz;
    auto get = [&](double** p, size_t cnt) {
      if (dev_alloc(c, p, cnt) != EREM_OK) return false;
      c->mg_bufs.push_back(*p);
      return true;
    };
    if (l == 0) {
      L.tx = c->tx; L.ty = c->ty; L.tz = c->tz; L.diag = c->pdiag; L.b = nullptr;
      if (!get(&L.x, n) || !get(&L.y, n)) return EREM_ENOMEM;
    } else {
      const size_t nfx = static_cast<size_t>(nz) * ny * (nx + 1);
      const size_t nfy = static_cast<size_t>(nz) * (ny + 1) * nx;
      const size_t nfz = static_cast<size_t>(nz + 1) * ny * nx;
      if (!get(&L.tx, nfx) || !get(&L.ty, nfy) || !get(&L.tz, nfz) || !get(&L.diag, n) ||
          !get(&L.b, n) || !get(&L.x, n) || !get(&L.y, n))
        return EREM_ENOMEM;
      (void)hipMemsetAsync(L.tz, 0, nfz * sizeof(double), c->stream);
    }
    ++l;
    if (n <= static_cast<size_t>(kMgBottomCells)) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    nz = nz > 1 ? (nz + 1) / 2 : 1;
  }
  h.nlev = l;
  h.lb = l - 1;
  {
    const MgLevelDev& B = h.lev[h.lb];
    const size_t nb = static_cast<size_t>(B.nx) * B.ny * B.nz;
    if (dev_alloc(c, &h.binv, nb * nb) != EREM_OK) return EREM_ENOMEM;
    c->mg_bufs.push_back(h.binv);
  }
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
    max_lds = 65536;
  // First level that fits one workgroup (cells and LDS, with 1 KiB kept for
  // the kernel's static LDS); if the runtime refuses the dynamic LDS size,
  // retry within 64 KiB.
  int lc = h.lb;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const size_t limit = static_cast<size_t>(attempt == 0 ? max_lds : std::min(max_lds, 65536)) - 1024;
    lc = h.lb;
    for (int k = 0; k <= h.lb; ++k) {
      const MgLevelDev& L = h.lev[k];
      const size_t n = static_cast<size_t>(L.nx) * L.ny * L.nz;
      const size_t bytes = mg_lds_layout(h, k, nullptr) * sizeof(double);
      if (n <= static_cast<size_t>(kMgLdsCells) && bytes <= limit) {
        lc = k;
        break;
      }
    }
    const size_t bytes = mg_lds_layout(h, lc, nullptr) * sizeof(double);
    if (mg_set_lds_limit(static_cast<int>(bytes)) == hipSuccess) break;
    (void)hipGetLastError();
    if (attempt == 1) return fail(c, EREM_EDEVICE, "cannot reserve LDS for the coarse multigrid solve");
  }
  h.lc = lc;
  // 2 x 2 (x 2) aggregation makes each Galerkin coarse operator about twice as
  // stiff as the operator of the coarse grid itself; over-correcting by 2.1
  // compensates (about 40% fewer CG iterations than 1.6 on 128^2 - 512^2
  // log-normal fields).
  h.omega_c = 2.1;
  MgCoarseArgs& a = h.coarse;
  a.nlev = h.lb - lc + 1;
  const MgLevelDev& L0 = h.lev[lc];
  a.n0 = L0.nx * L0.ny * L0.nz;
  a.nu = 2;
  a.omega_c = h.omega_c;
  // The LDS levels cost a few microseconds per cycle against tens for a CG
  // iteration on the grid: two cycles there, each solving the second level's
  // coarse problem by two V-cycles, come as close to an exact coarse solve
  // as the CG iteration count can tell on 512^2 log-normal fields (12
  // iterations against 21 with one V-cycle; 9.4 with three sweeps each way
  // on the 2D grid levels).  Repeated cycles keep the preconditioner
  // symmetric.
  a.ncyc = a.nlev > 1 ? kMgTopCycles : 1;
  a.ncyc1 = a.nlev > 2 ? kMgSubCycles : 1;
  h.lds_bytes = mg_lds_layout(h, lc, &a) * sizeof(double);
  for (int k = 0; k < a.nlev; ++k) a.lev[k] = h.lev[lc + k];
  h.coarse_threads = std::min(1024, ((a.n0 + 63) / 64) * 64);
  // the coarse kernel gives each thread at most one cell of its first level
  if (h.coarse_threads < a.n0) return fail(c, EREM_EDEVICE, "coarse multigrid level larger than one workgroup");
  return EREM_OK;
}

// Divided differences of phi_ell (ell = 1, 2) for (hc, hg) with at least n
// coefficients (cached per ell).
const std::vector<double>& divided_differences(erem_ctx* c, double hc, double hg, int n, int ell) {
  DivDiffCache& dd = ell == 2 ? c->dd2 : c->dd;
  if (!(dd.hc == hc && dd.hg == hg && dd.n >= n)) {
    dd.d.assign(n, 0.0);
    phi_divided_differences(ell, hc, hg, c->xi.data(), n, dd.d.data());
    dd.hc = hc;
    dd.hg = hg;
    dd.n = n;
  }
  return dd.d;
}

// Enqueue the readback of a residual kernel's results: the PCG state and
// the ||b||^2 and r.r partials (ring slot 0).  Sum them after the stream
// has been synchronised (residual_sums).
int enqueue_residual_readback(erem_ctx* c) {
  const size_t nb = static_cast<size_t>(c->pcg_nb);
  HIP_TRY(c, hipMemcpyAsync(c->h_pcg, c->pcg, sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_pcg_parts, c->pcg_parts, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_pcg_parts + nb, c->pcg_parts + 5 * nb, sizeof(double) * nb, hipMemcpyDeviceToHost,
                            c->stream));
  return EREM_OK;
}

// r.r and ||b||^2 of the last residual, the partials added in band order.
void residual_sums(const erem_ctx* c, double* rr, double* bb) {
  double a = 0.0, b = 0.0;
  for (int q = 0; q < c->pcg_nb; ++q) {
    b += c->h_pcg_parts[q];
    a += c->h_pcg_parts[c->pcg_nb + q];
  }
  *rr = a;
  *bb = b;
}

// Read the assembly reductions (Gershgorin interval, max |T|, max |v|).
int read_reduce(erem_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->h_red, c->red, sizeof(AsmReduce), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->alpha = slot_min(c->h_red->lo);
  c->beta = slot_max(c->h_red->hi);
  c->tmax = slot_max(c->h_red->tmax);
  return EREM_OK;
}

// Device buffers of the Newton passes in one precision: the stencil of J,
// the two q buffers and the accumulated polynomial p.
template <class V>
struct LejaBufs {
  const V* coef;
  V *qa, *qb, *p;
};

int ensure_mixed(erem_ctx* c) {
  if (!c->coef32) {
    const size_t n = c->d.N;
    int rc = EREM_OK;
    rc |= dev_alloc(c, &c->coef32, n * ndir(c));
    rc |= dev_alloc(c, &c->qa32, n);
    rc |= dev_alloc(c, &c->qb32, n);
    rc |= dev_alloc(c, &c->p32, n);
    if (rc) return EREM_ENOMEM;
  }
  if (!c->coef32_valid) {
    HIP_TRY(c, launch_cast_f32(c->coef, c->coef32, static_cast<long long>(c->d.N) * ndir(c), c->stream));
    c->coef32_valid = true;
  }
  return EREM_OK;
}

// Newton terms computed by the launch that starts at term k of at most K:
// four (2D, a whole stop-test group), else two, else one.
int leja_terms_per_launch(const Dims& d, int k, int K) {
  if (d.dim != 2) return 1;
  if (k + 3 <= K) return 4;
  return k + 1 <= K ? 2 : 1;
}

// One Newton-Leja evaluation over s substeps: its coefficient block, its s
// stop-state slots, the vector that accumulates the substep increments and,
// for the non-autonomous step, the time source g and the fixed phi2 term zt.
struct LejaPass {
  const LejaCoef* cf;
  LejaState* states;
  double* out;
  const double* g;   // source of substep j is v + (j delta) g + J u_j; null: v + J u_j
  const double* zt;  // added to out after every substep; null: nothing
  hipEvent_t* ev;    // 2 K events per timed substep (the first nprof), or null
  int nprof;
};

template <class V>
int leja_run(erem_ctx* c, const LejaBufs<V>& B, const LejaPass& P, const double* v, double delta, int s,
             int K) {
  const Dims& d = c->d;
  for (int j = 0; j < s; ++j) {
    LejaState* st = P.states + j;
    const double* src = v;
    if (j > 0) {
      HIP_TRY(c, launch_stencil_axpy(d, c->coef, v, P.out, c->w, c->stream, P.g, j * delta));
      src = c->w;
    }
    HIP_TRY(c, launch_leja_init<V>(d, P.cf, src, B.qa, B.p, c->part, c->stream));
    hipEvent_t* evj = j < P.nprof ? &P.ev[static_cast<size_t>(j) * 2 * K] : nullptr;
    int prev = -1;  // last term already checked
    V* cur = B.qa;  // latest q
    V* oth = B.qb;
    // 2D grids take the terms in groups of four (one stop-test group per
    // launch, so the stop test still follows every kCheckEvery terms)
    for (int k = 1, launch = 0; k <= K; ++launch) {
      const int nt = leja_terms_per_launch(d, k, K);
      const bool timed = evj && launch % c->prof == 0;
      hipEvent_t e0 = timed ? evj[2 * (k - 1)] : nullptr, e1 = timed ? evj[2 * (k - 1) + 1] : nullptr;
      if (nt > 1)
        HIP_TRY(c, launch_leja_terms<V>(d, P.cf, B.coef, cur, oth, B.p, st, c->part, k, nt, c->stream, e0, e1));
      else
        HIP_TRY(c, launch_leja_term<V>(d, P.cf, B.coef, cur, oth, B.p, st, c->part, k, c->stream, e0, e1));
      std::swap(cur, oth);
      k += nt;
      const int last = k - 1;
      if (last % kCheckEvery == 0 || last == K) {
        HIP_TRY(c, launch_leja_check(d, P.cf, st, c->part, prev + 1, last, c->stream));
        prev = last;
      }
    }
    HIP_TRY(c, launch_substep_update<V>(d, P.out, B.p, delta, j == 0 ? 1 : 0, c->stream, P.zt));
  }
  return EREM_OK;
}

// Newton coefficients of one pass: the divided differences dv of
// phi_ell(delta (c + gamma xi)), the shifts c/gamma + xi_{k-1}, and the
// stop-test factors |w dv_k| / (sqrt(N) scal), w the weight of the pass's
// polynomial in the increment (delta for phi1, delta^2 for phi2).
void fill_coef(LejaCoef* hc, const std::vector<double>& dv, int n, double cc, double gg, double w,
               const std::vector<double>& xi, double rootN, double scal, int p_order) {
  hc->inv_g = 1.0 / gg;
  hc->thresh = std::pow(10.0, -p_order);
  for (int k = 0; k < n; ++k) {
    hc->dk[k] = dv[k];
    hc->shift[k] = (k > 0) ? cc / gg + xi[k - 1] : 0.0;
    hc->estf[k] = std::fabs(w * dv[k]) / (rootN * scal);
  }
}

// Internal result of an evaluation enqueued on a predicted substep count
// whose prediction did not hold: evaluate again on the interval read back.
constexpr int kFallback = -100;  // not an EREM_ code

// Widest substep interval h (beta - alpha) / s of the evaluation's precision.
double substep_rho(const erem_opts* o) {
  return o->precision == EREM_PREC_MIXED ? std::min(o->rho_max, kMixedRhoMax) : o->rho_max;
}

// Substep count of an interval of the given width: h width / rho rounded
// up, at least 1, at most smax (one substep when rho <= 0).
int substeps_for(double h, double width, double rho, int smax) {
  int s = 1;
  if (rho > 0.0) {
    const double q = std::ceil(h * width / rho);
    s = q >= smax ? smax : (q > 1.0 ? static_cast<int>(q) : 1);
  }
  return std::min(s, smax);
}

// Term budget of an evaluation's first attempt: the previous evaluation's
// largest substep degree plus one stop-test group (the launches past the
// stop return at entry), else m_max; a degree that outgrows it restarts the
// evaluation with the full budget.
int first_budget(const erem_ctx* c, const erem_opts* o) {
  if (o->chunk > 0) return std::min(o->chunk, o->m_max);
  return c->last_m > 0 ? std::min(o->m_max, c->last_m + kCheckEvery) : o->m_max;
}

// The host's reading of the reduction slots after an evaluation whose
// coefficients the device formed (launch_leja_coef): the same checks and
// substep count as the synchronous path.  EREM_OK when the device's
// coefficients are the ones the synchronous path would have formed.
int confirm_device_coef(erem_ctx* c, double h, int s, const erem_opts* o, const LejaCoefArgs& a) {
  c->alpha = slot_min(c->h_red->lo);
  c->beta = slot_max(c->h_red->hi);
  c->tmax = slot_max(c->h_red->tmax);
  if (!std::isfinite(c->tmax)) return fail(c, EREM_ENONFINITE, "non-finite temperature");
  const double scal = o->tol_a + o->tol_r * c->tmax;
  if (!(scal > 0)) return fail(c, EREM_EINVAL, "error scale is zero (tol_a = 0 and T = 0)");
  const double width = c->beta - c->alpha;
  const double mag = std::max(std::fabs(c->alpha), std::fabs(c->beta));
  if (!std::isfinite(width)) return fail(c, EREM_ENONFINITE, "non-finite Gershgorin interval");
  if (width <= 1e-14 * mag || width == 0.0) return kFallback;
  if (substeps_for(h, width, a.rho, a.smax) != s) return kFallback;
  // the kernel marks refused states with checked = -2
  for (int j = 0; j < s; ++j)
    if (c->h_states[j].checked == -2) return kFallback;
  return EREM_OK;
}

// u <- h phi1(h J) v by s Leja substeps of delta = h/s, each an exact
// integration of the linear ODE u' = J u + v over delta:
//   u_{j+1} = u_j + delta phi1(delta J) (v + J u_j)   (Sec. 4.2 splitting).
// Returns EREM_OK, EREM_ENOCONV (some substep did not stop within K terms)
// or an error.  `m_used` receives the summed degree actually applied.  With
// `dev` the coefficients are formed on the device (launch_leja_coef) instead
// of uploaded, and kFallback means the interval read back afterwards does not
// give these coefficients (the caller evaluates again on it).
int leja_hphi1(erem_ctx* c, double h, const double* v, const double* g, double scal, int s, int K,
               const erem_opts* o, int* m_used, double* est_last, const LejaCoefArgs* dev = nullptr) {
  const int n = K + 1;
  const bool na = g != nullptr;  // non-autonomous: one phi2 pass first, in slot s
  const int npass = s + (na ? 1 : 0);
  const double delta = h / s;
  if (!dev) {
    const double a = c->alpha, b = c->beta;
    const double cc = 0.5 * (a + b);
    const double gg = 0.25 * (b - a);
    const double rootN = std::sqrt(static_cast<double>(c->d.N));
    fill_coef(c->h_cf, divided_differences(c, delta * cc, delta * gg, n, 1), n, cc, gg, delta, c->xi, rootN,
              scal, o->p_order);
    if (na)
      fill_coef(c->h_cf + 1, divided_differences(c, delta * cc, delta * gg, n, 2), n, cc, gg, delta * delta,
                c->xi, rootN, scal, o->p_order);
    const size_t cf_bytes = offsetof(LejaCoef, shift) + 3 * sizeof(double) * (kMaxTerms + 1);
    HIP_TRY(c, hipMemcpyAsync(c->cf, c->h_cf, na ? 2 * sizeof(LejaCoef) : cf_bytes, hipMemcpyHostToDevice,
                              c->stream));
  }
  HIP_TRY(c, launch_leja_reset(c->states, npass, K, c->stream));
  if (dev) HIP_TRY(c, launch_leja_coef(*dev, c->stream));
  const int nprof = c->prof ? std::min(s, kProfSubsteps) : 0;
  if (c->prof) {
    const int rc = ensure_events(c, static_cast<size_t>(nprof + 1) * 2 * K);
    if (rc) return rc;
  }
  hipEvent_t* ev = c->prof ? c->ev.data() : nullptr;
  // phi2 pass: zt = delta^2 phi2(delta J) g, the same vector on every
  // substep; then the phi1 substeps with the time source and zt added
  const LejaPass p2{c->cf + 1, c->states + s, c->zt, nullptr, nullptr, ev ? ev + static_cast<size_t>(nprof) * 2 * K : nullptr,
                    c->prof ? 1 : 0};
  const LejaPass p1{c->cf, c->states, c->u, g, na ? c->zt : nullptr, ev, nprof};
  int rc = EREM_OK;
  if (o->precision == EREM_PREC_MIXED) {
    rc = ensure_mixed(c);
    if (rc) return rc;
    const LejaBufs<float> B{c->coef32, c->qa32, c->qb32, c->p32};
    if (na) rc = leja_run<float>(c, B, p2, g, delta * delta, 1, K);
    if (!rc) rc = leja_run<float>(c, B, p1, v, delta, s, K);
  } else {
    const LejaBufs<double> B{c->coef, c->qa, c->qb, c->pacc};
    if (na) rc = leja_run<double>(c, B, p2, g, delta * delta, 1, K);
    if (!rc) rc = leja_run<double>(c, B, p1, v, delta, s, K);
  }
  if (rc) return rc;
  // Read the stop state of every pass (and the stop-test factors the device
  // formed).
  const size_t hdr = offsetof(LejaState, sums);
  for (int j = 0; j < npass; ++j)
    HIP_TRY(c, hipMemcpyAsync(reinterpret_cast<char*>(c->h_states + j),
                              reinterpret_cast<const char*>(c->states + j),
                              hdr + sizeof(double) * (K + 1), hipMemcpyDeviceToHost, c->stream));
  if (dev)
    HIP_TRY(c, hipMemcpyAsync(c->h_cf->estf, reinterpret_cast<const char*>(c->cf) + offsetof(LejaCoef, estf),
                              sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (dev) {
    const int crc = confirm_device_coef(c, h, s, o, *dev);
    if (crc) return crc;
  }
  int total = 0;
  double last = 0.0;
  c->applied.assign(s, 0);
  for (int j = 0; j < npass; ++j) {
    const LejaState& st = c->h_states[j];
    if (st.nonfinite) return fail(c, EREM_ENONFINITE, "non-finite Leja term norm");
    if (st.stopped < 0) return EREM_ENOCONV;
    // the stop test ran after every kCheckEvery terms: the terms up to the
    // end of the group in which it passed were applied
    const int applied = std::min(K, ((st.stopped + kCheckEvery - 1) / kCheckEvery) * kCheckEvery);
    total += applied;
    if (j < s) c->applied[j] = applied;
    // estimate of the last phi1 substep and of the phi2 pass
    if (j + 1 >= s) {
      const LejaCoef& hcf = c->h_cf[j < s ? 0 : 1];
      last = std::max(last, hcf.estf[st.stopped] * std::sqrt(st.sums[st.stopped]));
    }
    const int timed_slot = j < s ? (j < nprof ? j : -1) : (c->prof ? nprof : -1);
    if (timed_slot >= 0) {
      const hipEvent_t* evj = &c->ev[static_cast<size_t>(timed_slot) * 2 * K];
      for (int k = 1, launch = 0; k <= applied; ++launch) {
        const int nt = leja_terms_per_launch(c->d, k, K);
        if (launch % c->prof == 0) {
          c->t_leja += elapsed_ms(evj[2 * (k - 1)], evj[2 * (k - 1) + 1]);
          c->n_leja += nt;
        }
        k += nt;
      }
    }
  }
  *m_used = total;
  *est_last = last;
  return EREM_OK;
}

// u <- h phi1(h J) v by the Krylov projection of Sec. 4.1 (Eq. approphi):
// on each substep the Arnoldi basis V_{m+1}, H of w = v + J u is built on the
// device (Alg. alg:al2, with classical Gram-Schmidt applied twice), and on
// the host y = phi1(delta Hbar) e_1 with
// Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] is read off
// exp([[delta Hbar, e_1], [0, 0]]).  The a-posteriori estimate is the size of
// the last basis vector's contribution, delta beta |y_{m+1}| (scaled norm of
// Sec. 4.2); while 10^p times it is not below 1 the substep is halved, reusing
// the same basis.  Then u += delta beta V_{m+1} y.
int krylov_hphi1(erem_ctx* c, double h, const double* v, double scal, const erem_opts* o, erem_stats* stats) {
  const int m = o->krylov_m;
  if (m < 1 || m > kMaxKrylov) return fail(c, EREM_EINVAL, "krylov_m must be in [1, 64]");
  const size_t N = c->d.N;
  if (c->kry_m < m) {
    double** kbufs[] = {&c->kV, &c->kw, &c->kH, &c->kbeta, &c->kc, &c->kg, &c->kpart};
    for (double** b : kbufs)
      if (*b) { (void)hipFree(*b); *b = nullptr; }
    int rc = EREM_OK;
    rc |= dev_alloc(c, &c->kV, N * (m + 1));
    rc |= dev_alloc(c, &c->kw, 2 * N);
    rc |= dev_alloc(c, &c->kH, static_cast<size_t>(m + 1) * m);
    rc |= dev_alloc(c, &c->kbeta, 1);
    rc |= dev_alloc(c, &c->kc, m + 1);
    rc |= dev_alloc(c, &c->kg, m + 1);
    rc |= dev_alloc(c, &c->kpart, static_cast<size_t>(m + 1) * kry_num_blocks(c->d));
    if (rc) return EREM_ENOMEM;
    c->kry_m = m;
  }
  const Dims& d = c->d;
  const double thresh = std::pow(10.0, -o->p_order);
  const double rootN = std::sqrt(static_cast<double>(N));
  const int max_halvings = 60;
  c->hH.assign(static_cast<size_t>(m + 1) * m + 1, 0.0);
  double t = 0.0, delta = h;
  int nsub = 0, msum = 0;
  double last_est = 0.0;
  bool first = true;
  while (t < h) {
    if (nsub >= o->max_substeps)
      return fail(c, EREM_ENOCONV, "Krylov phi1 needs more than max_substeps substeps");
    // start vector v + J u (u = 0 on the first substep) into the first half of kw
    if (first) HIP_TRY(c, hipMemcpyAsync(c->kw, v, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else HIP_TRY(c, launch_stencil_axpy(d, c->coef, v, c->u, c->kw, c->stream));
    HIP_TRY(c, arnoldi_cgs2(d, c->coef, c->kV, c->kw, c->kH, c->kbeta, c->kg, c->kpart, m, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->hH.data(), c->kH, sizeof(double) * (m + 1) * m, hipMemcpyDeviceToHost, c->stream));
    double beta = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&beta, c->kbeta, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!std::isfinite(beta)) return fail(c, EREM_ENONFINITE, "non-finite Krylov vector norm");
    const std::vector<double>& H = c->hH;
    if (beta == 0.0) {
      // w = 0: u is a steady state of u' = J u + v, nothing changes any more
      if (first) HIP_TRY(c, launch_axpby(d, c->u, 0.0, v, 0.0, c->stream));
      break;
    }
    // Happy breakdown: the first column j whose subdiagonal h_{j+1,j} is
    // negligible against the entries so far gives an exact invariant
    // subspace; columns after it (built from a zero or noise vector) are
    // never read.
    double hnorm = 0.0;
    int me = m;
    bool exact = false;
    for (int j = 0; j < m; ++j) {
      for (int i = 0; i <= j; ++i) {
        const double e = H[i * m + j];
        if (!std::isfinite(e)) return fail(c, EREM_ENONFINITE, "non-finite Hessenberg entry");
        hnorm = std::max(hnorm, std::fabs(e));
      }
      const double hj = H[(j + 1) * m + j];
      if (!std::isfinite(hj)) return fail(c, EREM_ENONFINITE, "non-finite Hessenberg entry");
      if (hj <= 1e-14 * hnorm) {
        me = j + 1;
        exact = true;
        break;
      }
      hnorm = std::max(hnorm, hj);
    }
    const int n = exact ? me : me + 1;  // dimension of Hbar
    std::vector<double> A((n + 1) * (n + 1)), E((n + 1) * (n + 1)), y(n);
    double dl = std::min(delta, h - t);
    bool ok = false;
    double est = 0.0;
    for (int tries = 0; tries < max_halvings; ++tries) {
      std::fill(A.begin(), A.end(), 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < std::min(me, n); ++j)
          if (i <= j + 1 && i < m + 1 && j < m) A[i * (n + 1) + j] = dl * H[i * m + j];
      A[0 * (n + 1) + n] = 1.0;  // augmented column e_1
      dense_expm(n + 1, A.data(), E.data());
      for (int i = 0; i < n; ++i) y[i] = E[i * (n + 1) + n];
      est = exact ? 0.0 : dl * beta * std::fabs(y[n - 1]) / (rootN * scal);
      if (!std::isfinite(est)) return fail(c, EREM_ENONFINITE, "non-finite Krylov estimate");
      if (est < thresh) {  // 10^p * estimate < 1
        ok = true;
        break;
      }
      dl *= 0.5;
    }
    if (!ok) return fail(c, EREM_ENOCONV, "Krylov substep could not meet the tolerance");
    std::vector<double> coeffs(n);
    for (int i = 0; i < n; ++i) coeffs[i] = dl * beta * y[i];
    HIP_TRY(c, hipMemcpyAsync(c->kc, coeffs.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, krylov_combine(d, c->kV, n, c->kc, c->u, first ? 1 : 0, c->stream));
    // the coefficient upload reuses a host vector: wait before it goes out of scope
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    t += dl;
    delta = dl;
    first = false;
    ++nsub;
    msum += me;
    last_est = est;
  }
  if (stats) {
    stats->m_total = msum;
    stats->substeps = nsub;
    stats->est_err = last_est;
    stats->restarts = 0;
  }
  return EREM_OK;
}

// Bookkeeping of a converged Leja evaluation: the degree memory of the next
// term budget and the statistics.
void eval_done(erem_ctx* c, int s, int m_used, double est, int restarts, erem_stats* stats) {
  int m1 = 0;  // the largest phi1 degree of a substep
  for (int a : c->applied) m1 = std::max(m1, a);
  c->last_m = m1;
  if (stats) {
    stats->m_total = m_used;
    stats->substeps = s;
    stats->est_err = est;
    stats->restarts = restarts;
  }
}

// Full evaluation with the substep / restart policy.  On success c->u holds
// h phi1(h J) v, plus h^2 phi2(h J) g when g is not null (the increment of
// the non-autonomous step, Sec. 3.2.3, Eq. nEERMg; Leja method only).
// s_failed > 0: an attempt with s_failed substeps and budget K_failed has
// already run and not converged; the policy continues from it.
int hphi1_eval(erem_ctx* c, double h, const double* v, const double* g, double scal, const erem_opts* o,
               erem_stats* stats, int s_failed = 0, int K_failed = 0) {
  const double width = c->beta - c->alpha;
  const double mag = std::max(std::fabs(c->alpha), std::fabs(c->beta));
  if (!std::isfinite(width)) return fail(c, EREM_ENONFINITE, "non-finite Gershgorin interval");
  if (stats) { stats->alpha = c->alpha; stats->beta = c->beta; stats->restarts = 0; }
  if (width <= 1e-14 * mag || width == 0.0) {
    // Degenerate interval: J = c I (all Gershgorin radii zero, equal
    // diagonal), so h phi1(h J) v = h phi1(h c) v exactly, and likewise
    // h^2 phi2(h J) g = h^2 phi2(h c) g.
    const double z = h * 0.5 * (c->alpha + c->beta);
    const double f = (z == 0.0) ? h : h * (std::expm1(z) / z);
    HIP_TRY(c, launch_axpby(c->d, c->u, 0.0, v, f, c->stream));
    if (g) HIP_TRY(c, launch_axpby(c->d, c->u, 1.0, g, h * h * phi2_scalar(z), c->stream));
    c->applied.clear();
    c->last_w = 0.0;
    if (stats) { stats->m_total = 0; stats->substeps = 1; stats->est_err = 0.0; }
    return EREM_OK;
  }
  if (o->method == EREM_METHOD_KRYLOV) return krylov_hphi1(c, h, v, scal, o, stats);
  // the non-autonomous evaluation keeps one stop-state slot for its phi2 pass
  const int smax = std::min(o->max_substeps, g ? c->nstates - 1 : c->nstates);
  int s = substeps_for(h, width, substep_rho(o), smax);
  int K = first_budget(c, o);
  int restarts = 0;
  bool retry = s_failed > 0;
  if (retry) {
    s = s_failed;
    K = K_failed;
  }
  for (;;) {
    if (retry) {
      ++restarts;
      if (K < o->m_max) {
        K = o->m_max;
      } else if (2 * s <= smax) {
        s *= 2;
      } else {
        return fail(c, EREM_ENOCONV, "phi1 did not converge within m_max terms and max_substeps substeps");
      }
    }
    int m_used = 0;
    double est = 0.0;
    const int rc = leja_hphi1(c, h, v, g, scal, s, K, o, &m_used, &est);
    if (rc == EREM_OK) {
      eval_done(c, s, m_used, est, restarts, stats);
      c->last_w = width;
      return EREM_OK;
    }
    if (rc != EREM_ENOCONV) return rc;
    retry = true;
  }
}

// T += h phi1(h J) F (Leja method) enqueued right behind the assembly, with
// no host synchronisation before the Newton passes: the substep count is
// predicted from the previous evaluation's interval width, the coefficients
// are formed on the device from the assembly's reduction slots
// (launch_leja_coef), and the slots read back with the stop states confirm
// the prediction.  kFallback when there is no prediction or it did not hold
// (the step then runs on the interval read from the slots).
int step_predicted(erem_ctx* c, double h, double* d_T, const erem_opts* o, erem_stats* stats) {
  if (o->method != EREM_METHOD_LEJA || !(c->last_w > 0.0) || !std::isfinite(c->last_w)) return kFallback;
  const int smax = std::min(o->max_substeps, c->nstates);
  const double rho = substep_rho(o);
  const int s = substeps_for(h, c->last_w, rho, smax);
  const int K = first_budget(c, o);
  const int n = K + 1;
  // budgets past what the device forms in LDS take the synchronous path
  if (n > kCoefMaxN) return kFallback;
  HIP_TRY(c, hipMemcpyAsync(c->h_red, c->red, sizeof(AsmReduce), hipMemcpyDeviceToHost, c->stream));
  LejaCoefArgs a{};
  a.red = c->red;
  a.n = n;
  a.s = s;
  a.smax = smax;
  a.h = h;
  a.rho = rho;
  a.tol_a = o->tol_a;
  a.tol_r = o->tol_r;
  a.thresh = std::pow(10.0, -o->p_order);
  a.rootN = std::sqrt(static_cast<double>(c->d.N));
  a.xi = c->xi_dev;
  a.cache = c->ddc;
  a.cf = c->cf;
  a.st = c->states;
  int m_used = 0;
  double est = 0.0;
  int rc = leja_hphi1(c, h, c->F, nullptr, 0.0, s, K, o, &m_used, &est, &a);
  if (rc == kFallback) return kFallback;
  if (stats && (rc == EREM_OK || rc == EREM_ENOCONV)) {
    stats->alpha = c->alpha;
    stats->beta = c->beta;
    stats->restarts = 0;
  }
  if (rc == EREM_OK) {
    eval_done(c, s, m_used, est, 0, stats);
    c->last_w = c->beta - c->alpha;
  } else if (rc == EREM_ENOCONV) {
    rc = hphi1_eval(c, h, c->F, nullptr, o->tol_a + o->tol_r * c->tmax, o, stats, s, K);
  }
  if (rc) return rc;
  HIP_TRY(c, launch_axpby(c->d, d_T, 1.0, c->u, 1.0, c->stream));
  return EREM_OK;
}

// Conjugate gradients on A delta = prhs from delta = 0 (delta in c->pdelta)
// to the relative residual inner_tol, with the context's preconditioner, at
// most `budget` iterations.  *iters gets the iterations run, *done whether
// the tolerance was reached.
// Reduction asked of one correction solve: what the outer tolerance still
// needs (with a margin), between the reduction FP64 conjugate gradients reach
// reliably on the refined residual and a minimum that keeps each correction
// worth its setup.
double inner_tolerance(double relres, double rtol) {
  const double want = 0.5 * rtol / relres;
  return std::min(1e-2, std::max(1e-12, want));
}

int pcg_inner(erem_ctx* c, double inner_tol, int budget, int* iters, bool* done, int* last) {
  const Dims& d = c->d;
  HIP_TRY(c, launch_pcg_reset(c->pcg, inner_tol * inner_tol, c->stream));
  const int jac = c->use_mg ? 0 : 1;
  HIP_TRY(c, launch_pcg_start_rhs(d, c->tx, c->ty, c->tz, c->prhs, c->pdelta, c->pr, c->pz, c->pp0, c->pdiag,
                                  c->pcg, jac, c->stream));
  // 2D multigrid: Chronopoulos-Gear iterations folded into the finest legs
  // (no separate CG kernels); otherwise pcg_a, pcg_b and the preconditioner.
  const bool fuse = c->use_mg && mg_fuses_cg(c->mg);
  if (fuse) {
    const CgFuse cg0{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c->pw};
    HIP_TRY(c, mg_apply(c->mg, c->pr, c->pz, c->pcg, 0, c->stream, &cg0));
  } else if (c->use_mg) {
    HIP_TRY(c, mg_apply(c->mg, c->pr, c->pz, c->pcg, 0, c->stream));
  }
  // Iterations after convergence still launch (their kernels return at
  // entry), so the host polls where the solve is expected to end: with
  // multigrid the first poll follows the count of the previous solve of the
  // same kind and correction (*last) plus the test iteration (at most 24),
  // then every two iterations.
  const int first_chunk = c->use_mg ? (*last > 0 ? std::min(*last + 1, 24) : 8) : 64;
  const int chunk = c->use_mg ? 2 : 64;
  int it = 0;
  *done = false;
  if (c->prof) {
    const int rc = ensure_events(c, 6 * std::max(first_chunk, chunk));
    if (rc) return rc;
  }
  while (it < budget) {
    const int n = std::min(it == 0 ? first_chunk : chunk, budget - it);
    const int it0 = it;
    for (int j = 0; j < n; ++j, ++it) {
      double* pold = (it & 1) ? c->pp1 : c->pp0;
      double* pnew = (it & 1) ? c->pp0 : c->pp1;
      const bool timed = c->prof && it % c->prof == 0;  // sampled iterations
      // six events per iteration: kernel-level ones for pcg_a (0, 1) and
      // pcg_b (4, 5), ones around the preconditioner application (2, 3)
      hipEvent_t* ev = &c->ev[6 * j];
      if (fuse) {
        // r and s alternate between two buffers (neighbouring tiles read
        // the old ones); p, x, z and w are updated in place
        const CgFuse cg{1, it, c->pdelta, (it & 1) ? c->pr : c->pr2, c->pz, c->pw, c->pp0,
                        (it & 1) ? c->ps1 : c->ps0, (it & 1) ? c->ps0 : c->ps1, c->pw};
        if (timed) HIP_TRY(c, hipEventRecord(ev[2], c->stream));
        HIP_TRY(c, mg_apply(c->mg, (it & 1) ? c->pr2 : c->pr, c->pz, c->pcg, (it + 1) & 3, c->stream, &cg));
      } else {
        HIP_TRY(c, launch_pcg_a(d, c->tx, c->ty, c->tz, c->pz, pold, pnew, c->pq, c->pcg, it, c->stream,
                                timed ? ev[0] : nullptr, timed ? ev[1] : nullptr));
        HIP_TRY(c, launch_pcg_b(d, c->pdelta, c->pr, c->pz, pnew, c->pq, c->pdiag, c->pcg, it, jac, c->stream,
                                timed ? ev[4] : nullptr, timed ? ev[5] : nullptr));
        if (timed) HIP_TRY(c, hipEventRecord(ev[2], c->stream));
        if (c->use_mg) HIP_TRY(c, mg_apply(c->mg, c->pr, c->pz, c->pcg, (it + 1) & 3, c->stream));
      }
      if (timed) HIP_TRY(c, hipEventRecord(ev[3], c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(c->h_pcg, c->pcg, sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->h_pcg->nonfinite) return fail(c, EREM_ENONFINITE, "non-finite PCG residual");
    const bool fin = c->h_pcg->done != 0;
    if (c->prof) {
      // iterations it0 .. it_done-1 ran fully; the test launch it_done returned at entry
      const int ran = fin ? c->h_pcg->it_done - it0 : n;
      for (int j = 0; j < ran; ++j) {
        if ((it0 + j) % c->prof != 0) continue;
        const hipEvent_t* ev = &c->ev[6 * j];
        if (!fuse) {
          c->t_pcg_a += elapsed_ms(ev[0], ev[1]);
          ++c->n_pcg_a;
          c->t_pcg_b += elapsed_ms(ev[4], ev[5]);
          ++c->n_pcg_b;
        }
        if (c->use_mg) {
          c->t_mg += elapsed_ms(ev[2], ev[3]);
          ++c->n_mg;
        }
      }
    }
    if (fin) { *done = true; it = c->h_pcg->it_done; break; }
  }
  *iters = it;
  if (*done) *last = it;
  return EREM_OK;
}

int spd_solve(erem_ctx* c, const double* b, double* x, double rtol, int max_iter, int* iters) {
  const Dims& d = c->d;
  if (d.dim != 2) return fail(c, EREM_EINVAL, "the general right-hand-side solve supports 2D grids");
  HIP_TRY(c, hipMemsetAsync(x, 0, sizeof(double) * d.N, c->stream));
  int total = 0;
  bool ok = false;
  // multigrid setup behind the first residual readback, as in the pressure
  // solve (the residual does not read the hierarchy)
  bool setup_pending = c->use_mg;
  if (setup_pending && !c->ev_setup) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_setup, hipEventDisableTiming));
  for (int outer = 0; outer < 12; ++outer) {
    HIP_TRY(c, launch_pcg_reset(c->pcg, 0.0, c->stream));
    HIP_TRY(c, launch_spd_residual(d, c->tx, c->ty, x, b, c->prhs, c->pcg, c->stream));
    {
      const int rc = enqueue_residual_readback(c);
      if (rc) return rc;
    }
    if (setup_pending) {
      HIP_TRY(c, hipEventRecord(c->ev_setup, c->stream));
      HIP_TRY(c, mg_setup(c->mg, c->stream));
      setup_pending = false;
      HIP_TRY(c, hipEventSynchronize(c->ev_setup));
    } else {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    double rr = 0.0, bb = 0.0;
    residual_sums(c, &rr, &bb);
    if (!std::isfinite(rr)) return fail(c, EREM_ENONFINITE, "non-finite residual in the adjoint pressure solve");
    if (bb == 0.0 || rr <= rtol * rtol * bb) { ok = true; break; }
    if (total >= max_iter) break;
    int it = 0;
    bool done = false;
    const double relres = std::sqrt(rr / bb);
    const int rc = pcg_inner(c, inner_tolerance(relres, rtol), max_iter - total, &it, &done,
                             &c->pcg_last[1][std::min(outer, 3)]);
    if (rc) return rc;
    total += it;
    HIP_TRY(c, launch_axpby(d, x, 1.0, c->pdelta, 1.0, c->stream));
  }
  if (iters) *iters = total;
  if (!ok) return fail(c, EREM_ENOCONV, "adjoint pressure solve did not reach rtol within max_iter");
  return EREM_OK;
}

}  // namespace erem_internal

using namespace erem_internal;

extern "C" {

void erem_default_opts(erem_opts* o) {
  if (!o) return;
  o->method = EREM_METHOD_LEJA;
  o->precision = EREM_PREC_FP64;
  o->tol_a = 0.0;
  o->tol_r = 1e-12;
  o->p_order = 2;
  o->m_max = 256;
  o->max_substeps = 64;
  o->krylov_m = 10;
  o->chunk = 0;
  o->rho_max = 64.0;
}

int erem_create(const erem_grid* g, void* stream, erem_ctx** out) {
  if (!out) return EREM_EINVAL;
  *out = nullptr;
  if (!g) return EREM_EINVAL;
  if (g->dim != 2 && g->dim != 3) return EREM_EINVAL;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return EREM_EINVAL;
  if (g->dim == 2 && g->nz != 1) return EREM_EINVAL;
  if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0)) return EREM_EINVAL;
  // Cell and face indices are 32-bit: at most 2^30 cells, 65535 layers.
  // Launch grids put ny/4 blocks on the second grid axis (at most 65535).
  if (g->nx > (1 << 30) || g->ny > 4ll * 65535 || g->nz > 65535) return EREM_EINVAL;
  if (g->nx * g->ny > (1ll << 30)) return EREM_EINVAL;
  const long long N = g->nx * g->ny * g->nz;
  if (N + g->ny * g->nz > (1ll << 30) || N + g->nx * g->nz > (1ll << 30) || N + g->nx * g->ny > (1ll << 30))
    return EREM_EINVAL;
  erem_ctx* c = new (std::nothrow) erem_ctx();
  if (!c) return EREM_ENOMEM;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return EREM_EDEVICE; }
  c->d.nx = static_cast<int>(g->nx);
  c->d.ny = static_cast<int>(g->ny);
  c->d.nz = static_cast<int>(g->nz);
  c->d.dim = g->dim;
  c->d.N = static_cast<int>(N);
  c->d.dx = g->dx; c->d.dy = g->dy; c->d.dz = g->dz;
  const size_t n = static_cast<size_t>(N);
  c->nfx = static_cast<size_t>(g->nz) * g->ny * (g->nx + 1);
  c->nfy = static_cast<size_t>(g->nz) * (g->ny + 1) * g->nx;
  c->nfz = static_cast<size_t>(g->nz + 1) * g->ny * g->nx;
  int rc = EREM_OK;
  rc |= dev_alloc(c, &c->logk, n);
  rc |= dev_alloc(c, &c->poro, n);
  rc |= dev_alloc(c, &c->tx, c->nfx);
  rc |= dev_alloc(c, &c->ty, c->nfy);
  rc |= dev_alloc(c, &c->tz, c->nfz);
  rc |= dev_alloc(c, &c->fx, c->nfx);
  rc |= dev_alloc(c, &c->fy, c->nfy);
  rc |= dev_alloc(c, &c->fz, c->nfz);
  rc |= dev_alloc(c, &c->coef, n * ndir(c));
  rc |= dev_alloc(c, &c->F, n);
  rc |= dev_alloc(c, &c->qa, n);
  rc |= dev_alloc(c, &c->qb, n);
  rc |= dev_alloc(c, &c->pacc, n);
  rc |= dev_alloc(c, &c->u, n);
  rc |= dev_alloc(c, &c->w, n);
  rc |= dev_alloc(c, &c->pres, n);
  rc |= dev_alloc(c, &c->pr, n);
  rc |= dev_alloc(c, &c->pr2, n);
  rc |= dev_alloc(c, &c->pw, n);
  rc |= dev_alloc(c, &c->ps0, n);
  rc |= dev_alloc(c, &c->ps1, n);
  rc |= dev_alloc(c, &c->pz, n);
  rc |= dev_alloc(c, &c->pp0, n);
  rc |= dev_alloc(c, &c->pp1, n);
  rc |= dev_alloc(c, &c->pq, n);
  rc |= dev_alloc(c, &c->pdiag, n);
  rc |= dev_alloc(c, &c->pres_lo, n);
  rc |= dev_alloc(c, &c->pdelta, n);
  rc |= dev_alloc(c, &c->prhs, n);
  rc |= dev_alloc(c, &c->part, static_cast<size_t>(kLejaRing) * leja_num_blocks(c->d));
  c->nstates = 64;
  rc |= dev_alloc(c, &c->cf, 2);  // phi1 and phi2 coefficient blocks
  rc |= dev_alloc(c, &c->states, c->nstates);
  rc |= dev_alloc(c, &c->red, 1);
  rc |= dev_alloc(c, &c->pcg, 1);
  rc |= dev_alloc(c, &c->xi_dev, kMaxTerms + 1);
  rc |= dev_alloc(c, &c->ddc, 1);
  c->pcg_nb = cell_bands(c->d);
  rc |= dev_alloc(c, &c->pcg_parts, pcg_parts_words(c->pcg_nb));
  if (rc == EREM_OK) {
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_cf), 2 * sizeof(LejaCoef), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_states), sizeof(LejaState) * c->nstates, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_red), sizeof(AsmReduce), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_pcg), sizeof(PcgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_pcg_parts), 2 * sizeof(double) * c->pcg_nb,
                      hipHostMallocDefault) != hipSuccess)
      rc = EREM_ENOMEM;
  }
  if (rc == EREM_OK) {
    // the state's pointers into the partial slots, set once
    PcgState init{};
    pcg_bind_parts(&init, c->pcg_parts, c->pcg_nb);
    if (hipMemcpy(c->pcg, &init, sizeof(PcgState), hipMemcpyHostToDevice) != hipSuccess) rc = EREM_EDEVICE;
  }
  if (rc != EREM_OK) {
    free_all(c);
    delete c;
    return EREM_ENOMEM;
  }
  // Zero-initialise the state that is read before it is written.
  (void)hipMemsetAsync(c->pres, 0, n * sizeof(double), c->stream);
  (void)hipMemsetAsync(c->pres_lo, 0, n * sizeof(double), c->stream);
  (void)hipMemsetAsync(c->fz, 0, c->nfz * sizeof(double), c->stream);
  (void)hipMemsetAsync(c->tz, 0, c->nfz * sizeof(double), c->stream);
  (void)hipMemsetAsync(c->u, 0, n * sizeof(double), c->stream);
  if (!leja_points(kMaxTerms + 1, c->xi)) {
    free_all(c);
    delete c;
    return EREM_EINVAL;
  }
  // the device's copy of the points; an empty divided-difference cache
  (void)hipMemcpyAsync(c->xi_dev, c->xi.data(), sizeof(double) * (kMaxTerms + 1), hipMemcpyHostToDevice, c->stream);
  (void)hipMemsetAsync(c->ddc, 0, sizeof(DdCache), c->stream);
  {
    const int mrc = build_mg(c);
    if (mrc != EREM_OK) {
      free_mg(c);
      free_all(c);
      delete c;
      return mrc;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    free_mg(c);
    free_all(c);
    delete c;
    return EREM_EDEVICE;
  }
  // Defaults of the linear workloads; every setter overrides them.
  c->ph.law = EREM_LAW_CONSTANT;
  c->ph.dirichlet_left = 1;
  c->ph.c_f = 4200.0; c->ph.mu0 = 1e-3; c->ph.rho0 = 1000.0;
  c->ph.lam = 2.5; c->ph.rhoc_s = 2.4e6;
  c->ph.p_left = 0.0; c->ph.p_right = 0.0; c->ph.T_left = 20.0; c->ph.T_right = 20.0;
  *out = c;
  return EREM_OK;
}

int erem_destroy(erem_ctx* c) {
  if (!c) return EREM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  if (c->ev_setup) (void)hipEventDestroy(c->ev_setup);
  c->ev_setup = nullptr;
  free_mg(c);
  free_all(c);
  delete c;
  return EREM_OK;
}

const char* erem_last_error(const erem_ctx* c) {
  if (!c) return "NULL context";
  return c->err.c_str();
}

int erem_set_rock(erem_ctx* c, const double* d_logk, const double* d_poro, double lambda, double rhoc_s) {
  if (!c) return EREM_EINVAL;
  if (!d_logk || !d_poro) return fail(c, EREM_EINVAL, "logk and poro are required");
  if (!(lambda > 0) || !(rhoc_s >= 0)) return fail(c, EREM_EINVAL, "lambda must be > 0, rhoc_s >= 0");
  const size_t bytes = sizeof(double) * c->d.N;
  HIP_TRY(c, hipMemcpyAsync(c->logk, d_logk, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->poro, d_poro, bytes, hipMemcpyDeviceToDevice, c->stream));
  c->ph.lam = lambda;
  c->ph.rhoc_s = rhoc_s;
  c->rock_set = true;
  return EREM_OK;
}

int erem_set_fluid(erem_ctx* c, int32_t law, double c_f, double mu0, double rho0) {
  if (!c) return EREM_EINVAL;
  if (law != EREM_LAW_CONSTANT && law != EREM_LAW_WATER) return fail(c, EREM_EINVAL, "unknown law");
  if (!(c_f > 0) || !(mu0 > 0) || !(rho0 > 0)) return fail(c, EREM_EINVAL, "c_f, mu0, rho0 must be > 0");
  c->ph.law = law;
  c->ph.c_f = c_f;
  c->ph.mu0 = mu0;
  c->ph.rho0 = rho0;
  c->fluid_set = true;
  return EREM_OK;
}

int erem_set_bc(erem_ctx* c, double p_left, double p_right, double T_left, double T_right,
                int32_t dirichlet_left) {
  if (!c) return EREM_EINVAL;
  if (!std::isfinite(p_left) || !std::isfinite(p_right) || !std::isfinite(T_left) || !std::isfinite(T_right))
    return fail(c, EREM_EINVAL, "boundary values must be finite");
  c->ph.p_left = p_left;
  c->ph.p_right = p_right;
  c->ph.T_left = T_left;
  c->ph.T_right = T_right;
  c->ph.dirichlet_left = dirichlet_left ? 1 : 0;
  c->bc_set = true;
  return EREM_OK;
}

int erem_assemble_transmissibilities(erem_ctx* c, const double* d_T) {
  if (!c) return EREM_EINVAL;
  if (!c->rock_set) return fail(c, EREM_EINVAL, "erem_set_rock must come first");
  HIP_TRY(c, launch_transmissibility(c->d, c->ph, c->logk, d_T, c->tx, c->ty, c->tz, c->stream));
  c->trans_set = true;
  return EREM_OK;
}

int erem_solve_pressure(erem_ctx* c, double rtol, int32_t max_iter, int32_t warm, double* d_p, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  if (!c->trans_set) return fail(c, EREM_EINVAL, "erem_assemble_transmissibilities must come first");
  if (!(rtol > 0) || max_iter < 1) return fail(c, EREM_EINVAL, "rtol must be > 0 and max_iter >= 1");
  const Dims& d = c->d;
  const size_t bytes = sizeof(double) * d.N;
  if (warm && d_p) HIP_TRY(c, hipMemcpyAsync(c->pres, d_p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (!warm) HIP_TRY(c, hipMemsetAsync(c->pres, 0, bytes, c->stream));
  if (!warm || d_p) HIP_TRY(c, hipMemsetAsync(c->pres_lo, 0, bytes, c->stream));
  if (warm == 2 && !d_p) {
    // linear extrapolation from the last two solutions (first call: keep p^n)
    if (!c->pres_prev && dev_alloc(c, &c->pres_prev, d.N)) return EREM_ENOMEM;
    HIP_TRY(c, launch_pressure_extrapolate(d, c->pres, c->pres_lo, c->pres_prev, c->pres_prev_set ? 1 : 0,
                                           c->stream));
    c->pres_prev_set = true;
  } else {
    c->pres_prev_set = false;
  }
  // Iterative refinement: residual of the double-double pressure, PCG on the
  // correction to the reduction the tolerance still needs (at most 1e-12 per
  // correction), double-double update.
  int total = 0;
  bool ok = false;
  double relres = NAN;
  // The multigrid setup (coarse operators, bottom inverse) follows the first
  // residual readback on the stream, and the host waits for the readback
  // only: the device builds the hierarchy while the host reads the residual
  // and enqueues the iterations, which queue behind it.  The residual does
  // not read the hierarchy.
  bool setup_pending = c->use_mg;
  if (setup_pending && !c->ev_setup) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_setup, hipEventDisableTiming));
  for (int outer = 0; outer < 8; ++outer) {
    HIP_TRY(c, launch_pcg_reset(c->pcg, 0.0, c->stream));
    HIP_TRY(c, launch_dd_residual(d, c->ph, c->tx, c->ty, c->tz, c->pres, c->pres_lo, c->prhs, c->pcg, c->stream));
    {
      const int rc = enqueue_residual_readback(c);
      if (rc) return rc;
    }
    if (setup_pending) {
      HIP_TRY(c, hipEventRecord(c->ev_setup, c->stream));
      HIP_TRY(c, mg_setup(c->mg, c->stream));
      setup_pending = false;
      HIP_TRY(c, hipEventSynchronize(c->ev_setup));
    } else {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    double rr = 0.0, bb = 0.0;
    residual_sums(c, &rr, &bb);
    if (!std::isfinite(rr)) return fail(c, EREM_ENONFINITE, "non-finite pressure residual");
    relres = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    if (relres <= rtol || rr == 0.0) { ok = true; break; }
    if (total >= max_iter) break;
    int it = 0;
    bool done = false;
    {
      const int rc = pcg_inner(c, inner_tolerance(relres, rtol), max_iter - total, &it, &done,
                               &c->pcg_last[0][std::min(outer, 3)]);
      if (rc) return rc;
    }
    total += it;
    HIP_TRY(c, launch_dd_update(d, c->pres, c->pres_lo, c->pdelta, c->stream));
    if (!done) {
      // the iteration cap was reached inside this correction; check the
      // residual once more and stop
      if (total >= max_iter) continue;
    }
  }
  if (stats) { stats->iterations = total; stats->est_err = relres; }
  if (!ok) return fail(c, EREM_ENOCONV, "pressure solve did not reach rtol within max_iter");
  HIP_TRY(c, launch_face_fluxes_dd(d, c->ph, c->pres, c->pres_lo, c->tx, c->ty, c->tz, c->fx, c->fy, c->fz,
                                   c->stream));
  if (d_p) HIP_TRY(c, hipMemcpyAsync(d_p, c->pres, bytes, hipMemcpyDeviceToDevice, c->stream));
  c->flux_set = true;
  return EREM_OK;
}

int erem_set_face_fluxes(erem_ctx* c, const double* d_fx, const double* d_fy, const double* d_fz) {
  if (!c) return EREM_EINVAL;
  if (!d_fx || !d_fy || (c->d.dim == 3 && !d_fz)) return fail(c, EREM_EINVAL, "flux arrays missing");
  HIP_TRY(c, hipMemcpyAsync(c->fx, d_fx, c->nfx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->fy, d_fy, c->nfy * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (d_fz) HIP_TRY(c, hipMemcpyAsync(c->fz, d_fz, c->nfz * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  else HIP_TRY(c, hipMemsetAsync(c->fz, 0, c->nfz * sizeof(double), c->stream));
  c->flux_set = true;
  return EREM_OK;
}

int erem_get_faces(erem_ctx* c, double* d_fx, double* d_fy, double* d_fz, double* d_tx, double* d_ty,
                   double* d_tz) {
  if (!c) return EREM_EINVAL;
  struct { double* dst; const double* src; size_t n; } cp[] = {
      {d_fx, c->fx, c->nfx}, {d_fy, c->fy, c->nfy}, {d_fz, c->fz, c->nfz},
      {d_tx, c->tx, c->nfx}, {d_ty, c->ty, c->nfy}, {d_tz, c->tz, c->nfz}};
  for (auto& e : cp)
    if (e.dst) HIP_TRY(c, hipMemcpyAsync(e.dst, e.src, e.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return EREM_OK;
}

int erem_form_jacobian(erem_ctx* c, const double* d_T) {
  if (!c) return EREM_EINVAL;
  if (!d_T) return fail(c, EREM_EINVAL, "T is NULL");
  if (!c->rock_set || !c->flux_set) return fail(c, EREM_EINVAL, "rock and face fluxes must be set first");
  HIP_TRY(c, launch_reset_reduce(c->red, c->stream));
  HIP_TRY(c, launch_assemble(c->d, c->ph, c->poro, c->fx, c->fy, c->fz, d_T, c->coef, c->F, c->red, c->stream));
  c->jac_set = true;
  c->op_pressure = false;
  c->coef32_valid = false;
  return EREM_OK;
}

int erem_get_jacobian(erem_ctx* c, double* d_coef, double* d_F) {
  if (!c) return EREM_EINVAL;
  if (!c->jac_set) return fail(c, EREM_EINVAL, "erem_form_jacobian must come first");
  if (c->op_pressure) return fail(c, EREM_EINVAL, kHoldsPressure);
  const size_t n = c->d.N;
  if (d_coef) HIP_TRY(c, hipMemcpyAsync(d_coef, c->coef, n * ndir(c) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (d_F) HIP_TRY(c, hipMemcpyAsync(d_F, c->F, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return EREM_OK;
}

int erem_phi1_apply(erem_ctx* c, double h, const double* d_v, double* d_out, const erem_opts* o, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!d_v || !d_out || d_v == d_out) return fail(c, EREM_EINVAL, "v and out must be distinct non-NULL");
  if (!c->jac_set) return fail(c, EREM_EINVAL, "erem_form_jacobian must come first");
  if (c->op_pressure) return fail(c, EREM_EINVAL, kHoldsPressure);
  if (!(h > 0) || !std::isfinite(h)) return fail(c, EREM_EINVAL, "h must be > 0");
  if (o->method == EREM_METHOD_KRYLOV && o->precision != EREM_PREC_FP64)
    return fail(c, EREM_EINVAL, "the Krylov method runs in FP64 only");
  // max |v| (the Gershgorin interval of the last assembly is kept)
  HIP_TRY(c, launch_absmax(c->d, d_v, c->red, c->stream));
  rc = read_reduce(c);
  if (rc) return rc;
  const double vmax = slot_max(c->h_red->vmax);
  const double scal = o->tol_a + o->tol_r * h * vmax;
  if (vmax == 0.0) {
    HIP_TRY(c, hipMemsetAsync(d_out, 0, sizeof(double) * c->d.N, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (stats) { std::memset(stats, 0, sizeof(*stats)); stats->alpha = c->alpha; stats->beta = c->beta; }
    return EREM_OK;
  }
  rc = hphi1_eval(c, h, d_v, nullptr, scal, o, stats);
  if (rc) return rc;
  HIP_TRY(c, launch_axpby(c->d, d_out, 0.0, c->u, 1.0 / h, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return EREM_OK;
}

int erem_set_jacobian(erem_ctx* c, const double* d_coef, const double* d_F) {
  if (!c) return EREM_EINVAL;
  if (!d_coef || !d_F) return fail(c, EREM_EINVAL, "coef and F are required");
  const size_t n = c->d.N;
  HIP_TRY(c, hipMemcpyAsync(c->coef, d_coef, n * ndir(c) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->F, d_F, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, launch_gershgorin(c->d, c->coef, c->red, c->stream));
  c->jac_set = true;
  c->op_pressure = false;
  c->coef32_valid = false;
  return EREM_OK;
}

namespace {

int step_checks(erem_ctx* c, double h, double* d_T, const erem_opts* o) {
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!d_T) return fail(c, EREM_EINVAL, "T is NULL");
  if (!(h > 0) || !std::isfinite(h)) return fail(c, EREM_EINVAL, "h must be > 0");
  if (o->method == EREM_METHOD_KRYLOV && o->precision != EREM_PREC_FP64)
    return fail(c, EREM_EINVAL, "the Krylov method runs in FP64 only");
  return EREM_OK;
}

// T += h phi1(h J) F (+ h^2 phi2(h J) g when g is not null) with the
// context's J, F and interval; tmax = ||T||_inf.
int step_core(erem_ctx* c, double h, double* d_T, const erem_opts* o, erem_stats* stats, double tmax,
              const double* g = nullptr) {
  if (!std::isfinite(tmax)) return fail(c, EREM_ENONFINITE, "non-finite temperature");
  const double scal = o->tol_a + o->tol_r * tmax;
  if (!(scal > 0)) return fail(c, EREM_EINVAL, "error scale is zero (tol_a = 0 and T = 0)");
  int rc = hphi1_eval(c, h, c->F, g, scal, o, stats);
  if (rc) return rc;
  HIP_TRY(c, launch_axpby(c->d, d_T, 1.0, c->u, 1.0, c->stream));
  return EREM_OK;
}

}  // namespace

int erem_step(erem_ctx* c, double h, double* d_T, const erem_opts* o, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = step_checks(c, h, d_T, o);
  if (rc) return rc;
  rc = erem_form_jacobian(c, d_T);
  if (rc) return rc;
  rc = step_predicted(c, h, d_T, o, stats);
  if (rc != kFallback) return rc;
  rc = read_reduce(c);
  if (rc) return rc;
  return step_core(c, h, d_T, o, stats, c->tmax);
}

int erem_step_nonautonomous(erem_ctx* c, double h, double T_left, double T_right, double dT_left_dt,
                            double dT_right_dt, double* d_T, const erem_opts* o, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = step_checks(c, h, d_T, o);
  if (rc) return rc;
  if (o->method != EREM_METHOD_LEJA) return fail(c, EREM_EINVAL, "the non-autonomous step runs with the Leja method");
  if (!std::isfinite(T_left) || !std::isfinite(T_right) || !std::isfinite(dT_left_dt) || !std::isfinite(dT_right_dt))
    return fail(c, EREM_EINVAL, "boundary temperatures and their rates must be finite");
  if (!c->gt) {
    rc = dev_alloc(c, &c->gt, c->d.N);
    if (!rc) rc = dev_alloc(c, &c->zt, c->d.N);
    if (rc) return EREM_ENOMEM;
  }
  c->ph.T_left = T_left;
  c->ph.T_right = T_right;
  rc = erem_form_jacobian(c, d_T);
  if (rc) return rc;
  HIP_TRY(c, launch_time_rate(c->d, c->ph, c->poro, c->fx, d_T, dT_left_dt, dT_right_dt, c->gt, c->stream));
  rc = read_reduce(c);
  if (rc) return rc;
  return step_core(c, h, d_T, o, stats, c->tmax, c->gt);
}

int erem_face_fluxes_from_pressure(erem_ctx* c, const double* d_p) {
  if (!c) return EREM_EINVAL;
  if (!d_p) return fail(c, EREM_EINVAL, "p is NULL");
  if (!c->trans_set) return fail(c, EREM_EINVAL, "erem_assemble_transmissibilities must come first");
  HIP_TRY(c, launch_face_fluxes(c->d, c->ph, d_p, c->tx, c->ty, c->tz, c->fx, c->fy, c->fz, c->stream));
  c->flux_set = true;
  return EREM_OK;
}

int erem_step_pressure(erem_ctx* c, double h, double* d_p, const double* d_T, double alpha_b, double beta_f,
                       const erem_opts* o, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!d_p || !d_T) return fail(c, EREM_EINVAL, "p and T must be non-NULL");
  if (!(h > 0) || !std::isfinite(h)) return fail(c, EREM_EINVAL, "h must be > 0");
  if (!(alpha_b >= 0) || !(beta_f >= 0) || !(alpha_b + beta_f > 0) || !std::isfinite(alpha_b + beta_f))
    return fail(c, EREM_EINVAL, "alpha_b and beta_f must be >= 0, finite and not both 0");
  if (!c->trans_set) return fail(c, EREM_EINVAL, "erem_assemble_transmissibilities must come first");
  if (!c->jac_set) return fail(c, EREM_EINVAL, "G2 = dT/dt must be in the context (erem_form_jacobian or erem_step)");
  if (c->op_pressure)
    return fail(c, EREM_EINVAL, "G2 = dT/dt must be formed again (erem_form_jacobian or erem_step): the context holds "
                                "the pressure operator of the previous erem_step_pressure");
  if (o->method == EREM_METHOD_KRYLOV && o->precision != EREM_PREC_FP64)
    return fail(c, EREM_EINVAL, "the Krylov method runs in FP64 only");
  HIP_TRY(c, launch_pressure_ode(c->d, c->ph, c->poro, d_T, d_p, c->tx, c->ty, c->tz, alpha_b, beta_f, c->coef,
                                 c->F, c->red, c->stream));
  c->coef32_valid = false;
  c->op_pressure = true;
  // the pressure keeps its own Newton-degree and interval memory (the
  // temperature evaluations of the same steps need far fewer terms)
  std::swap(c->last_m, c->last_m_p);
  std::swap(c->last_w, c->last_w_p);
  rc = step_predicted(c, h, d_p, o, stats);
  if (rc == kFallback) {
    rc = read_reduce(c);
    if (!rc) rc = step_core(c, h, d_p, o, stats, c->tmax);
  }
  std::swap(c->last_m, c->last_m_p);
  std::swap(c->last_w, c->last_w_p);
  return rc;
}

int erem_step_frozen(erem_ctx* c, double h, double* d_T, const erem_opts* o, erem_stats* stats) {
  if (!c) return EREM_EINVAL;
  int rc = step_checks(c, h, d_T, o);
  if (rc) return rc;
  if (!c->jac_set) return fail(c, EREM_EINVAL, "no Jacobian in the context");
  if (c->op_pressure) return fail(c, EREM_EINVAL, kHoldsPressure);
  HIP_TRY(c, launch_absmax(c->d, d_T, c->red, c->stream));
  rc = read_reduce(c);
  if (rc) return rc;
  return step_core(c, h, d_T, o, stats, slot_max(c->h_red->vmax));
}

int erem_profile(erem_ctx* c, int32_t enable) {
  if (!c) return EREM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->prof = enable > 0 ? enable : 0;
  c->t_leja = c->t_pcg_a = c->t_pcg_b = c->t_mg = c->t_adj = c->t_bicg = 0.0;
  c->n_leja = c->n_pcg_a = c->n_pcg_b = c->n_mg = c->n_adj = c->n_bicg = 0;
  return EREM_OK;
}

int erem_profile_read(erem_ctx* c, erem_kernel_times* out) {
  if (!c || !out) return EREM_EINVAL;
  out->leja_term_ms = c->t_leja;
  out->leja_term_launches = c->n_leja;
  out->pcg_a_ms = c->t_pcg_a;
  out->pcg_a_launches = c->n_pcg_a;
  out->pcg_b_ms = c->t_pcg_b;
  out->pcg_b_launches = c->n_pcg_b;
  out->mg_ms = c->t_mg;
  out->mg_cycles = c->n_mg;
  out->adj_rev_ms = c->t_adj;
  out->adj_rev_launches = c->n_adj;
  out->bicg_ms = c->t_bicg;
  out->bicg_iterations = c->n_bicg;
  return EREM_OK;
}

int erem_set_pressure_preconditioner(erem_ctx* c, int32_t kind) {
  if (!c) return EREM_EINVAL;
  if (kind != EREM_PRECOND_JACOBI && kind != EREM_PRECOND_MULTIGRID)
    return fail(c, EREM_EINVAL, "unknown preconditioner");
  c->use_mg = kind == EREM_PRECOND_MULTIGRID;
  return EREM_OK;
}

int erem_leja_points(int32_t n, double* out) {
  if (n < 0 || n > kMaxTerms + 1 || (n > 0 && !out)) return EREM_EINVAL;
  std::vector<double> v;
  if (!leja_points(n, v)) return EREM_EINVAL;
  std::copy(v.begin(), v.end(), out);
  return EREM_OK;
}

int erem_phi2_divided_differences(double hc, double hg, const double* xi, int32_t n, double* out) {
  if (n < 0 || n > kMaxTerms + 1 || (n > 0 && (!xi || !out))) return EREM_EINVAL;
  if (!std::isfinite(hc) || !std::isfinite(hg)) return EREM_EINVAL;
  if (n == 0) return EREM_OK;
  phi_divided_differences(2, hc, hg, xi, n, out);
  return EREM_OK;
}

int erem_phi1_divided_differences(double hc, double hg, const double* xi, int32_t n, double* out) {
  if (n < 0 || n > kMaxTerms + 1 || (n > 0 && (!xi || !out))) return EREM_EINVAL;
  if (!std::isfinite(hc) || !std::isfinite(hg)) return EREM_EINVAL;
  if (n == 0) return EREM_OK;
  phi1_divided_differences(hc, hg, xi, n, out);
  return EREM_OK;
}

}  // extern "C"
