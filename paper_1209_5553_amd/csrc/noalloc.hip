// erem_phi1_apply_noalloc: out = phi1(h J) v for a caller's stencil J with
// every device buffer of the evaluation in one file-scope array, for callers
// that cannot allocate.  The operation is that of erem_set_jacobian followed
// by erem_phi1_apply (Sec. 4.2: Gershgorin interval, real Leja points,
// divided differences, Newton form with the scaled-norm stop test, substeps),
// in FP64, on the same kernels; only the host driver and the home of the
// scratch buffers differ.
#include "erem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "device.h"
#include "host_numerics.h"
#include "leja.h"

namespace erem {
namespace {

// Limits of the allocation-free evaluation.
constexpr long long kNaMaxCells = 1ll << 18;  // 262 144 cells (512 x 512, 64^3)
constexpr int kNaMaxBlocks = 16384;           // 64 x 4 cell blocks of the grid
constexpr int kNaMaxTerms = 256;              // m_max
constexpr int kNaSubsteps = 64;               // stop-state slots (max substeps)

// Scratch layout, in doubles: five vectors of kNaMaxCells (q, q', p, u, w),
// the term partials (kLejaRing slots per block), the Newton coefficients, the
// stop states, the reduction targets.
constexpr size_t kNaVec = static_cast<size_t>(kNaMaxCells);
constexpr size_t kNaPart = static_cast<size_t>(kLejaRing) * kNaMaxBlocks;
constexpr size_t kNaCoefWords = (sizeof(LejaCoef) + 255) / 256 * 32;
constexpr size_t kNaStateWords = (sizeof(LejaState) * kNaSubsteps + 255) / 256 * 32;
constexpr size_t kNaRedWords = (sizeof(AsmReduce) + 255) / 256 * 32;
constexpr size_t kNaWords = 5 * kNaVec + kNaPart + kNaCoefWords + kNaStateWords + kNaRedWords;

// The scratch buffer: one copy per GPU, held until the process ends.  Host
// code never uses this name as an address: it uses the device pointer that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNaWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // scratch address per device
double g_xi[kMaxLeja];           // real Leja points (host)
bool g_xi_set = false;
// host workspace of the divided differences (guarded by g_mu)
double g_ddw[2 * (kNaMaxTerms + 2) + 2 * (kNaMaxTerms + 2) * (kNaMaxTerms + 2)];

// Set-up, once per device with that device current: the scratch address,
// and once per process the Leja points.
int setup(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EREM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_xi_set) {
    std::vector<double> xi;
    if (!leja_points(kNaMaxTerms + 1, xi)) return EREM_EINVAL;
    std::copy(xi.begin(), xi.end(), g_xi);
    g_xi_set = true;
  }
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EREM_EDEVICE;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return EREM_OK;
}

struct NaBufs {
  double *qa, *qb, *p, *u, *w, *part;
  LejaCoef* cf;
  LejaState* states;
  AsmReduce* red;
};

NaBufs carve(double* base) {
  NaBufs b{};
  b.qa = base;
  b.qb = base + kNaVec;
  b.p = base + 2 * kNaVec;
  b.u = base + 3 * kNaVec;
  b.w = base + 4 * kNaVec;
  b.part = base + 5 * kNaVec;
  double* rest = b.part + kNaPart;
  b.cf = reinterpret_cast<LejaCoef*>(rest);
  b.states = reinterpret_cast<LejaState*>(rest + kNaCoefWords);
  b.red = reinterpret_cast<AsmReduce*>(rest + kNaCoefWords + kNaStateWords);
  return b;
}

#define NA_TRY(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return EREM_EDEVICE; \
  } while (0)

int terms_per_launch(const Dims& d, int k, int K) {
  if (d.dim != 2) return 1;
  if (k + 3 <= K) return 4;
  return k + 1 <= K ? 2 : 1;
}

// u <- h phi1(h J) v by s substeps of delta = h / s, at most K Newton terms
// each: u_{j+1} = u_j + delta phi1(delta J)(v + J u_j).  EREM_ENOCONV when a
// substep did not stop within K terms.
int leja_eval(const Dims& d, const NaBufs& B, const double* coef, const double* v, double h, double alpha,
              double beta, double scal, int s, int K, int p_order, hipStream_t st, int* m_used, double* est_last) {
  const double cc = 0.5 * (alpha + beta), gg = 0.25 * (beta - alpha);
  const double delta = h / s;
  const int n = K + 1;
  const double rootN = std::sqrt(static_cast<double>(d.N));
  LejaCoef hc;  // host copy of the coefficient block
  std::memset(&hc, 0, sizeof(hc));
  {
    std::lock_guard<std::mutex> lock(g_mu);
    phi_divided_differences_ws(1, delta * cc, delta * gg, g_xi, n, hc.dk, g_ddw);
  }
  hc.inv_g = 1.0 / gg;
  hc.thresh = std::pow(10.0, -p_order);
  for (int k = 0; k < n; ++k) {
    hc.shift[k] = (k > 0) ? cc / gg + g_xi[k - 1] : 0.0;
    hc.estf[k] = std::fabs(delta * hc.dk[k]) / (rootN * scal);
  }
  NA_TRY(hipMemcpyAsync(B.cf, &hc, sizeof(LejaCoef), hipMemcpyHostToDevice, st));
  NA_TRY(launch_leja_reset(B.states, s, K, st));
  for (int j = 0; j < s; ++j) {
    LejaState* sj = B.states + j;
    const double* src = v;
    if (j > 0) {
      NA_TRY(launch_stencil_axpy(d, coef, v, B.u, B.w, st));
      src = B.w;
    }
    NA_TRY(launch_leja_init<double>(d, B.cf, src, B.qa, B.p, B.part, st));
    int prev = -1;
    double* cur = B.qa;
    double* oth = B.qb;
    for (int k = 1; k <= K;) {
      const int nt = terms_per_launch(d, k, K);
      if (nt > 1)
        NA_TRY(launch_leja_terms<double>(d, B.cf, coef, cur, oth, B.p, sj, B.part, k, nt, st));
      else
        NA_TRY(launch_leja_term<double>(d, B.cf, coef, cur, oth, B.p, sj, B.part, k, st));
      std::swap(cur, oth);
      k += nt;
      const int last = k - 1;
      if (last % kCheckEvery == 0 || last == K) {
        NA_TRY(launch_leja_check(d, B.cf, sj, B.part, prev + 1, last, st));
        prev = last;
      }
    }
    NA_TRY(launch_substep_update<double>(d, B.u, B.p, delta, j == 0 ? 1 : 0, st));
  }
  // the hc copy must outlive the transfer; the stop states come back here
  NA_TRY(hipStreamSynchronize(st));
  int total = 0;
  double last = 0.0;
  const size_t hdr = offsetof(LejaState, sums);
  for (int j = 0; j < s; ++j) {
    LejaState hs;
    NA_TRY(hipMemcpyAsync(&hs, B.states + j, hdr + sizeof(double) * (K + 1), hipMemcpyDeviceToHost, st));
    NA_TRY(hipStreamSynchronize(st));
    if (hs.nonfinite) return EREM_ENONFINITE;
    if (hs.stopped < 0) return EREM_ENOCONV;
    total += std::min(K, ((hs.stopped + kCheckEvery - 1) / kCheckEvery) * kCheckEvery);
    if (j + 1 == s) last = hc.estf[hs.stopped] * std::sqrt(hs.sums[hs.stopped]);
  }
  *m_used = total;
  *est_last = last;
  return EREM_OK;
}

}  // namespace
}  // namespace erem

using namespace erem;

extern "C" int erem_phi1_apply_noalloc(const erem_grid* g, const double* d_coef, double h, const double* d_v,
                                       double* d_out, const erem_opts* o, void* stream, erem_stats* stats) {
  if (!g || !d_coef || !d_v || !d_out || !o || d_v == d_out) return EREM_EINVAL;
  if (!(g->dim == 2 && g->nz == 1) && g->dim != 3) return EREM_EINVAL;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return EREM_EINVAL;
  if (g->nx > kNaMaxCells || g->ny > kNaMaxCells || g->nz > kNaMaxCells) return EREM_EINVAL;
  const long long N = g->nx * g->ny * g->nz;
  if (N > kNaMaxCells) return EREM_EINVAL;
  if (!(h > 0) || !std::isfinite(h)) return EREM_EINVAL;
  if (o->method != EREM_METHOD_LEJA || o->precision != EREM_PREC_FP64) return EREM_EINVAL;
  if (o->m_max < 5 || o->m_max > kNaMaxTerms || o->max_substeps < 1) return EREM_EINVAL;
  if (!(o->tol_a >= 0) || !(o->tol_r >= 0) || (o->tol_a == 0 && o->tol_r == 0) || o->p_order < 0 ||
      o->p_order > 15 || !(o->rho_max >= 0))
    return EREM_EINVAL;
  Dims d{};
  d.nx = static_cast<int>(g->nx);
  d.ny = static_cast<int>(g->ny);
  d.nz = static_cast<int>(g->nz);
  d.dim = g->dim;
  d.N = static_cast<int>(N);
  d.dx = g->dx;
  d.dy = g->dy;
  d.dz = g->dz;
  if (leja_num_blocks(d) > kNaMaxBlocks) return EREM_EINVAL;
  double* base = nullptr;
  int rc = setup(&base);
  if (rc) return rc;
  const NaBufs B = carve(base);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Gershgorin interval of J and max |v| (reduction targets reset by the launchers)
  NA_TRY(launch_gershgorin(d, d_coef, B.red, st));
  NA_TRY(launch_absmax(d, d_v, B.red, st));
  AsmReduce hr;
  NA_TRY(hipMemcpyAsync(&hr, B.red, sizeof(AsmReduce), hipMemcpyDeviceToHost, st));
  NA_TRY(hipStreamSynchronize(st));
  const double alpha = slot_min(hr.lo), beta = slot_max(hr.hi), vmax = slot_max(hr.vmax);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->alpha = alpha;
    stats->beta = beta;
  }
  if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(vmax)) return EREM_ENONFINITE;
  if (vmax == 0.0) {
    NA_TRY(hipMemsetAsync(d_out, 0, sizeof(double) * N, st));
    NA_TRY(hipStreamSynchronize(st));
    return EREM_OK;
  }
  const double scal = o->tol_a + o->tol_r * h * vmax;
  const double width = beta - alpha;
  const double mag = std::max(std::fabs(alpha), std::fabs(beta));
  if (width <= 1e-14 * mag || width == 0.0) {
    // degenerate interval: J = c I, phi1(h J) v = phi1(h c) v
    const double z = h * 0.5 * (alpha + beta);
    const double f = (z == 0.0) ? 1.0 : std::expm1(z) / z;
    NA_TRY(launch_axpby(d, d_out, 0.0, d_v, f, st));
    NA_TRY(hipStreamSynchronize(st));
    if (stats) stats->substeps = 1;
    return EREM_OK;
  }
  const int smax = std::min(o->max_substeps, kNaSubsteps);
  int s = 1;
  if (o->rho_max > 0.0) s = std::max(1, static_cast<int>(std::ceil(h * width / o->rho_max)));
  if (s > smax) s = smax;
  int K = o->chunk > 0 ? std::min(o->chunk, o->m_max) : o->m_max;
  int restarts = 0;
  for (;;) {
    int m_used = 0;
    double est = 0.0;
    rc = leja_eval(d, B, d_coef, d_v, h, alpha, beta, scal, s, K, o->p_order, st, &m_used, &est);
    if (rc == EREM_OK) {
      NA_TRY(launch_axpby(d, d_out, 0.0, B.u, 1.0 / h, st));
      NA_TRY(hipStreamSynchronize(st));
      if (stats) {
        stats->m_total = m_used;
        stats->substeps = s;
        stats->est_err = est;
        stats->restarts = restarts;
      }
      return EREM_OK;
    }
    if (rc != EREM_ENOCONV) return rc;
    ++restarts;
    if (K < o->m_max) {
      K = o->m_max;
    } else if (2 * s <= smax) {
      s *= 2;
    } else {
      return EREM_ENOCONV;
    }
  }
}
