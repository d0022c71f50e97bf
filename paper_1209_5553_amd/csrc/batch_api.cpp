// C ABI of the batched form (erem_batch_*): per-problem setup through the
// single-problem path, packing, per-problem Leja data, and the one launch of
// batch.hip that runs every problem for all steps (optionally captured in a
// hipGraph).
#include "erem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "batch.h"
#include "device.h"
#include "host_numerics.h"
#include "leja.h"

using namespace erem;

struct erem_batch {
  hipStream_t stream = nullptr;
  int device = 0;
  int nprob = 0;
  std::vector<erem_grid> grids;
  std::vector<long long> off;  // nprob + 1
  long long ntot = 0;
  std::vector<double> alpha, beta;
  std::vector<char> set;
  // device arrays
  double *coef = nullptr, *g = nullptr, *v = nullptr, *u = nullptr, *q0 = nullptr, *q1 = nullptr, *p = nullptr;
  float* coef32 = nullptr;
  double *dk = nullptr, *shift = nullptr, *tscratch = nullptr;
  BProb* prob = nullptr;
  int* order = nullptr;  // largest problem first
  BDyn* dyn = nullptr;
  // prepared state
  bool prepared = false;
  int fp32 = 0, m_max = 0;
  double tol_a = 0.0, tol_r = 1e-12, thresh = 1e-2;
  int shape = 3;  // 1024 threads x 2 cells: fastest on the 256-realisation workload
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (nsteps, shape) -> graph
  const double* graph_T = nullptr;                       // T array the graphs were captured with
  // per-size single-problem contexts used for setup
  std::map<std::pair<long long, long long>, erem_ctx*> ctxs;
  double *tmp_coef = nullptr, *tmp_F = nullptr;
  size_t tmp_n = 0;
  AsmReduce* red = nullptr;
  AsmReduce* h_red = nullptr;
  std::string err;
};

namespace {

int bfail(erem_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define BHIP(b, expr)                                                                         \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) return bfail((b), EREM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

template <class T>
int balloc(erem_batch* b, T** p, size_t n) {
  if (n == 0) n = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess)
    return bfail(b, EREM_ENOMEM, "hipMalloc failed");
  return EREM_OK;
}

void free_batch(erem_batch* b) {
  double** d[] = {&b->coef, &b->g, &b->v, &b->u, &b->q0, &b->q1, &b->p, &b->dk, &b->shift,
                  &b->tscratch, &b->tmp_coef, &b->tmp_F};
  for (double** x : d)
    if (*x) { (void)hipFree(*x); *x = nullptr; }
  if (b->coef32) (void)hipFree(b->coef32);
  if (b->prob) (void)hipFree(b->prob);
  if (b->order) (void)hipFree(b->order);
  if (b->dyn) (void)hipFree(b->dyn);
  if (b->red) (void)hipFree(b->red);
  if (b->h_red) (void)hipHostFree(b->h_red);
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  for (auto& kv : b->ctxs) erem_destroy(kv.second);
  b->ctxs.clear();
}

void drop_graphs(erem_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

BatchArgs make_args(erem_batch* b, double* T, int nsteps) {
  BatchArgs a{};
  a.prob = b->prob;
  a.dyn = b->dyn;
  a.order = b->order;
  a.coef64 = b->coef;
  a.coef = b->fp32 ? static_cast<const void*>(b->coef32) : static_cast<const void*>(b->coef);
  a.g = b->g;
  a.T = T;
  a.v = b->v;
  a.u = b->u;
  a.q0 = b->q0;
  a.q1 = b->q1;
  a.p = b->p;
  a.dk = b->dk;
  a.shift = b->shift;
  a.ntot = b->ntot;
  a.nprob = b->nprob;
  a.nsteps = nsteps;
  a.m_max = b->m_max;
  a.tol_a = b->tol_a;
  a.tol_r = b->tol_r;
  a.thresh = b->thresh;
  return a;
}

// One workgroup per problem; the hardware hands the next (smaller) problem to
// a CU as soon as one finishes, so the largest-first order balances the load.
int grid_size(erem_batch* b) { return std::min(b->nprob, 1 << 20); }

// One launch (optionally through a cached graph).  Synchronises the stream.
int launch(erem_batch* b, double* T, int nsteps, bool use_graph, erem_batch_stats* st) {
  const BatchArgs a = make_args(b, T, nsteps);
  const int grid = grid_size(b);
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  bool graphed = false;
  BHIP(b, hipEventRecord(e0, b->stream));
  if (use_graph) {
    const auto key = std::make_pair(nsteps, b->shape);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      hipGraph_t graph;
      hipGraphExec_t exec;
      bool ok = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const hipError_t le = batch_launch(a, b->shape, b->fp32, grid, b->stream);
        const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
        ok = le == hipSuccess && ce == hipSuccess;
        if (ok) {
          ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
          (void)hipGraphDestroy(graph);
        }
      }
      (void)hipGetLastError();
      if (ok) it = b->graphs.emplace(key, exec).first;
    }
    if (it != b->graphs.end()) {
      // the captured launch holds T's pointer: replay only for the same array
      BHIP(b, hipGraphLaunch(it->second, b->stream));
      graphed = true;
    }
  }
  if (!graphed) BHIP(b, batch_launch(a, b->shape, b->fp32, grid, b->stream));
  BHIP(b, hipEventRecord(e1, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::vector<BDyn> dyn(b->nprob);
  BHIP(b, hipMemcpy(dyn.data(), b->dyn, sizeof(BDyn) * b->nprob, hipMemcpyDeviceToHost));
  long long tot = 0;
  int tmin = 1 << 30, tmax = 0, failed = 0, flags = 0;
  double bytes = 0.0;
  const double per_cell = b->fp32 ? 36.0 : 72.0;  // 5 coef + q_in + p rd/wr + q_out
  for (int i = 0; i < b->nprob; ++i) {
    const BDyn& d = dyn[i];
    bytes += per_cell * static_cast<double>(d.terms) * static_cast<double>(b->off[i + 1] - b->off[i]);
    tot += d.terms;
    tmin = std::min(tmin, d.terms);
    tmax = std::max(tmax, d.terms);
    if (d.flags || d.step < nsteps) ++failed;
    flags |= d.flags;
  }
  if (st) {
    st->terms_total = tot;
    st->terms_min = b->nprob ? tmin : 0;
    st->terms_max = tmax;
    st->failed = failed;
    st->tile_shape = b->shape;
    st->graph = graphed ? 1 : 0;
    st->grid = grid;
    st->ms = ms;
    st->leja_bytes = bytes;
  }
  if (flags & 2) return bfail(b, EREM_ENONFINITE, "non-finite Leja norm in a batch problem");
  if (failed) return bfail(b, EREM_ENOCONV, "a batch problem did not converge within m_max terms");
  return EREM_OK;
}

}  // namespace

extern "C" {

int erem_batch_create(int32_t nprob, const erem_grid* grids, void* stream, erem_batch** out) {
  if (!out) return EREM_EINVAL;
  *out = nullptr;
  if (nprob < 1 || nprob > (1 << 20) || !grids) return EREM_EINVAL;
  for (int i = 0; i < nprob; ++i) {
    const erem_grid& g = grids[i];
    if (g.dim != 2 || g.nz != 1 || g.nx < 1 || g.ny < 1 || g.nx > 65536 || g.ny > 65536) return EREM_EINVAL;
    if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0)) return EREM_EINVAL;
  }
  erem_batch* b = new (std::nothrow) erem_batch();
  if (!b) return EREM_ENOMEM;
  b->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return EREM_EDEVICE;
  }
  b->nprob = nprob;
  b->grids.assign(grids, grids + nprob);
  b->off.assign(nprob + 1, 0);
  for (int i = 0; i < nprob; ++i) b->off[i + 1] = b->off[i] + grids[i].nx * grids[i].ny;
  b->ntot = b->off[nprob];
  if (b->ntot > (1ll << 31)) { delete b; return EREM_EINVAL; }
  b->alpha.assign(nprob, 0.0);
  b->beta.assign(nprob, 0.0);
  b->set.assign(nprob, 0);
  const size_t n = static_cast<size_t>(b->ntot);
  int rc = EREM_OK;
  rc |= balloc(b, &b->coef, 5 * n);
  rc |= balloc(b, &b->g, n);
  rc |= balloc(b, &b->v, n);
  rc |= balloc(b, &b->u, n);
  rc |= balloc(b, &b->q0, n);
  rc |= balloc(b, &b->q1, n);
  rc |= balloc(b, &b->p, n);
  rc |= balloc(b, &b->tscratch, n);
  rc |= balloc(b, &b->dyn, nprob);
  rc |= balloc(b, &b->prob, nprob);
  rc |= balloc(b, &b->order, nprob);
  rc |= balloc(b, &b->red, 1);
  if (rc == EREM_OK && hipHostMalloc(reinterpret_cast<void**>(&b->h_red), sizeof(AsmReduce), hipHostMallocDefault) != hipSuccess)
    rc = EREM_ENOMEM;
  if (rc == EREM_OK) {
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->off[x + 1] - b->off[x] > b->off[y + 1] - b->off[y]; });
    if (hipMemcpy(b->order, order.data(), sizeof(int) * nprob, hipMemcpyHostToDevice) != hipSuccess) rc = EREM_EDEVICE;
  }
  if (rc != EREM_OK) {
    free_batch(b);
    delete b;
    return rc < 0 ? rc : EREM_ENOMEM;
  }
  *out = b;
  return EREM_OK;
}

int erem_batch_destroy(erem_batch* b) {
  if (!b) return EREM_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  delete b;
  return EREM_OK;
}

const char* erem_batch_last_error(const erem_batch* b) { return b ? b->err.c_str() : "NULL batch"; }

int erem_batch_offsets(const erem_batch* b, int64_t* out) {
  if (!b || !out) return EREM_EINVAL;
  for (int i = 0; i <= b->nprob; ++i) out[i] = b->off[i];
  return EREM_OK;
}

int erem_batch_set_problem(erem_batch* b, int32_t i, const double* d_logk, const double* d_poro, double lambda,
                           double rhoc_s, double c_f, double mu0, double rho0, double p_left, double p_right,
                           double T_left, double T_right, const double* d_T0) {
  if (!b) return EREM_EINVAL;
  if (i < 0 || i >= b->nprob || !d_logk || !d_poro || !d_T0) return bfail(b, EREM_EINVAL, "bad problem index or NULL array");
  const erem_grid& g = b->grids[i];
  const auto key = std::make_pair(static_cast<long long>(g.nx), static_cast<long long>(g.ny));
  erem_ctx* ctx = nullptr;
  auto it = b->ctxs.find(key);
  if (it == b->ctxs.end()) {
    const int rc = erem_create(&g, b->stream, &ctx);
    if (rc) return bfail(b, rc, "cannot create the setup context");
    b->ctxs.emplace(key, ctx);
  } else {
    ctx = it->second;
  }
  const size_t N = static_cast<size_t>(g.nx * g.ny);
  if (b->tmp_n < N) {
    if (b->tmp_coef) (void)hipFree(b->tmp_coef);
    if (b->tmp_F) (void)hipFree(b->tmp_F);
    b->tmp_coef = b->tmp_F = nullptr;
    if (balloc(b, &b->tmp_coef, 5 * N) || balloc(b, &b->tmp_F, N)) return EREM_ENOMEM;
    b->tmp_n = N;
  }
  int rc = erem_set_rock(ctx, d_logk, d_poro, lambda, rhoc_s);
  if (!rc) rc = erem_set_fluid(ctx, EREM_LAW_CONSTANT, c_f, mu0, rho0);
  if (!rc) rc = erem_set_bc(ctx, p_left, p_right, T_left, T_right, 1);
  if (!rc) rc = erem_assemble_transmissibilities(ctx, nullptr);
  erem_stats st{};
  if (!rc) rc = erem_solve_pressure(ctx, 1e-16, 50000, 0, nullptr, &st);
  if (!rc) rc = erem_form_jacobian(ctx, d_T0);
  if (!rc) rc = erem_get_jacobian(ctx, b->tmp_coef, b->tmp_F);
  if (rc) return bfail(b, rc, std::string("problem setup failed: ") + erem_last_error(ctx));
  BHIP(b, batch_pack(static_cast<int>(g.nx), static_cast<int>(g.ny), b->tmp_coef, b->tmp_F, d_T0, b->coef, b->g,
                     b->ntot, b->off[i], b->stream));
  Dims d{};
  d.nx = static_cast<int>(g.nx);
  d.ny = static_cast<int>(g.ny);
  d.nz = 1;
  d.dim = 2;
  d.N = static_cast<int>(N);
  d.dx = g.dx; d.dy = g.dy; d.dz = g.dz;
  BHIP(b, launch_gershgorin(d, b->tmp_coef, b->red, b->stream));
  BHIP(b, hipMemcpyAsync(b->h_red, b->red, sizeof(AsmReduce), hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  b->alpha[i] = slot_min(b->h_red->lo);
  b->beta[i] = slot_max(b->h_red->hi);
  b->set[i] = 1;
  b->prepared = false;
  return EREM_OK;
}

int erem_batch_prepare(erem_batch* b, double h, const erem_opts* o) {
  if (!b) return EREM_EINVAL;
  if (!o || !(h > 0) || !std::isfinite(h)) return bfail(b, EREM_EINVAL, "bad h or opts");
  if (o->method != EREM_METHOD_LEJA) return bfail(b, EREM_EINVAL, "the batch runs the Leja method");
  if (o->m_max < 5 || o->m_max > kMaxTerms) return bfail(b, EREM_EINVAL, "m_max must be in [5, 1024]");
  if (!(o->tol_a >= 0) || !(o->tol_r >= 0) || (o->tol_a == 0 && o->tol_r == 0))
    return bfail(b, EREM_EINVAL, "bad tolerances");
  for (int i = 0; i < b->nprob; ++i)
    if (!b->set[i]) return bfail(b, EREM_EINVAL, "every problem must be set before prepare");
  const int M = o->m_max;
  std::vector<double> xi;
  if (!leja_points(M + 1, xi)) return bfail(b, EREM_EINVAL, "Leja points");
  std::vector<double> dk(static_cast<size_t>(b->nprob) * (M + 1)), sh(dk.size());
  std::vector<BProb> prob(b->nprob);
  std::vector<double> cc(b->nprob), gg(b->nprob);
  for (int i = 0; i < b->nprob; ++i) {
    const double a = b->alpha[i], be = b->beta[i];
    const double width = be - a;
    if (!std::isfinite(width)) return bfail(b, EREM_ENONFINITE, "non-finite Gershgorin interval");
    if (!(width > 1e-14 * std::max(std::fabs(a), std::fabs(be)))) return bfail(b, EREM_EINVAL, "degenerate interval in a batch problem");
    int s = 1;
    if (o->rho_max > 0) s = std::max(1, static_cast<int>(std::ceil(h * width / o->rho_max)));
    s = std::min(s, std::max(1, o->max_substeps));
    cc[i] = 0.5 * (a + be);
    gg[i] = 0.25 * width;
    BProb& P = prob[i];
    P.nx = static_cast<int>(b->grids[i].nx);
    P.ny = static_cast<int>(b->grids[i].ny);
    P.s = s;
    P.off = b->off[i];
    P.inv_g = 1.0 / gg[i];
    P.delta = h / s;
    P.coef_off = i * (M + 1);
    for (int k = 0; k <= M; ++k) sh[P.coef_off + k] = k > 0 ? cc[i] / gg[i] + xi[k - 1] : 0.0;
  }
  // divided differences of every problem, in parallel on the host
  {
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t)
      pool.emplace_back([&, t]() {
        for (int i = static_cast<int>(t); i < b->nprob; i += static_cast<int>(nt))
          phi1_divided_differences(prob[i].delta * cc[i], prob[i].delta * gg[i], xi.data(), M + 1,
                                   &dk[static_cast<size_t>(i) * (M + 1)]);
      });
    for (auto& th : pool) th.join();
  }
  if (b->dk) (void)hipFree(b->dk);
  if (b->shift) (void)hipFree(b->shift);
  b->dk = b->shift = nullptr;
  if (balloc(b, &b->dk, dk.size()) || balloc(b, &b->shift, sh.size())) return EREM_ENOMEM;
  BHIP(b, hipMemcpy(b->dk, dk.data(), sizeof(double) * dk.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->shift, sh.data(), sizeof(double) * sh.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->prob, prob.data(), sizeof(BProb) * b->nprob, hipMemcpyHostToDevice));
  b->fp32 = o->precision == EREM_PREC_MIXED ? 1 : 0;
  if (b->fp32) {
    if (!b->coef32 && balloc(b, &b->coef32, 5 * static_cast<size_t>(b->ntot))) return EREM_ENOMEM;
    BHIP(b, launch_cast_f32(b->coef, b->coef32, 5 * b->ntot, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
  }
  b->m_max = M;
  b->tol_a = o->tol_a;
  b->tol_r = o->tol_r;
  b->thresh = std::pow(10.0, -o->p_order);
  drop_graphs(b);
  b->prepared = true;
  return EREM_OK;
}

int erem_batch_autotune(erem_batch* b, const double* d_T, int32_t nsteps, int32_t* chosen) {
  if (!b) return EREM_EINVAL;
  if (!b->prepared) return bfail(b, EREM_EINVAL, "erem_batch_prepare must come first");
  if (!d_T || nsteps < 1) return bfail(b, EREM_EINVAL, "bad arguments");
  double best = 1e300;
  int best_s = 0;
  for (int s = 0; s < kNumTileShapes; ++s) {
    b->shape = s;
    BHIP(b, hipMemcpyAsync(b->tscratch, d_T, sizeof(double) * b->ntot, hipMemcpyDeviceToDevice, b->stream));
    erem_batch_stats st{};
    const int rc = launch(b, b->tscratch, nsteps, false, &st);
    if (rc) return rc;
    if (st.ms < best) {
      best = st.ms;
      best_s = s;
    }
  }
  b->shape = best_s;
  if (chosen) *chosen = best_s;
  return EREM_OK;
}

int erem_batch_set_tile_shape(erem_batch* b, int32_t shape) {
  if (!b) return EREM_EINVAL;
  if (shape < 0 || shape >= kNumTileShapes) return bfail(b, EREM_EINVAL, "tile shape index out of range");
  b->shape = shape;
  return EREM_OK;
}

int erem_batch_run(erem_batch* b, double* d_T, int32_t nsteps, int32_t use_graph, erem_batch_stats* st) {
  if (!b) return EREM_EINVAL;
  if (!b->prepared) return bfail(b, EREM_EINVAL, "erem_batch_prepare must come first");
  if (!d_T || nsteps < 1) return bfail(b, EREM_EINVAL, "bad arguments");
  // a captured graph bakes in the T pointer: keep one graph per (nsteps, shape) and pointer
  if (use_graph && b->graph_T != d_T) {
    drop_graphs(b);
    b->graph_T = d_T;
  }
  return launch(b, d_T, nsteps, use_graph != 0, st);
}

}  // extern "C"
