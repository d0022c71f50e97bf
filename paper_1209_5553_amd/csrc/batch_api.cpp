// C ABI of the batched form (erem_batch_*): per-problem setup through the
// single-problem path, packing, per-problem Leja data, the tile list, and the
// sequence of phase launches of batch.hip that runs every problem for all
// steps (captured in one hipGraph, or enqueued from the host in chunks).
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
  double *coef = nullptr, *g = nullptr, *v = nullptr, *u0 = nullptr, *u1 = nullptr, *T1 = nullptr;
  double *q0 = nullptr, *q1 = nullptr, *p0 = nullptr, *p1 = nullptr;  // FP64 or FP32 (sized for FP64)
  float* coef32 = nullptr;
  double *dk = nullptr, *shift = nullptr, *tscratch = nullptr, *part = nullptr;
  BProb* prob = nullptr;
  BTile* tile = nullptr;
  BState* state = nullptr;
  int* ndone = nullptr;
  int* h_ndone = nullptr;  // pinned
  int ntiles = 0, tile_cap = 0;
  std::vector<BProb> hprob;
  // prepared state
  bool prepared = false;
  int fp32 = 0, m_max = 0;
  double tol_a = 0.0, tol_r = 1e-12, thresh = 1e-2;
  int shape = 0;
  int prof_stride = 0;  // work passes between timed ones (0: no timing)
  struct Graph {
    hipGraphExec_t exec = nullptr;
    int phases = 0;                   // work passes captured
  };
  std::map<std::pair<int, int>, Graph> graphs;  // (nsteps, shape) -> graph
  const double* graph_T = nullptr;              // T array the graphs were captured with
  std::map<std::pair<int, int>, int> calib;     // (nsteps, shape) -> work passes of a calibration run
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

void drop_graphs(erem_batch* b) {
  for (auto& kv : b->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  b->graphs.clear();
}

void free_batch(erem_batch* b) {
  double** d[] = {&b->coef, &b->g, &b->v, &b->u0, &b->u1, &b->T1, &b->q0, &b->q1, &b->p0, &b->p1,
                  &b->dk, &b->shift, &b->tscratch, &b->part, &b->tmp_coef, &b->tmp_F};
  for (double** x : d)
    if (*x) { (void)hipFree(*x); *x = nullptr; }
  if (b->coef32) (void)hipFree(b->coef32);
  if (b->prob) (void)hipFree(b->prob);
  if (b->tile) (void)hipFree(b->tile);
  if (b->state) (void)hipFree(b->state);
  if (b->ndone) (void)hipFree(b->ndone);
  if (b->h_ndone) (void)hipHostFree(b->h_ndone);
  if (b->red) (void)hipFree(b->red);
  if (b->h_red) (void)hipHostFree(b->h_red);
  drop_graphs(b);
  for (auto& kv : b->ctxs) erem_destroy(kv.second);
  b->ctxs.clear();
}

// Tile list and per-problem tile ranges for the current shape (64 x rows
// tiles, each problem's tiles row by row).  The work pass deals the tile
// list to the XCDs in eight contiguous chunks, so the order of the problems
// decides which XCD works on which problem.  Once the intervals are known
// the problems go in order of their schedule length h (beta - alpha) (the
// Newton terms of a step grow with it), dealt to eight groups in serpentine
// order (1..8, 8..1, ...), and the groups follow each other: each XCD gets a
// like mix of long and short schedules, and the last phases, where only the
// longest problems are left, run on all XCDs.  Each problem's own results do
// not depend on the order.
int build_tiles(erem_batch* b) {
  const int rows = kBatchTileRows[b->shape];
  std::vector<BTile> tiles;
  std::vector<int> ord(b->nprob);
  std::vector<double> len(b->nprob, 0.0);
  for (int i = 0; i < b->nprob; ++i) {
    const BProb& P = b->hprob[i];
    ord[i] = i;
    len[i] = P.inv_g > 0.0 ? P.delta * P.s * 4.0 / P.inv_g : 0.0;  // h (beta - alpha); 0 before prepare
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return len[x] > len[y]; });
  std::vector<std::vector<int>> groups(kXcds);
  for (size_t r = 0; r < ord.size(); ++r) {
    const size_t q = r % (2 * kXcds);
    groups[q < kXcds ? q : 2 * kXcds - 1 - q].push_back(ord[r]);
  }
  ord.clear();
  for (const auto& g : groups) ord.insert(ord.end(), g.begin(), g.end());
  for (const int i : ord) {
    BProb& P = b->hprob[i];
    const int tx = static_cast<int>((b->grids[i].nx + kBatchTileX - 1) / kBatchTileX);
    const int ty = static_cast<int>((b->grids[i].ny + rows - 1) / rows);
    P.tile0 = static_cast<int>(tiles.size());
    P.ntiles = tx * ty;
    P.tiles_x = tx;
    for (int y = 0; y < ty; ++y)
      for (int x = 0; x < tx; ++x) tiles.push_back(BTile{i, x * kBatchTileX, y * rows, 0});
  }
  if (tiles.size() > static_cast<size_t>(1 << 30)) return bfail(b, EREM_EINVAL, "too many tiles");
  b->ntiles = static_cast<int>(tiles.size());
  if (b->ntiles > b->tile_cap) {
    // sized once for the largest tile count of any shape (the fewest rows),
    // so that the arrays the graphs hold are never reallocated
    long long cap = 0;
    int rmin = kBatchTileRows[0];
    for (int k = 1; k < kNumTileShapes; ++k) rmin = std::min(rmin, kBatchTileRows[k]);
    for (int i = 0; i < b->nprob; ++i)
      cap += ((b->grids[i].nx + kBatchTileX - 1) / kBatchTileX) * ((b->grids[i].ny + rmin - 1) / rmin);
    cap = std::max<long long>(cap, b->ntiles);
    if (b->tile) (void)hipFree(b->tile);
    if (b->part) (void)hipFree(b->part);
    b->tile = nullptr;
    b->part = nullptr;
    if (balloc(b, &b->tile, cap) || balloc(b, &b->part, kBatchPartStride * static_cast<size_t>(cap)))
      return EREM_ENOMEM;
    b->tile_cap = static_cast<int>(cap);
  }
  BHIP(b, hipMemcpy(b->tile, tiles.data(), sizeof(BTile) * tiles.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->prob, b->hprob.data(), sizeof(BProb) * b->nprob, hipMemcpyHostToDevice));
  return EREM_OK;
}

BatchArgs make_args(erem_batch* b, double* T, int nsteps) {
  BatchArgs a{};
  a.prob = b->prob;
  a.tile = b->tile;
  a.state = b->state;
  a.ndone = b->ndone;
  a.coef64 = b->coef;
  a.coef = b->fp32 ? static_cast<const void*>(b->coef32) : static_cast<const void*>(b->coef);
  a.g = b->g;
  a.T0 = T;
  a.T1 = b->T1;
  a.u0 = b->u0;
  a.u1 = b->u1;
  a.v = b->v;
  a.q0 = b->q0;
  a.q1 = b->q1;
  a.p0 = b->p0;
  a.p1 = b->p1;
  a.dk = b->dk;
  a.shift = b->shift;
  a.part = b->part;
  a.ntot = b->ntot;
  a.nprob = b->nprob;
  a.ntiles = b->ntiles;
  a.nsteps = nsteps;
  a.m_max = b->m_max;
  a.tol_a = b->tol_a;
  a.tol_r = b->tol_r;
  a.thresh = b->thresh;
  a.nt = kBatchPassTerms[b->shape];
  return a;
}

// Upper bound of the work passes a run can take: every problem needs, per
// step and substep, one start pass and at most m_max / 4 term passes, and
// one finish pass.
long long max_phases(erem_batch* b, int nsteps) {
  int smax = 1;
  for (const BProb& P : b->hprob) smax = std::max(smax, P.s);
  return static_cast<long long>(nsteps) * smax * (1 + b->m_max / 4) + 2;
}

// Phases enqueued eagerly in chunks, the host reading the count of finished
// problems after each chunk, until every problem is done.  Returns the work
// passes enqueued.  With prof_stride > 0 every prof_stride-th work launch
// records its own start and stop (events of the dispatch itself), read when
// its chunk has finished, into *work_ms / *timed.
int run_eager(erem_batch* b, const BatchArgs& a, long long start, long long* passes, double* work_ms, int* timed) {
  constexpr int kChunk = 64;
  const long long limit = max_phases(b, a.nsteps);
  long long n = start;
  std::vector<hipEvent_t> ev;
  auto drop = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  };
  if (b->prof_stride > 0) {
    ev.resize(2 * kChunk, nullptr);
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        drop();
        return bfail(b, EREM_EDEVICE, "hipEventCreate failed");
      }
  }
  std::vector<char> was_timed(kChunk, 0);
  while (true) {
    BHIP(b, hipMemcpyAsync(b->h_ndone, b->ndone, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    const hipError_t se = hipStreamSynchronize(b->stream);
    if (se != hipSuccess) {
      drop();
      return bfail(b, EREM_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(se));
    }
    for (int c = 0; c < kChunk; ++c) {
      if (!was_timed[c]) continue;
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]) == hipSuccess) {
        *work_ms += ms;
        ++*timed;
      } else {
        (void)hipGetLastError();  // leave no error behind for the caller's next check
      }
      was_timed[c] = 0;
    }
    if (*b->h_ndone >= b->nprob) break;
    if (n >= limit) {
      drop();
      return bfail(b, EREM_EDEVICE, "batch run did not finish within its phase bound");
    }
    for (int c = 0; c < kChunk && n < limit; ++c, ++n) {
      const bool time_it = !ev.empty() && n % b->prof_stride == 0;
      const hipError_t le = batch_phase(a, b->shape, b->fp32, b->stream, time_it ? ev[2 * c] : nullptr,
                                        time_it ? ev[2 * c + 1] : nullptr);
      if (le != hipSuccess) {
        drop();
        return bfail(b, EREM_EDEVICE, std::string("batch phase launch: ") + hipGetErrorString(le));
      }
      was_timed[c] = time_it ? 1 : 0;
    }
  }
  drop();
  *passes = n;
  return EREM_OK;
}

// Capture reset + `phases` work passes into a graph.
int capture(erem_batch* b, const BatchArgs& a, int phases, erem_batch::Graph* g) {
  g->phases = phases;
  hipGraph_t graph;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = batch_reset(a, b->stream);
  for (int n = 0; n < phases && le == hipSuccess; ++n) le = batch_phase(a, b->shape, b->fp32, b->stream);
  const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, EREM_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ce));
  }
  const hipError_t ie = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return bfail(b, EREM_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
  return EREM_OK;
}

// One run of nsteps steps on T (synchronises the stream).
int launch(erem_batch* b, double* T, int nsteps, bool use_graph, erem_batch_stats* st) {
  const BatchArgs a = make_args(b, T, nsteps);
  const auto key = std::make_pair(nsteps, b->shape);
  erem_batch::Graph* g = nullptr;
  // timed work launches need their own dispatch events: such runs go eagerly
  if (b->prof_stride > 0) use_graph = false;
  if (use_graph) {
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      // the budget of captured passes comes from a calibration run on a copy
      auto ci = b->calib.find(key);
      if (ci == b->calib.end()) {
        BHIP(b, hipMemcpyAsync(b->tscratch, T, sizeof(double) * b->ntot, hipMemcpyDeviceToDevice, b->stream));
        const BatchArgs ac = make_args(b, b->tscratch, nsteps);
        BHIP(b, batch_reset(ac, b->stream));
        long long used = 0;
        double wm = 0.0;
        int tn = 0;
        const int saved = b->prof_stride;
        b->prof_stride = 0;
        const int rc = run_eager(b, ac, 0, &used, &wm, &tn);
        b->prof_stride = saved;
        if (rc) return rc;
        // passes up to the last problem's finish (the eager run overshoots by < one chunk)
        std::vector<BState> S(b->nprob);
        BHIP(b, hipMemcpy(S.data(), b->state, sizeof(BState) * b->nprob, hipMemcpyDeviceToHost));
        int need = 0;
        for (const BState& s : S) need = std::max(need, s.phases);
        ci = b->calib.emplace(key, need).first;
      }
      const int budget = ci->second + std::max(8, ci->second / 32);
      erem_batch::Graph ng;
      const int rc = capture(b, a, budget, &ng);
      if (rc) {
        if (ng.exec) (void)hipGraphExecDestroy(ng.exec);
        return rc;
      }
      it = b->graphs.emplace(key, std::move(ng)).first;
    }
    g = &it->second;
  }
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  BHIP(b, hipEventRecord(e0, b->stream));
  long long passes = 0;
  double work_ms = 0.0;
  int timed = 0;
  int rc = EREM_OK;
  if (g) {
    BHIP(b, hipGraphLaunch(g->exec, b->stream));
    // a run that needs more passes than the graph holds continues eagerly
    rc = run_eager(b, a, g->phases, &passes, &work_ms, &timed);
  } else {
    BHIP(b, batch_reset(a, b->stream));
    rc = run_eager(b, a, 0, &passes, &work_ms, &timed);
  }
  BHIP(b, hipEventRecord(e1, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  if (rc) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
  }
  float ms = 0.0f;
  BHIP(b, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::vector<BState> S(b->nprob);
  BHIP(b, hipMemcpy(S.data(), b->state, sizeof(BState) * b->nprob, hipMemcpyDeviceToHost));
  long long tot = 0;
  int tmin = 1 << 30, tmax = 0, failed = 0, flags = 0, phases = 0;
  double bytes = 0.0;
  const double per_cell = b->fp32 ? 36.0 : 72.0;  // 5 coef + q_in + p rd/wr + q_out
  for (int i = 0; i < b->nprob; ++i) {
    const BState& d = S[i];
    bytes += per_cell * static_cast<double>(d.terms) * static_cast<double>(b->off[i + 1] - b->off[i]);
    tot += d.terms;
    tmin = std::min(tmin, d.terms);
    tmax = std::max(tmax, d.terms);
    phases = std::max(phases, d.phases);
    if (d.flags || d.step < nsteps) ++failed;
    flags |= d.flags;
  }
  if (st) {
    st->terms_total = tot;
    st->terms_min = b->nprob ? tmin : 0;
    st->terms_max = tmax;
    st->failed = failed;
    st->tile_shape = b->shape;
    st->graph = g ? 1 : 0;
    st->grid = b->ntiles;
    st->ms = ms;
    st->leja_bytes = bytes;
    st->phases = phases;
    st->passes = g ? std::max<long long>(g->phases, passes) : passes;
    st->work_ms = work_ms;
    st->work_timed = timed;
  }
  if (flags & 2) return bfail(b, EREM_ENONFINITE, "non-finite Leja norm in a batch problem");
  if (flags & 4) return bfail(b, EREM_EINVAL, "error scale is zero in a batch problem (tol_a = 0 and T = 0)");
  if (failed) return bfail(b, EREM_ENOCONV, "a batch problem did not converge within m_max terms");
  return EREM_OK;
}

// Switch the tile shape: the tile list changes, so the captured graphs go.
// Whether a tile shape's dynamic LDS (at the batch's precision) fits the
// device's limit per workgroup.
bool shape_fits(const erem_batch* b, int shape) {
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return batch_lds_bytes(shape, b->fp32) + 1024 <= static_cast<size_t>(max_lds);  // + the static reduction arrays
}

int set_shape(erem_batch* b, int shape) {
  if (shape == b->shape) return EREM_OK;
  BHIP(b, hipStreamSynchronize(b->stream));
  drop_graphs(b);
  b->shape = shape;
  return build_tiles(b);
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
  rc |= balloc(b, &b->u0, n);
  rc |= balloc(b, &b->u1, n);
  rc |= balloc(b, &b->T1, n);
  rc |= balloc(b, &b->q0, n);
  rc |= balloc(b, &b->q1, n);
  rc |= balloc(b, &b->p0, n);
  rc |= balloc(b, &b->p1, n);
  rc |= balloc(b, &b->tscratch, n);
  rc |= balloc(b, &b->prob, nprob);
  rc |= balloc(b, &b->state, nprob);
  rc |= balloc(b, &b->ndone, 1);
  rc |= balloc(b, &b->red, 1);
  if (rc == EREM_OK && hipHostMalloc(reinterpret_cast<void**>(&b->h_red), sizeof(AsmReduce), hipHostMallocDefault) != hipSuccess)
    rc = EREM_ENOMEM;
  if (rc == EREM_OK && hipHostMalloc(reinterpret_cast<void**>(&b->h_ndone), sizeof(int), hipHostMallocDefault) != hipSuccess)
    rc = EREM_ENOMEM;
  if (rc == EREM_OK) {
    b->hprob.assign(nprob, BProb{});
    for (int i = 0; i < nprob; ++i) {
      b->hprob[i].nx = static_cast<int>(grids[i].nx);
      b->hprob[i].ny = static_cast<int>(grids[i].ny);
      b->hprob[i].s = 1;
      b->hprob[i].off = b->off[i];
    }
    rc = build_tiles(b);
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
  std::vector<BProb>& prob = b->hprob;
  std::vector<double> cc(b->nprob), gg(b->nprob);
  for (int i = 0; i < b->nprob; ++i) {
    const double a = b->alpha[i], be = b->beta[i];
    const double width = be - a;
    if (!std::isfinite(width)) return bfail(b, EREM_ENONFINITE, "non-finite Gershgorin interval");
    if (!(width > 1e-14 * std::max(std::fabs(a), std::fabs(be)))) return bfail(b, EREM_EINVAL, "degenerate interval in a batch problem");
    int s = 1;
    const double rho = o->precision == EREM_PREC_MIXED ? std::min(o->rho_max, kMixedRhoMax) : o->rho_max;
    if (rho > 0) s = std::max(1, static_cast<int>(std::ceil(h * width / rho)));
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
    P.rootN = std::sqrt(static_cast<double>(P.nx) * P.ny);
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
  const int trc = build_tiles(b);  // uploads the problem records
  if (trc) return trc;
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
  b->calib.clear();
  b->prepared = true;
  return EREM_OK;
}

int erem_batch_autotune(erem_batch* b, const double* d_T, int32_t nsteps, int32_t* chosen) {
  if (!b) return EREM_EINVAL;
  if (!b->prepared) return bfail(b, EREM_EINVAL, "erem_batch_prepare must come first");
  if (!d_T || nsteps < 1) return bfail(b, EREM_EINVAL, "bad arguments");
  double best = 1e300;
  int best_s = 0;
  const int saved = b->prof_stride;
  b->prof_stride = 0;
  for (int s = 0; s < kNumTileShapes; ++s) {
    if (!shape_fits(b, s)) continue;
    const int rc0 = set_shape(b, s);
    if (rc0) return rc0;
    BHIP(b, hipMemcpyAsync(b->tscratch, d_T, sizeof(double) * b->ntot, hipMemcpyDeviceToDevice, b->stream));
    erem_batch_stats st{};
    const int rc = launch(b, b->tscratch, nsteps, false, &st);
    if (rc) {
      b->prof_stride = saved;
      return rc;
    }
    if (st.ms < best) {
      best = st.ms;
      best_s = s;
    }
  }
  b->prof_stride = saved;
  const int rc = set_shape(b, best_s);
  if (rc) return rc;
  if (chosen) *chosen = best_s;
  return EREM_OK;
}

int erem_batch_set_tile_shape(erem_batch* b, int32_t shape) {
  if (!b) return EREM_EINVAL;
  if (shape < 0 || shape >= kNumTileShapes) return bfail(b, EREM_EINVAL, "tile shape index out of range");
  if (!shape_fits(b, shape)) return bfail(b, EREM_EINVAL, "tile shape needs more LDS than the device has");
  return set_shape(b, shape);
}

int erem_batch_profile(erem_batch* b, int32_t stride) {
  if (!b) return EREM_EINVAL;
  if (stride < 0) return bfail(b, EREM_EINVAL, "stride must be >= 0");
  if (stride != b->prof_stride) {
    BHIP(b, hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->prof_stride = stride;
  }
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
