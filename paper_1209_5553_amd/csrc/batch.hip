// Batched EREM for many independent linear problems.
//
// Every problem p (its own n_x x n_y grid, packed one after the other) has a
// constant Jacobian J_p and G_p(T) = J_p T + g_p (fixed fluxes, constant
// capacity), so one EREM step is T <- T + h phi1(h J_p)(J_p T + g_p)
// (Eq. EERM) with a Gershgorin interval, substep count and divided
// differences fixed for the whole run (Sec. 4.2).
//
// MI355X mapping.  The problems are cut into 64 x rows tiles and all tiles
// of all problems form one list.  A run is a sequence of phases; in each
// phase ONE work launch covers the whole tile list and advances every
// problem that is not done by one step of its own schedule:
//
//   start pass  q_0 = v + J u, p = d_0 q_0 (with the end of the previous
//               substep, u += delta p, or of the previous step,
//               T += u + delta p, folded in: a cell's neighbours' values are
//               formed from their own u, p, T, so no extra pass is needed);
//   term pass   NT = 4 or 8 Newton terms
//               q_k = ((J - cI)/gamma - xi_{k-1}) q_{k-1}, p += d_k q_k
//               (Eq. newt) on the tile, computed over the tile plus the halo
//               that NT stencil applications need; the intermediate terms
//               never leave the CU;
//   finish pass T += u + delta p of the last step.
//
// Each tile stores its block partial sums (sum q_k^2 per term, in FP64); a
// control kernel then reduces each problem's partials in a fixed order (one
// wavefront per problem), applies the scaled-norm stop test of Sec. 4.2 to
// the pass's NT estimates in order, and sets the problem's next phase.
// Problems of every size and substep count thus share every launch, the
// work spreads over all CUs whatever the mix, and the whole run is a fixed
// sequence of launches with no grid-wide synchronisation and no waiting
// inside a kernel, which a hipGraph captures.  Tiles of problems that are
// done return at entry.  Buffers the start pass reads with a halo and
// rewrites (T, u, p) are ping-ponged so that no tile reads a neighbour's
// updated value.
#include "batch.h"

#include <cmath>

namespace erem {

namespace {

template <class V>
__device__ inline V cv(double x) { return static_cast<V>(x); }

// Two buffers in the frame of q_{k-1} (the tile plus a halo of NT): the
// first holds q_{k-1}, then the odd intermediate terms; the second the even
// ones.
template <int TY, int NT, class V>
constexpr size_t work_lds_bytes() {
  return 2 * sizeof(V) * static_cast<size_t>(TY + 2 * NT) * (kBatchTileX + 2 * NT);
}

// Sum (or max) over the workgroup of one double per thread; fixed order
// (each wavefront by a shuffle tree, then the wavefronts in order); the
// result is valid in thread 0.
template <int NW, bool MAX>
__device__ inline double block_reduce(double v, double* sh, int tid) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = MAX ? fmax(v, o) : v + o;
  }
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0) {
    r = sh[0];
    for (int w = 1; w < NW; ++w) r = MAX ? fmax(r, sh[w]) : r + sh[w];
  }
  __syncthreads();
  return r;
}

template <int TY, int BY, int NT, bool XCD, class V>
__global__ __launch_bounds__(kBatchTileX* BY) void k_bt_work(BatchArgs a) {
  static_assert(TY % BY == 0, "whole thread rows per tile");
  static_assert(NT >= 2 && NT <= kBatchPartStride, "terms per pass");
  constexpr int NTH = kBatchTileX * BY;  // threads
  constexpr int NW = NTH / 64;
  constexpr int R = TY / BY;             // tile rows per thread in the start and finish passes
  constexpr int H = NT - 1;
  constexpr int WQ = kBatchTileX + 2 * NT, HQ = TY + 2 * NT;  // q_{k-1}: halo NT
  constexpr int WI = kBatchTileX + 2 * H, HI = TY + 2 * H;    // stencil, intermediates: halo NT - 1
  extern __shared__ __align__(16) unsigned char smem[];
  V(*sq)[WQ] = reinterpret_cast<V(*)[WQ]>(smem);  // q_{k-1}, then the odd terms
  V(*sb)[WQ] = reinterpret_cast<V(*)[WQ]>(smem + sizeof(V) * HQ * WQ);  // the even terms
  __shared__ double red[NT][NW];

  const int t = XCD ? xcd_tile_id() : static_cast<int>(blockIdx.x);
  const BTile tl = a.tile[t];
  if (tl.done) return;  // the tiles of a finished problem stop here, before its state is read
  const BState S = a.state[tl.pid];
  if (S.phase == kPhDone) return;
  const BProb P = a.prob[tl.pid];
  const int nx = P.nx, ny = P.ny;
  const long long o = P.off, Nt = a.ntot;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int tid = lx + kBatchTileX * ly;
  const int x = tl.x0 + lx;
  double* part = a.part + static_cast<long long>(kBatchPartStride) * t;

  if (S.phase == kPhFinish) {
    // T^N = T^{N-1} + u + delta p (a failed problem keeps its last step's T)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = tl.y0 + ly + r * BY;
      if (x < nx && y < ny) {
        const long long i = o + x + static_cast<long long>(nx) * y;
        const double* Tc = S.tpar ? a.T1 : a.T0;
        double Tn = Tc[i];
        if (S.flags == 0) {
          const V* pc = reinterpret_cast<const V*>(S.ppar ? a.p1 : a.p0);
          const double* uc = S.upar ? a.u1 : a.u0;
          Tn += (P.s > 1 ? uc[i] : 0.0) + P.delta * static_cast<double>(pc[i]);
        }
        a.T0[i] = Tn;
      }
    }
    return;
  }

  if (S.phase == kPhInit) {
    // start of substep S.sub of step S.step
    double s0 = 0.0, mx = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = tl.y0 + ly + r * BY;
      if (!(x < nx && y < ny)) continue;
      const long long i = o + x + static_cast<long long>(nx) * y;
      const long long jw = x > 0 ? i - 1 : i, je = x + 1 < nx ? i + 1 : i;
      const long long js = y > 0 ? i - nx : i, jn = y + 1 < ny ? i + nx : i;
      const long long jj[5] = {i, jw, je, js, jn};
      double c[5], w[5];
#pragma unroll
      for (int d = 0; d < 5; ++d) c[d] = a.coef64[d * Nt + i];  // 0 toward missing neighbours
      const double* Tc = S.tpar ? a.T1 : a.T0;
      const double* uc = S.upar ? a.u1 : a.u0;
      const V* pc = reinterpret_cast<const V*>(S.ppar ? a.p1 : a.p0);
      if (S.kind == kInitFirst) {
#pragma unroll
        for (int d = 0; d < 5; ++d) w[d] = Tc[jj[d]];
      } else if (S.kind == kInitStep) {
        // T^{n} = T^{n-1} + u + delta p at the cell and its neighbours
        const bool use_u = P.s > 1;
#pragma unroll
        for (int d = 0; d < 5; ++d)
          w[d] = Tc[jj[d]] + (use_u ? uc[jj[d]] : 0.0) + P.delta * static_cast<double>(pc[jj[d]]);
      } else {
        // u after substep S.sub - 1: u + delta p (u = 0 after the first)
        const bool use_u = S.sub > 1;
#pragma unroll
        for (int d = 0; d < 5; ++d) w[d] = (use_u ? uc[jj[d]] : 0.0) + P.delta * static_cast<double>(pc[jj[d]]);
      }
      double jw_ = c[0] * w[0];
#pragma unroll
      for (int d = 1; d < 5; ++d) jw_ += c[d] * w[d];
      double q;
      if (S.kind == kInitSub) {
        (S.upar ? a.u0 : a.u1)[i] = w[0];
        q = a.v[i] + jw_;
      } else {
        if (S.kind == kInitStep) (S.tpar ? a.T0 : a.T1)[i] = w[0];
        q = jw_ + a.g[i];
        a.v[i] = q;
        mx = fmax(mx, fabs(w[0]));
      }
      const V qv = cv<V>(q);
      reinterpret_cast<V*>(a.q0)[i] = qv;
      reinterpret_cast<V*>(S.ppar ? a.p0 : a.p1)[i] = cv<V>(a.dk[P.coef_off]) * qv;
      s0 += static_cast<double>(qv) * static_cast<double>(qv);
    }
    const double S0 = block_reduce<NW, false>(s0, &red[0][0], tid);
    const double M0 = block_reduce<NW, true>(mx, &red[1][0], tid);
    if (tid == 0) {
      part[0] = S0;
      part[1] = M0;
    }
    return;
  }

  // NT Newton terms S.k .. S.k + NT - 1 on the tile.  The tile plus its
  // halo of NT - 1 (the "box", HI x WI cells) is cut into vertical strips of
  // SH cells, one per thread, consecutive threads taking consecutive
  // columns.  A thread keeps the stencil and the current term of its strip
  // in registers and computes its cells in every term whose region (the box
  // shrinking by one cell per term) holds them: the north and south
  // neighbours come from its own registers (from LDS at the strip's ends),
  // the west and east ones from LDS, where every term is written for the
  // neighbouring strips.  p and the partial sums accumulate for the strip's
  // cells in the tile.
  const int grp = (S.k - 1) / NT;
  const V* __restrict__ qin = reinterpret_cast<const V*>((grp & 1) ? a.q1 : a.q0);
  V* __restrict__ qout = reinterpret_cast<V*>((grp & 1) ? a.q0 : a.q1);
  V* __restrict__ p = reinterpret_cast<V*>(S.ppar ? a.p1 : a.p0);
  const V* __restrict__ coef = reinterpret_cast<const V*>(a.coef);
  const int x0 = tl.x0, y0 = tl.y0;
  constexpr int UQ = (HQ * WQ + NTH - 1) / NTH;  // q values staged per thread
  constexpr int SROWS = NTH / WI;                // strip rows the threads can cover
  static_assert(SROWS >= 1, "a thread per box column");
  constexpr int SH = (HI + SROWS - 1) / SROWS;   // cells per strip
  constexpr int NSR = (HI + SH - 1) / SH;        // strip rows used
  const bool has_strip = tid < NSR * WI;
  const int bx = has_strip ? tid % WI : 0;
  const int by0 = has_strip ? (tid / WI) * SH : HI;  // first cell of the strip (box rows)
  // every load of the tile is issued (into registers) before the first LDS
  // store, so the tile waits for one memory latency
  V rq[UQ];
#pragma unroll
  for (int u = 0; u < UQ; ++u) {
    const int e = tid + u * NTH;
    const int ry = e / WQ, rx = e - ry * WQ;
    const int gx = x0 - NT + rx, gy = y0 - NT + ry;
    rq[u] = (e < HQ * WQ && gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? qin[o + gx + nx * gy] : V(0);
  }
  const int gx = x0 - H + bx;
  const bool col_in = has_strip && gx >= 0 && gx < nx;
  const bool col_tile = has_strip && bx >= H && bx < H + kBatchTileX;
  V rc[5][SH], acc[SH];
#pragma unroll
  for (int r = 0; r < SH; ++r) {
    const int by = by0 + r, gy = y0 - H + by;
    const bool in = col_in && by < HI && gy >= 0 && gy < ny;
    const long long j = o + (in ? gx + static_cast<long long>(nx) * gy : 0);
#pragma unroll
    for (int d = 0; d < 5; ++d) rc[d][r] = in ? coef[d * Nt + j] : V(0);
    const bool tile_cell = in && col_tile && by >= H && by < H + TY;
    acc[r] = tile_cell ? p[j] : V(0);
  }
#pragma unroll
  for (int u = 0; u < UQ; ++u) {
    const int e = tid + u * NTH;
    if (e < HQ * WQ) sq[e / WQ][e % WQ] = rq[u];
  }
  __syncthreads();
  // the strip's q_{k-1} (rows up to HI: the halo of q_{k-1} above the box)
  V cur[SH];
#pragma unroll
  for (int r = 0; r < SH; ++r) cur[r] = has_strip && by0 + r <= HI ? sq[by0 + r + 1][bx + 1] : V(0);
  const V ig = cv<V>(P.inv_g);
  const double* shf = a.shift + P.coef_off + S.k;
  const double* dkp = a.dk + P.coef_off + S.k;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const V sh = cv<V>(shf[tt]);
    const V dkt = cv<V>(dkp[tt]);
    const V(*src)[WQ] = (tt & 1) ? sb : sq;
    V(*dst)[WQ] = (tt & 1) ? sq : sb;
    double sum = 0.0;  // this thread's share of sum q_k^2 over the tile
    // the cell below the strip, from LDS (the strip above computed it)
    const V below = has_strip ? src[by0][bx + 1] : V(0);
    const V above = has_strip && by0 + SH + 1 < HQ ? src[by0 + SH + 1][bx + 1] : V(0);
    V nxt[SH];
#pragma unroll
    for (int r = 0; r < SH; ++r) {
      const int by = by0 + r;
      nxt[r] = cur[r];
      // the region of term tt: the box less tt cells on every side
      if (has_strip && by >= tt && by < HI - tt && bx >= tt && bx < WI - tt) {
        const V qc = cur[r];
        const V qw = src[by + 1][bx];
        const V qe = src[by + 1][bx + 2];
        const V qs = r > 0 ? cur[r - 1] : below;
        const V qn = r + 1 < SH ? cur[r + 1] : above;
        V jq = rc[0][r] * qc;
        jq += rc[1][r] * qw;
        jq += rc[2][r] * qe;
        jq += rc[3][r] * qs;
        jq += rc[4][r] * qn;
        const V qo = jq * ig - sh * qc;  // zero outside the grid (stencil and q are)
        nxt[r] = qo;
        if (tt + 1 < NT) dst[by + 1][bx + 1] = qo;
        if (col_tile && by >= H && by < H + TY) {
          acc[r] += dkt * qo;
          sum += static_cast<double>(qo) * static_cast<double>(qo);
          if (tt + 1 == NT) {
            // the last term: p and q_k of the tile go straight out
            const int gy = y0 - H + by;
            if (col_in && gy < ny) {
              const long long j = o + gx + static_cast<long long>(nx) * gy;
              p[j] = acc[r];
              qout[j] = qo;
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < SH; ++r) cur[r] = nxt[r];
    // the wavefront's share of the term's norm, to LDS in wavefront order
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    if ((tid & 63) == 0) red[tt][tid >> 6] = sum;
    if (tt + 1 < NT) __syncthreads();
  }
  __syncthreads();
  if (tid < NT) {
    double v = red[tid][0];
    for (int w = 1; w < NW; ++w) v += red[tid][w];
    part[tid] = v;
  }
}

// One wavefront per problem: reduce the problem's tile partials of the last
// work pass in a fixed order, apply the stop test and pick the next phase.
constexpr int kCtrlThreads = 64;  // one wavefront (one problem) per workgroup

__global__ __launch_bounds__(kCtrlThreads) void k_bt_ctrl(BatchArgs a) {
  const int lane = threadIdx.x & 63;
  const int pid = blockIdx.x * (kCtrlThreads / 64) + (threadIdx.x >> 6);
  if (pid >= a.nprob) return;
  // the state and the problem record are loaded together, then the partials
  // with the stop test's coefficients: two memory round trips
  BState S = a.state[pid];
  const BProb P = a.prob[pid];
  if (S.phase == kPhDone) return;
  if (S.phase == kPhFinish) {
    // the finish pass is done: from the next launch on the problem's tiles
    // return at entry
    for (int tt = lane; tt < P.ntiles; tt += 64) a.tile[P.tile0 + tt].done = 1;
    if (lane == 0) {
      S.phase = kPhDone;
      ++S.phases;
      a.state[pid] = S;
      atomicAdd(a.ndone, 1);
    }
    return;
  }
  const bool init = S.phase == kPhInit;
  const int nt = a.nt;
  const double* dk = a.dk + P.coef_off;
  double dkv[kBatchPartStride];
#pragma unroll
  for (int j = 0; j < kBatchPartStride; ++j) dkv[j] = init ? dk[0] : (j < nt ? dk[S.k + j] : 0.0);
  const double* pp = a.part + static_cast<long long>(kBatchPartStride) * P.tile0;
  double s[kBatchPartStride];
#pragma unroll
  for (int j = 0; j < kBatchPartStride; ++j) s[j] = 0.0;
  double mx = 0.0;
  for (int tt = lane; tt < P.ntiles; tt += 64) {
    const double* pt = pp + kBatchPartStride * tt;
    if (init) {
      s[0] += pt[0];
      mx = fmax(mx, pt[1]);
    } else {
#pragma unroll
      for (int j = 0; j < kBatchPartStride; ++j)
        if (j < nt) s[j] += pt[j];
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int j = 0; j < kBatchPartStride; ++j) s[j] += __shfl_down(s[j], off, 64);
    mx = fmax(mx, __shfl_down(mx, off, 64));
  }
  // the pass's scaled estimates |delta d_k| ||q_k|| / (sqrt(N) scal), lane j
  // forming term S.k + j's (each the expression a sequential loop would
  // evaluate, so the same bits), then gathered in lane 0
  mx = __shfl(mx, 0, 64);
  if (init && S.kind != kInitSub) S.scal = a.tol_a + a.tol_r * mx;
  double sj = 0.0, dj = 0.0;
#pragma unroll
  for (int j = 0; j < kBatchPartStride; ++j) {
    const double v = __shfl(s[j], 0, 64);
    if (lane == j) {
      sj = v;
      dj = dkv[j];
    }
  }
  const double est = fabs(P.delta * dj) * sqrt(sj) / (P.rootN * S.scal);
  double estv[kBatchPartStride];
#pragma unroll
  for (int j = 0; j < kBatchPartStride; ++j) estv[j] = __shfl(est, j, 64);
  if (lane != 0) return;
  ++S.phases;
  bool stop = false;  // no further Newton work for this problem
  if (init) {
    if (S.kind == kInitStep) S.tpar ^= 1;
    if (S.kind == kInitSub) S.upar ^= 1;
    S.ppar ^= 1;
    if (!isfinite(s[0]) || !isfinite(mx)) {
      S.flags |= 2;
      stop = true;
    } else if (!(S.scal > 0.0)) {
      S.flags |= 4;
      stop = true;
    } else if (nt > a.m_max) {
      S.flags |= 1;  // not even one pass fits the term budget
      stop = true;
    } else {
      S.ring[0] = estv[0];
      S.k = 1;
      S.phase = kPhTerms;
    }
  } else {
    // the terms in order until the test passes; every index below is a
    // compile-time constant (the unrolled loops select the ring slot), so
    // the state stays in registers
    bool done = false, bad = false;
    double ring[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) ring[q] = S.ring[q];
#pragma unroll
    for (int j = 0; j < kBatchPartStride; ++j) {
      if (j >= nt || done || bad) continue;
      const int kk = S.k + j;
      if (!isfinite(s[j])) {
        bad = true;
        continue;
      }
      const int slot = kk % 5;
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if (q == slot) ring[q] = estv[j];
      if (kk >= 4) {
        const double mean = 0.2 * (ring[0] + ring[1] + ring[2] + ring[3] + ring[4]);
        done = mean < a.thresh;
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) S.ring[q] = ring[q];
    S.terms += nt;  // all terms of the pass are kept
    if (bad) {
      S.flags |= 2;
      stop = true;
    } else if (done) {
      if (S.sub + 1 < P.s) {
        ++S.sub;
        S.kind = kInitSub;
        S.phase = kPhInit;
      } else {
        ++S.step;
        S.sub = 0;
        if (S.step == a.nsteps) {
          S.phase = kPhFinish;
        } else {
          S.kind = kInitStep;
          S.phase = kPhInit;
        }
      }
    } else if (S.k + 2 * nt - 1 > a.m_max) {
      S.flags |= 1;
      stop = true;
    } else {
      S.k += nt;
    }
  }
  // a failed problem still takes the finish pass, which copies the T of its
  // last completed step into the caller's array
  if (stop) S.phase = kPhFinish;
  a.state[pid] = S;
}

__global__ void k_bt_reset(BatchArgs a) {
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid == 0) *a.ndone = 0;
  if (pid < a.ntiles) a.tile[pid].done = 0;
  if (pid >= a.nprob) return;
  BState S{};
  S.phase = kPhInit;
  S.kind = kInitFirst;
  S.k = 1;
  a.state[pid] = S;
}

// Pack one problem's stencil (SoA, stride N) into the batch layout (SoA,
// stride ntot, offset off) and form g = F - J T0 (so that G(T) = J T + g).
__global__ __launch_bounds__(256) void k_batch_pack(int nx, int ny, const double* __restrict__ coef,
                                                    const double* __restrict__ F, const double* __restrict__ T0,
                                                    double* __restrict__ bcoef, double* __restrict__ g,
                                                    long long ntot, long long off) {
  const int N = nx * ny;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const int x = i % nx, y = i / nx;
    double jt = coef[i] * T0[i];
    if (x > 0) jt += coef[N + i] * T0[i - 1];
    if (x + 1 < nx) jt += coef[2 * N + i] * T0[i + 1];
    if (y > 0) jt += coef[3 * N + i] * T0[i - nx];
    if (y + 1 < ny) jt += coef[4 * N + i] * T0[i + nx];
    for (int d = 0; d < 5; ++d) bcoef[d * ntot + off + i] = coef[d * N + i];
    g[off + i] = F[i] - jt;
  }
}

template <int TY, int BY, int NT, bool XCD, class V>
hipError_t launch_work(const BatchArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const size_t bytes = work_lds_bytes<TY, NT, V>();
  if (bytes > 65536) {
    static bool granted = false;
    if (!granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_work<TY, BY, NT, XCD, V>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
      if (e != hipSuccess) return e;
      granted = true;
    }
  }
  launch_timed(k_bt_work<TY, BY, NT, XCD, V>, dim3(a.ntiles), dim3(kBatchTileX, BY), static_cast<unsigned>(bytes), s,
               e0, e1, a);
  return hipGetLastError();
}

template <class V>
hipError_t launch_work_shape(const BatchArgs& a, int shape, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (shape) {
    case 0: return launch_work<8, 8, 4, false, V>(a, s, e0, e1);
    case 1: return launch_work<16, 16, 4, false, V>(a, s, e0, e1);
    case 2: return launch_work<8, 8, 4, true, V>(a, s, e0, e1);
    case 3: return launch_work<16, 8, 4, true, V>(a, s, e0, e1);
    case 4: return launch_work<32, 8, 4, true, V>(a, s, e0, e1);
    case 5: return launch_work<16, 8, 8, true, V>(a, s, e0, e1);
    case 6: return launch_work<8, 8, 8, true, V>(a, s, e0, e1);
    case 7: return launch_work<32, 8, 8, true, V>(a, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t batch_lds_bytes(int shape, int fp32) {
  const size_t vb = fp32 ? sizeof(float) : sizeof(double);
  const size_t rows = kBatchTileRows[shape], nt = kBatchPassTerms[shape];
  return 2 * vb * (rows + 2 * nt) * (kBatchTileX + 2 * nt);
}

hipError_t batch_pack(int nx, int ny, const double* coef, const double* F, const double* T0, double* bcoef,
                      double* g, long long ntot, long long off, hipStream_t s) {
  const int N = nx * ny;
  int blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_batch_pack, dim3(blocks), dim3(256), 0, s, nx, ny, coef, F, T0, bcoef, g, ntot, off);
  return hipGetLastError();
}

hipError_t batch_reset(const BatchArgs& a, hipStream_t s) {
  const int n = a.nprob > a.ntiles ? a.nprob : a.ntiles;  // a thread per problem state and per tile
  hipLaunchKernelGGL(k_bt_reset, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t batch_phase(const BatchArgs& a, int shape, int fp32, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const hipError_t e = fp32 ? launch_work_shape<float>(a, shape, s, e0, e1) : launch_work_shape<double>(a, shape, s, e0, e1);
  if (e != hipSuccess) return e;
  const int per = kCtrlThreads / 64;
  hipLaunchKernelGGL(k_bt_ctrl, dim3((a.nprob + per - 1) / per), dim3(kCtrlThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace erem
