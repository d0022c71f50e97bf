// Batched EREM for many independent linear problems in one persistent launch.
//
// Every problem p (its own n_x x n_y grid, packed one after the other) has a
// constant Jacobian J_p and G_p(T) = J_p T + g_p (fixed fluxes, constant
// capacity), so one EREM step is T <- T + h phi1(h J_p)(J_p T + g_p)
// (Eq. EERM) with a Gershgorin interval, substep count and divided
// differences fixed for the whole run.
//
// MI355X mapping: one workgroup owns one whole problem at a time (the batch
// is a queue of problems, largest first, taken round-robin by the resident
// workgroups; with 256 realisations each of the 256 CUs gets one).  All
// steps, substeps and Newton-Leja terms (Eq. newt) of that problem run inside
// the workgroup, separated only by workgroup barriers, and the scaled-norm
// stop test of Sec. 4.2 is a workgroup reduction, so every problem converges
// on its own with no grid-wide synchronisation and no atomics.  The launch
// can be captured in a hipGraph.  The tunable "tile" is the workgroup size
// and the number of cells a thread loads ahead in each Newton pass.
#include "batch.h"

#include <cmath>

namespace erem {

namespace {

template <class V>
__device__ inline V cv(double x) { return static_cast<V>(x); }

// Sum (and max) over the workgroup; every thread gets the result.
template <int NT>
__device__ inline double wg_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

template <int NT>
__device__ inline double wg_max(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s = fmax(s, sh[w]);
  __syncthreads();
  return s;
}

template <int NT, int U, class V>
__global__ __launch_bounds__(NT) void k_batch_blocks(BatchArgs a) {
  __shared__ double sh[NT / 64];
  const long long Ntot = a.ntot;
  const double* c64 = a.coef64;
  const V* cV = reinterpret_cast<const V*>(a.coef);
  V* q0 = reinterpret_cast<V*>(a.q0);
  V* q1 = reinterpret_cast<V*>(a.q1);
  V* pv = reinterpret_cast<V*>(a.p);
  for (int slot = blockIdx.x; slot < a.nprob; slot += gridDim.x) {
    const int pid = a.order[slot];
    const BProb P = a.prob[pid];
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    const long long o = P.off;
    const double* dk = a.dk + P.coef_off;
    const double* sf = a.shift + P.coef_off;
    const double rootN = sqrt(static_cast<double>(N));
    // (x, y) of a thread's cells advance by (sx, sy) per NT cells and (ux, uy) per U NT
    const int sx = NT % nx, sy = NT / nx, ux = (U * NT) % nx, uy = (U * NT) / nx;
    const int x0 = threadIdx.x % nx, y0 = threadIdx.x / nx;
    int terms = 0, flags = 0, steps = 0;
    for (int step = 0; step < a.nsteps && !flags; ++step) {
      // v = J T + g (FP64), max |T| for the error scale
      double mx = 0.0;
      for (int c = threadIdx.x; c < N; c += NT) {
        const long long i = o + c;
        const int x = c % nx, y = c / nx;
        const double* T = a.T;
        double jt = c64[i] * T[i];
        if (x > 0) jt += c64[Ntot + i] * T[i - 1];
        if (x + 1 < nx) jt += c64[2 * Ntot + i] * T[i + 1];
        if (y > 0) jt += c64[3 * Ntot + i] * T[i - nx];
        if (y + 1 < ny) jt += c64[4 * Ntot + i] * T[i + nx];
        a.v[i] = jt + a.g[i];
        mx = fmax(mx, fabs(T[i]));
      }
      const double scal = a.tol_a + a.tol_r * wg_max<NT>(mx, sh);
      for (int j = 0; j < P.s && !flags; ++j) {
        // q_0 = v + J u (u = 0 on the first substep), p = d_0 q_0
        double s0 = 0.0;
        for (int c = threadIdx.x; c < N; c += NT) {
          const long long i = o + c;
          double w = a.v[i];
          if (j > 0) {
            const int x = c % nx, y = c / nx;
            const double* u = a.u;
            double ju = c64[i] * u[i];
            if (x > 0) ju += c64[Ntot + i] * u[i - 1];
            if (x + 1 < nx) ju += c64[2 * Ntot + i] * u[i + 1];
            if (y > 0) ju += c64[3 * Ntot + i] * u[i - nx];
            if (y + 1 < ny) ju += c64[4 * Ntot + i] * u[i + nx];
            w += ju;
          }
          const V q = cv<V>(w);
          q0[i] = q;
          pv[i] = cv<V>(dk[0]) * q;
          s0 += static_cast<double>(q) * static_cast<double>(q);
        }
        double ring[5];
        ring[0] = fabs(P.delta * dk[0]) * sqrt(wg_sum<NT>(s0, sh)) / (rootN * scal);
        bool done = false;
        for (int k = 1; k <= a.m_max; ++k) {
          const V* __restrict__ qin = (k & 1) ? q0 : q1;
          V* __restrict__ qout = (k & 1) ? q1 : q0;
          const V ig = cv<V>(P.inv_g), sk = cv<V>(sf[k]), dkk = cv<V>(dk[k]);
          double sk2 = 0.0;
          int x = x0, y = y0;
          for (int c = threadIdx.x; c < N; c += U * NT) {
            // U cells per thread with every load issued before any use
            long long ii[U];
            bool in[U], hw[U], he[U], hs[U], hn[U];
            int xu = x, yu = y;
#pragma unroll
            for (int u = 0; u < U; ++u) {
              in[u] = c + u * NT < N;
              ii[u] = o + (in[u] ? c + u * NT : N - 1);
              hw[u] = in[u] && xu > 0;
              he[u] = in[u] && xu + 1 < nx;
              hs[u] = in[u] && yu > 0;
              hn[u] = in[u] && yu + 1 < ny;
              xu += sx;
              yu += sy;
              if (xu >= nx) {
                xu -= nx;
                ++yu;
              }
            }
            V qc[U], a0[U], aw[U], ae[U], as[U], an[U], qw[U], qe[U], qs[U], qn[U], pp[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const long long i = ii[u];
              qc[u] = qin[i];
              a0[u] = cV[i];
              aw[u] = cV[Ntot + i];
              ae[u] = cV[2 * Ntot + i];
              as[u] = cV[3 * Ntot + i];
              an[u] = cV[4 * Ntot + i];
              qw[u] = qin[hw[u] ? i - 1 : i];
              qe[u] = qin[he[u] ? i + 1 : i];
              qs[u] = qin[hs[u] ? i - nx : i];
              qn[u] = qin[hn[u] ? i + nx : i];
              pp[u] = pv[i];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              V jq = a0[u] * qc[u];
              if (hw[u]) jq += aw[u] * qw[u];
              if (he[u]) jq += ae[u] * qe[u];
              if (hs[u]) jq += as[u] * qs[u];
              if (hn[u]) jq += an[u] * qn[u];
              const V r = jq * ig - sk * qc[u];
              if (in[u]) {
                pv[ii[u]] = pp[u] + dkk * r;
                qout[ii[u]] = r;
                sk2 += static_cast<double>(r) * static_cast<double>(r);
              }
            }
            x += ux;
            y += uy;
            if (x >= nx) {
              x -= nx;
              ++y;
            }
          }
          const double S = wg_sum<NT>(sk2, sh);  // also orders qout before the next term
          ++terms;
          if (!isfinite(S)) {
            flags |= 2;
            break;
          }
          ring[k % 5] = fabs(P.delta * dk[k]) * sqrt(S) / (rootN * scal);
          if (k >= 4) {
            const double mean = 0.2 * (ring[0] + ring[1] + ring[2] + ring[3] + ring[4]);
            if (mean < a.thresh) {
              done = true;
              break;
            }
          }
        }
        if (!done) {
          if (!flags) flags |= 1;
          break;
        }
        // substep end: u += delta p (earlier substeps) or T += u + delta p (last)
        const bool last = j + 1 == P.s;
        for (int c = threadIdx.x; c < N; c += NT) {
          const long long i = o + c;
          const double pi = static_cast<double>(pv[i]);
          if (!last) a.u[i] = (j == 0 ? 0.0 : a.u[i]) + P.delta * pi;
          else a.T[i] += (P.s > 1 ? a.u[i] : 0.0) + P.delta * pi;
        }
        __syncthreads();
      }
      if (!flags) ++steps;
    }
    if (threadIdx.x == 0) {
      BDyn& D = a.dyn[pid];
      D.terms = terms;
      D.flags = flags;
      D.step = steps;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fused variant: the same per-problem workgroup (1024 threads), but the Newton
// terms go four at a time.  For each group of four terms the workgroup walks
// its problem in 64 x 16 tiles; a tile stages q_{k-1} with a halo of four
// cells and the stencil with a halo of three in LDS, computes the four terms
// on shrinking regions (the last on the tile), and writes only p and the
// group's last q.  The stop test of Sec. 4.2 runs on the group's four
// estimates in order, as the single-problem path does after every four terms.
// ---------------------------------------------------------------------------
constexpr int kFX = 64, kFY = 16, kFThreads = kFX * kFY;
constexpr int kFWQ = kFX + 8, kFHQ = kFY + 8;   // q_{k-1}: halo 4
constexpr int kFWI = kFX + 6, kFHI = kFY + 6;   // stencil, intermediates: halo 3
static_assert(kFHQ * kFWQ <= 2 * kFThreads && kFHI * kFWI <= 2 * kFThreads, "two staged values per thread");
#ifndef EREM_BATCH_LOAD_GROUPS
#define EREM_BATCH_LOAD_GROUPS 2
#endif
constexpr int kFLoadGroups = EREM_BATCH_LOAD_GROUPS;  // 1 or 2
static_assert(kFLoadGroups == 1 || kFLoadGroups == 2, "one or two load groups");

template <class V>
constexpr size_t fused_lds_bytes() {
  return sizeof(V) * (static_cast<size_t>(kFHQ) * kFWQ + 7 * static_cast<size_t>(kFHI) * kFWI);
}

template <class V>
__global__ __launch_bounds__(kFThreads) void k_batch_fused(BatchArgs a) {
  extern __shared__ unsigned char fsm[];
  V(*sq)[kFWQ] = reinterpret_cast<V(*)[kFWQ]>(fsm);
  V(*sc)[kFHI][kFWI] = reinterpret_cast<V(*)[kFHI][kFWI]>(fsm + sizeof(V) * kFHQ * kFWQ);
  V(*sb)[kFHI][kFWI] = sc + 5;
  __shared__ double sh[kFThreads / 64];
  __shared__ double red[4][kFThreads / 64];
  const int tid = threadIdx.x;
  const int lx = tid % kFX, ly = tid / kFX;
  const long long Ntot = a.ntot;
  const double* c64 = a.coef64;
  const V* cV = reinterpret_cast<const V*>(a.coef);
  V* q0 = reinterpret_cast<V*>(a.q0);
  V* q1 = reinterpret_cast<V*>(a.q1);
  V* pv = reinterpret_cast<V*>(a.p);
  for (int slot = blockIdx.x; slot < a.nprob; slot += gridDim.x) {
    const int pid = a.order[slot];
    const BProb P = a.prob[pid];
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    const long long o = P.off;
    const double* dk = a.dk + P.coef_off;
    const double* sf = a.shift + P.coef_off;
    const double rootN = sqrt(static_cast<double>(N));
    int terms = 0, flags = 0, steps = 0;
    for (int step = 0; step < a.nsteps && !flags; ++step) {
      double mx = 0.0;
      for (int c = tid; c < N; c += kFThreads) {
        const long long i = o + c;
        const int x = c % nx, y = c / nx;
        const double* T = a.T;
        double jt = c64[i] * T[i];
        if (x > 0) jt += c64[Ntot + i] * T[i - 1];
        if (x + 1 < nx) jt += c64[2 * Ntot + i] * T[i + 1];
        if (y > 0) jt += c64[3 * Ntot + i] * T[i - nx];
        if (y + 1 < ny) jt += c64[4 * Ntot + i] * T[i + nx];
        a.v[i] = jt + a.g[i];
        mx = fmax(mx, fabs(T[i]));
      }
      const double scal = a.tol_a + a.tol_r * wg_max<kFThreads>(mx, sh);
      for (int j = 0; j < P.s && !flags; ++j) {
        double s0 = 0.0;
        for (int c = tid; c < N; c += kFThreads) {
          const long long i = o + c;
          double w = a.v[i];
          if (j > 0) {
            const int x = c % nx, y = c / nx;
            const double* u = a.u;
            double ju = c64[i] * u[i];
            if (x > 0) ju += c64[Ntot + i] * u[i - 1];
            if (x + 1 < nx) ju += c64[2 * Ntot + i] * u[i + 1];
            if (y > 0) ju += c64[3 * Ntot + i] * u[i - nx];
            if (y + 1 < ny) ju += c64[4 * Ntot + i] * u[i + nx];
            w += ju;
          }
          const V q = cv<V>(w);
          q0[i] = q;
          pv[i] = cv<V>(dk[0]) * q;
          s0 += static_cast<double>(q) * static_cast<double>(q);
        }
        double ring[5];
        ring[0] = fabs(P.delta * dk[0]) * sqrt(wg_sum<kFThreads>(s0, sh)) / (rootN * scal);
        bool done = false;
        const V ig = cv<V>(P.inv_g);
        for (int k = 1; k + 3 <= a.m_max; k += 4) {
          const int g = (k - 1) / 4;
          const V* __restrict__ qin = (g & 1) ? q1 : q0;
          V* __restrict__ qout = (g & 1) ? q0 : q1;
          double part[4] = {0.0, 0.0, 0.0, 0.0};
          for (int y0 = 0; y0 < ny; y0 += kFY)
            for (int x0 = 0; x0 < nx; x0 += kFX) {
              // the tile's loads are issued in groups before their LDS
              // stores (q with the first half of the stencil, then the
              // second half), so the tile waits for a few memory latencies
              // instead of one per loop trip
              const int gx = x0 + lx, gy = y0 + ly;
              const bool own = gx < nx && gy < ny;
              const long long i = o + gx + nx * gy;
              V acc;
#pragma unroll
              for (int grp = 0; grp < kFLoadGroups; ++grp) {
                constexpr int UG = 2 / kFLoadGroups;  // stencil values per thread and group
                V rq[2], rc[5][UG];
                if (grp == 0) {
#pragma unroll
                  for (int u = 0; u < 2; ++u) {
                    const int e = tid + u * kFThreads;
                    const int ry = e / kFWQ, rx = e - ry * kFWQ;
                    const int qx = x0 - 4 + rx, qy = y0 - 4 + ry;
                    rq[u] = (e < kFHQ * kFWQ && qx >= 0 && qx < nx && qy >= 0 && qy < ny) ? qin[o + qx + nx * qy]
                                                                                        : V(0);
                  }
                  acc = own ? pv[i] : V(0);
                }
#pragma unroll
                for (int uu = 0; uu < UG; ++uu) {
                  const int e = tid + (grp * UG + uu) * kFThreads;
                  const int ry = e / kFWI, rx = e - ry * kFWI;
                  const int cx = x0 - 3 + rx, cy = y0 - 3 + ry;
                  const bool in = e < kFHI * kFWI && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
                  const long long ci = o + cx + nx * cy;
#pragma unroll
                  for (int d = 0; d < 5; ++d) rc[d][uu] = in ? cV[d * Ntot + ci] : V(0);
                }
                if (grp == 0) {
#pragma unroll
                  for (int u = 0; u < 2; ++u) {
                    const int e = tid + u * kFThreads;
                    if (e < kFHQ * kFWQ) sq[e / kFWQ][e % kFWQ] = rq[u];
                  }
                }
#pragma unroll
                for (int uu = 0; uu < UG; ++uu) {
                  const int e = tid + (grp * UG + uu) * kFThreads;
                  if (e < kFHI * kFWI) {
#pragma unroll
                    for (int d = 0; d < 5; ++d) sc[d][e / kFWI][e % kFWI] = rc[d][uu];
                  }
                }
              }
              __syncthreads();
              V last = V(0);
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int h = 3 - t;
                const V shk = cv<V>(sf[k + t]);
                const int w = kFX + 2 * h, hh = kFY + 2 * h;
                V(*outb)[kFWI] = sb[t & 1];
                for (int e = tid; e < w * hh; e += kFThreads) {
                  const int ry = e / w, rx = e - ry * w;
                  const int iy = ry + t, ix = rx + t;
                  V qc, qw, qe, qs, qn;
                  if (t == 0) {
                    qc = sq[iy + 1][ix + 1];
                    qw = sq[iy + 1][ix];
                    qe = sq[iy + 1][ix + 2];
                    qs = sq[iy][ix + 1];
                    qn = sq[iy + 2][ix + 1];
                  } else {
                    const V(*prev)[kFWI] = sb[(t - 1) & 1];
                    qc = prev[iy][ix];
                    qw = prev[iy][ix - 1];
                    qe = prev[iy][ix + 1];
                    qs = prev[iy - 1][ix];
                    qn = prev[iy + 1][ix];
                  }
                  V jq = sc[0][iy][ix] * qc;
                  jq += sc[1][iy][ix] * qw;
                  jq += sc[2][iy][ix] * qe;
                  jq += sc[3][iy][ix] * qs;
                  jq += sc[4][iy][ix] * qn;
                  outb[iy][ix] = jq * ig - shk * qc;
                }
                __syncthreads();
                const V qo = outb[ly + 3][lx + 3];
                acc += cv<V>(dk[k + t]) * qo;
                if (own) part[t] += static_cast<double>(qo) * static_cast<double>(qo);
                last = qo;
              }
              if (own) {
                pv[i] = acc;
                qout[i] = last;
              }
              __syncthreads();  // the next tile reuses LDS
            }
          // the four sums, in the same order in every thread
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            double v = part[t];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if ((tid & 63) == 0) red[t][tid >> 6] = v;
          }
          __syncthreads();
          double S[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            double v = 0.0;
            for (int w = 0; w < kFThreads / 64; ++w) v += red[t][w];
            S[t] = v;
          }
          __syncthreads();
          terms += 4;
          for (int t = 0; t < 4 && !done; ++t) {
            const int kk = k + t;
            if (!isfinite(S[t])) {
              flags |= 2;
              break;
            }
            ring[kk % 5] = fabs(P.delta * dk[kk]) * sqrt(S[t]) / (rootN * scal);
            if (kk >= 4) {
              const double mean = 0.2 * (ring[0] + ring[1] + ring[2] + ring[3] + ring[4]);
              if (mean < a.thresh) done = true;
            }
          }
          if (flags || done) break;  // the substep end needs p only
        }
        if (!done) {
          if (!flags) flags |= 1;
          break;
        }
        const bool lastsub = j + 1 == P.s;
        for (int c = tid; c < N; c += kFThreads) {
          const long long i = o + c;
          const double pi = static_cast<double>(pv[i]);
          if (!lastsub) a.u[i] = (j == 0 ? 0.0 : a.u[i]) + P.delta * pi;
          else a.T[i] += (P.s > 1 ? a.u[i] : 0.0) + P.delta * pi;
        }
        __syncthreads();
      }
      if (!flags) ++steps;
    }
    if (tid == 0) {
      BDyn& D = a.dyn[pid];
      D.terms = terms;
      D.flags = flags;
      D.step = steps;
    }
    __syncthreads();
  }
}

hipError_t launch_fused(const BatchArgs& a, int fp32, int grid, hipStream_t s) {
  static bool granted[2] = {false, false};
  const size_t bytes = fp32 ? fused_lds_bytes<float>() : fused_lds_bytes<double>();
  if (!granted[fp32]) {
    const hipError_t e = fp32 ? hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_fused<float>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes))
                              : hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_fused<double>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (e != hipSuccess) return e;
    granted[fp32] = true;
  }
  if (fp32)
    hipLaunchKernelGGL(k_batch_fused<float>, dim3(grid), dim3(kFThreads), bytes, s, a);
  else
    hipLaunchKernelGGL(k_batch_fused<double>, dim3(grid), dim3(kFThreads), bytes, s, a);
  return hipGetLastError();
}

template <int NT, int U, class V>
hipError_t launch_variant(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_blocks<NT, U, V>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

// Pack one problem's stencil (SoA, stride N) into the batch layout (SoA,
// stride ntot, offset off) and form g = F - J T0 (so that G(T) = J T + g).
__global__ __launch_bounds__(256) void k_batch_pack(int nx, int ny, const double* __restrict__ coef,
                                          const double* __restrict__ F, const double* __restrict__ T0,
                                          double* __restrict__ bcoef, double* __restrict__ g, long long ntot,
                                          long long off) {
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

}  // namespace

// {threads, cells loaded ahead per thread}; the last shape is the fused
// variant (1024 threads, four Newton terms per pass over 64 x 16 tiles).
const int kTileShapes[kNumTileShapes][2] = {{256, 4}, {256, 8}, {512, 4}, {1024, 2}, {1024, 0}};

hipError_t batch_pack(int nx, int ny, const double* coef, const double* F, const double* T0, double* bcoef,
                      double* g, long long ntot, long long off, hipStream_t s) {
  const int N = nx * ny;
  int blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_batch_pack, dim3(blocks), dim3(256), 0, s, nx, ny, coef, F, T0, bcoef, g, ntot, off);
  return hipGetLastError();
}

hipError_t batch_launch(const BatchArgs& a, int shape, int fp32, int grid, hipStream_t s) {
  switch (shape * 2 + fp32) {
    case 0: return launch_variant<256, 4, double>(a, grid, s);
    case 1: return launch_variant<256, 4, float>(a, grid, s);
    case 2: return launch_variant<256, 8, double>(a, grid, s);
    case 3: return launch_variant<256, 8, float>(a, grid, s);
    case 4: return launch_variant<512, 4, double>(a, grid, s);
    case 5: return launch_variant<512, 4, float>(a, grid, s);
    case 6: return launch_variant<1024, 2, double>(a, grid, s);
    case 7: return launch_variant<1024, 2, float>(a, grid, s);
    case 8: return launch_fused(a, 0, grid, s);
    case 9: return launch_fused(a, 1, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace erem
