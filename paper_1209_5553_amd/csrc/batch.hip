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

const int kTileShapes[kNumTileShapes][2] = {{256, 4}, {256, 8}, {512, 4}, {1024, 2}};

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
    default: return hipErrorInvalidValue;
  }
}

}  // namespace erem
