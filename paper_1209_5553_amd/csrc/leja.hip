// Newton-Leja evaluation of phi1(delta J) v on the device (Sec. 4.2):
//
//   q_0 = v,  p_0 = d_0 q_0,
//   q_k = ((J - c I)/gamma - xi_{k-1} I) q_{k-1},  p_k = p_{k-1} + d_k q_k   (Eq. newt)
//
// One fused pass per term reads the stencil of J and q_{k-1}, updates p and
// writes q_k; each block also stores its partial sum of q_k^2 (in FP64 in
// both precisions).  A one-workgroup check kernel, launched after every few
// terms, reduces those partials in a fixed order (so results are
// reproducible bit for bit), forms the scaled error estimates
// ||delta d_k q_k|| = |delta d_k| ||q_k||_2 / (sqrt(N) scal) and applies the
// stop test 10^p * mean(last five estimates) < 1 (Sec. 4.2).  Once it holds,
// later term launches return at entry.
//
// Value type V is double (FP64 path) or float (mixed path: FP32 stencil,
// vectors and accumulation; FP64 divided differences, norms and update).
#include "device.h"
#include "leja.h"

#include <cmath>

namespace erem {

namespace {

template <class V>
__device__ inline V to_v(double x) { return static_cast<V>(x); }

// Sum of one double over the 256-thread cell block; valid in thread 0.
__device__ inline double block_sum256(double v) {
  __shared__ double sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int t = threadIdx.x + threadIdx.y * kBX;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  return t == 0 ? sh[0] + sh[1] + sh[2] + sh[3] : 0.0;
}

__device__ inline int block_id() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

__global__ void k_leja_reset(LejaState* st, int nslots, int nterms) {
  for (int s = blockIdx.x; s < nslots; s += gridDim.x) {
    LejaState* t = st + s;
    for (int j = threadIdx.x; j <= nterms; j += blockDim.x) t->sums[j] = 0.0;
    if (threadIdx.x == 0) {
      t->stopped = -1;
      t->nonfinite = 0;
      t->checked = -1;
    }
  }
}

template <class V>
__global__ __launch_bounds__(kThreads) void k_leja_init(Dims d, const LejaCoef* __restrict__ cf,
                                              const double* __restrict__ v, V* __restrict__ q0,
                                              V* __restrict__ p, double* __restrict__ part) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const V vi = to_v<V>(v[i]);
    q0[i] = vi;
    p[i] = to_v<V>(cf->dk[0]) * vi;
    s = static_cast<double>(vi) * static_cast<double>(vi);
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = s;  // ring slot 0
}

template <int DIM, class V>
__global__ __launch_bounds__(kThreads) void k_leja_term(Dims d, const LejaCoef* __restrict__ cf,
                                              const V* __restrict__ coef, const V* __restrict__ qin,
                                              V* __restrict__ qout, V* __restrict__ p,
                                              const LejaState* __restrict__ st, double* __restrict__ part,
                                              int nb, int k) {
  // the stop flag is read while the operand loads are in flight; nothing is
  // written before it is known
  const bool stopped = *(volatile const int*)&st->stopped >= 0;
  const int tile = xcd_tile_id();
  const int tx = tile % gridDim.x, ty = (tile / gridDim.x) % gridDim.y;
  const int x = tx * kBX + threadIdx.x;
  const int y = ty * kBY + threadIdx.y;
  const int z = tile / (gridDim.x * gridDim.y);
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const int N = d.N;
    const int i = x + d.nx * (y + d.ny * z);
    const V qi = qin[i];
    V jq = coef[i] * qi;
    jq += coef[N + i] * qin[x > 0 ? i - 1 : i];
    jq += coef[2 * N + i] * qin[x + 1 < d.nx ? i + 1 : i];
    jq += coef[3 * N + i] * qin[y > 0 ? i - d.nx : i];
    jq += coef[4 * N + i] * qin[y + 1 < d.ny ? i + d.nx : i];
    if (DIM == 3) {
      const int pl = d.nx * d.ny;
      jq += coef[5 * N + i] * qin[z > 0 ? i - pl : i];
      jq += coef[6 * N + i] * qin[z + 1 < d.nz ? i + pl : i];
    }
    const V r = jq * to_v<V>(cf->inv_g) - to_v<V>(cf->shift[k]) * qi;
    const V pi = p[i];
    if (stopped) return;
    p[i] = pi + to_v<V>(cf->dk[k]) * r;
    qout[i] = r;
    s = static_cast<double>(r) * static_cast<double>(r);
  } else if (stopped) {
    return;
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[(k % kLejaRing) * nb + tile] = s;  // slot of the tile
}

// NT Newton terms in one pass (2D), NT = 2 or 4: q_{k-1} is staged in LDS on
// the block's 64 x TY tile plus a halo of NT cells and the stencil on the
// tile plus a halo of NT - 1; term k + t is then computed on the tile plus a
// halo of NT - 1 - t, so the last one lands on the tile.  p gets d_k q_k,
// then d_{k+1} q_{k+1}, ... (the order of single passes); the intermediate
// q's never go to memory.  Each thread owns TY / 4 cells of the tile (rows
// threadIdx.y, threadIdx.y + 4, ...).  The per-block partial sums of every
// term's q^2 go to the term's ring slot in the slot layout of the one-term
// kernel (one slot per 64 x 4 band): the block's sum in the slot of its first
// band, zeros in the slots of its other bands, so the check kernel reduces
// the same number of slots in the same order.
template <int NT, int TY, int BY, class V>
__global__ __launch_bounds__(kBX * BY) void k_leja_terms(Dims d, const LejaCoef* __restrict__ cf,
                                               const V* __restrict__ coef, const V* __restrict__ qin,
                                               V* __restrict__ qout, V* __restrict__ p,
                                               const LejaState* __restrict__ st, double* __restrict__ part, int nb,
                                               int k) {
  static_assert(TY % BY == 0 && TY % kBY == 0, "whole thread rows and 64 x 4 bands per tile");
  constexpr int NTH = kBX * BY;                     // threads
  constexpr int R = TY / BY;                        // own cells per thread
  constexpr int H = NT - 1;                         // halo of the stencil / intermediates
  constexpr int WQ = kBX + 2 * NT, HQ = TY + 2 * NT;
  constexpr int WI = kBX + 2 * H, HI = TY + 2 * H;
  __shared__ V sq[HQ][WQ];           // q_{k-1}, halo NT
  __shared__ V sc[5][HI][WI];        // stencil, halo NT - 1
  __shared__ V sb[2][HI][WI];        // intermediates, halo NT - 1
  const bool stopped = *(volatile const int*)&st->stopped >= 0;
  const int nx = d.nx, ny = d.ny, N = d.N;
  // plain placement: the eight XCDs take interleaved tile columns, each
  // column's vertical halos stay in one L2 (measured slightly faster here
  // than contiguous tile ranges per XCD)
  const int bx = blockIdx.x, by = blockIdx.y;
  const int x0 = bx * kBX, y0 = by * TY;
  const int tid = threadIdx.x + threadIdx.y * kBX;
  // every load of the tile is issued (into registers) before the first LDS
  // store, so the tile waits for one memory latency instead of one per trip
  constexpr int UQ = (HQ * WQ + NTH - 1) / NTH, UI = (HI * WI + NTH - 1) / NTH;
  V rq[UQ], rc[5][UI];
#pragma unroll
  for (int u = 0; u < UQ; ++u) {
    const int e = tid + u * NTH;
    const int ly = e / WQ, lx = e - ly * WQ;
    const int gx = x0 - NT + lx, gy = y0 - NT + ly;
    rq[u] = (e < HQ * WQ && gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? qin[gx + nx * gy] : V(0);
  }
#pragma unroll
  for (int u = 0; u < UI; ++u) {
    const int e = tid + u * NTH;
    const int ly = e / WI, lx = e - ly * WI;
    const int gx = x0 - H + lx, gy = y0 - H + ly;
    const bool in = e < HI * WI && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int j = gx + nx * gy;
#pragma unroll
    for (int c = 0; c < 5; ++c) rc[c][u] = in ? coef[c * N + j] : V(0);
  }
  const int gx = x0 + threadIdx.x;
  V acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = y0 + threadIdx.y + BY * r;
    acc[r] = (gx < nx && gy < ny) ? p[gx + nx * gy] : V(0);
  }
#pragma unroll
  for (int u = 0; u < UQ; ++u) {
    const int e = tid + u * NTH;
    if (e < HQ * WQ) sq[e / WQ][e % WQ] = rq[u];
  }
#pragma unroll
  for (int u = 0; u < UI; ++u) {
    const int e = tid + u * NTH;
    if (e < HI * WI) {
#pragma unroll
      for (int c = 0; c < 5; ++c) sc[c][e / WI][e % WI] = rc[c][u];
    }
  }
  if (stopped) return;  // stop test already passed
  __syncthreads();
  const V ig = to_v<V>(cf->inv_g);
  double a[NT];
  V last[R];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int h = H - t;  // halo of the region computed in this phase
    const V sh = to_v<V>(cf->shift[k + t]);
    const int w = kBX + 2 * h, hh = TY + 2 * h;
    V(*out)[WI] = sb[t & 1];
    for (int e = tid; e < w * hh; e += NTH) {
      const int ry = e / w, rx = e - ry * w;
      const int iy = ry + t, ix = rx + t;  // position in the halo-H buffers
      V qc, qw, qe, qs, qn;
      if (t == 0) {
        qc = sq[iy + 1][ix + 1];
        qw = sq[iy + 1][ix];
        qe = sq[iy + 1][ix + 2];
        qs = sq[iy][ix + 1];
        qn = sq[iy + 2][ix + 1];
      } else {
        const V(*prev)[WI] = sb[(t - 1) & 1];
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
      out[iy][ix] = jq * ig - sh * qc;  // zero outside the grid (stencil and q are)
    }
    __syncthreads();
    const V dk = to_v<V>(cf->dk[k + t]);
    double sq2 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ly = threadIdx.y + BY * r;
      const V qo = out[ly + H][threadIdx.x + H];
      acc[r] += dk * qo;
      if (gx < nx && y0 + ly < ny) sq2 += static_cast<double>(qo) * static_cast<double>(qo);
      last[r] = qo;
    }
    a[t] = sq2;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = y0 + threadIdx.y + BY * r;
    if (gx < nx && gy < ny) {
      p[gx + nx * gy] = acc[r];
      qout[gx + nx * gy] = last[r];
    }
  }
  __shared__ double red[NT][BY];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double v = a[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) red[t][tid >> 6] = v;
  }
  __syncthreads();
  // slot layout of the one-term kernel: band b of this tile is global band
  // by * NB + b, slot bx + gridDim.x * band
  constexpr int NB = TY / kBY;  // 64 x 4 bands per tile
  const int nbands = (ny + kBY - 1) / kBY;
  for (int e = tid; e < NT * NB; e += NTH) {
    const int t = e / NB, b = e - t * NB;
    const int band = by * NB + b;
    if (band < nbands) {
      double sum = 0.0;
      if (b == 0)
        for (int w = 0; w < BY; ++w) sum += red[t][w];
      part[((k + t) % kLejaRing) * nb + bx + gridDim.x * band] = sum;
    }
  }
}

// Reduce the partials of terms k1..k2 (in order), record their sums and
// apply the stop test.  One workgroup of kCheckThreads threads.
__global__ __launch_bounds__(kCheckThreads) void k_leja_check(const LejaCoef* __restrict__ cf, LejaState* st,
                                                    const double* __restrict__ part, int nb, int k1, int k2) {
  if (st->stopped >= 0) return;
  __shared__ double sh[kCheckThreads / 64];
  __shared__ int stop_sh;
  for (int k = k1; k <= k2; ++k) {
    const double* pk = part + (k % kLejaRing) * nb;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kCheckThreads) v += pk[b];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double S = 0.0;
      for (int w = 0; w < kCheckThreads / 64; ++w) S += sh[w];
      st->sums[k] = S;
      int stop = 0;
      if (!isfinite(S)) {
        st->nonfinite = 1;
        stop = 1;
      } else if (k >= 4) {
        double mean = 0.0;
        for (int j = k - 4; j <= k; ++j) mean += cf->estf[j] * sqrt(st->sums[j]);
        mean *= 0.2;
        stop = mean < cf->thresh;
      }
      if (stop) st->stopped = k;
      st->checked = k;
      stop_sh = stop;
    }
    __syncthreads();
    if (stop_sh) return;
  }
}

// u = (first ? 0 : u) + delta * p (+ zt)  (FP64 update of the substep
// increment; zt, when not null, is a fixed vector added on every substep)
template <class V>
__global__ __launch_bounds__(kThreads) void k_substep_update(Dims d, double* __restrict__ u, const V* __restrict__ p,
                                                   double delta, int first, const double* __restrict__ zt) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const double pi = static_cast<double>(p[i]);
  double r = first ? delta * pi : u[i] + delta * pi;
  if (zt) r += zt[i];
  u[i] = r;
}

__global__ void k_cast_f32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    b[i] = static_cast<float>(a[i]);
}

constexpr int kCoefM = kCoefMaxN + 1;  // largest order of the augmented matrix
constexpr int kCoefLd = kCoefM + 1;     // row stride of the LDS matrices (rows on distinct banks)
constexpr int kTaylorDegree = 20;

// Coefficients of one phi1 evaluation from the reduction slots (one
// workgroup of 16 x 16 threads; launch_leja_coef).  Thread (ty, tx) owns the
// entries (ty + 16 a, tx + 16 b), a, b < RB, of the lower triangle of the two
// LDS matrices; RB = ceil((n + 1) / 16) blocks of 16 rows cover the matrix.
template <int RB>
__global__ __launch_bounds__(kCoefThreads) void k_leja_coef(LejaCoefArgs a) {
  // every operation rounded on its own, in the host routine's order, so the
  // coefficients equal the host's bit for bit
#pragma clang fp contract(off)
  __shared__ double sA[kCoefM * kCoefLd], sB[kCoefM * kCoefLd];
  __shared__ double dg[kCoefM], sd[kCoefM], dd[kCoefM], inv[kTaylorDegree + 1];
  __shared__ double bc[6];
  __shared__ double wmax[kCoefThreads / 64];
  __shared__ int okf, hit;
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  if (t < 64) {
    // fold the 64 slots of each target (the encodings order like the values)
    unsigned long long lo = a.red->lo[t], hi = a.red->hi[t];
    unsigned long long sm = a.red->tmax[t];
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long l2 = __shfl_xor(lo, off, 64);
      const unsigned long long h2 = __shfl_xor(hi, off, 64);
      const unsigned long long s2 = __shfl_xor(sm, off, 64);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
      sm = s2 > sm ? s2 : sm;
    }
    if (t == 0) {
      const double alpha = ord_decode(lo), beta = ord_decode(hi), tm = ord_decode(sm);
      const double width = beta - alpha;
      const double mag = fmax(fabs(alpha), fabs(beta));
      const double scal = a.tol_a + a.tol_r * tm;
      bool ok = isfinite(tm) && scal > 0.0 && isfinite(width) && !(width <= 1e-14 * mag || width == 0.0);
      if (ok) {
        int s = 1;
        if (a.rho > 0.0) {
          const double q = ceil(a.h * width / a.rho);
          s = q >= a.smax ? a.smax : (q > 1.0 ? static_cast<int>(q) : 1);
        }
        ok = s == a.s;
      }
      const double cc = 0.5 * (alpha + beta), gg = 0.25 * (beta - alpha);
      const double delta = a.h / a.s;
      bc[0] = cc;
      bc[1] = gg;
      bc[2] = delta;
      bc[3] = delta * cc;
      bc[4] = delta * gg;
      bc[5] = scal;
      okf = ok;
      hit = ok && a.cache->n >= a.n && a.cache->hc == bc[3] && a.cache->hg == bc[4];
    }
  }
  __syncthreads();
  if (!okf) {
    for (int j = t; j < a.s; j += kCoefThreads) {
      a.st[j].stopped = 0;
      a.st[j].checked = -2;  // refused: the host evaluates again
    }
    return;
  }
  const int n = a.n, M = n + 1;
  if (hit) {
    if (t < n) dd[t] = a.cache->d[t];
  } else {
    // Augmented lower-bidiagonal matrix: diagonal (0, hc + hg xi_0, ...,
    // hc + hg xi_{n-1}), subdiagonal A[1][0] = 1, A[i][i-1] = hg (i >= 2).
    // The first column of its exponential is (1, phi1(hc I + hg L) e_1), the
    // divided differences of phi1(hc + hg xi).  Scaling by 2^-q brings its
    // 1-norm (the largest column sum) to at most 1/2.
    const double hc = bc[3], hg = bc[4];
    double nrm = 0.0;
    if (t < M) {
      const double dj = t == 0 ? 0.0 : hc + hg * a.xi[t - 1];
      const double below = t + 1 < M ? (t == 0 ? 1.0 : fabs(hg)) : 0.0;
      nrm = fabs(dj) + below;
    }
    for (int off = 32; off > 0; off >>= 1) nrm = fmax(nrm, __shfl_xor(nrm, off, 64));
    if ((t & 63) == 0) wmax[t >> 6] = nrm;
    // E = I on the leading M x M block, zero elsewhere (rows and columns past
    // M and the upper triangle stay zero throughout)
    for (int e = t; e < kCoefM * kCoefLd; e += kCoefThreads) {
      const int i = e / kCoefLd;
      sA[e] = (e - i * kCoefLd == i && i < M) ? 1.0 : 0.0;
      sB[e] = 0.0;
    }
    if (t >= 1 && t <= kTaylorDegree) inv[t] = 1.0 / t;
    __syncthreads();
    nrm = wmax[0];
    for (int w = 1; w < kCoefThreads / 64; ++w) nrm = fmax(nrm, wmax[w]);
    int nsq = 0;  // ceil(log2(nrm / 0.5)) exactly, as on the host
    if (nrm > 0.5) {
      int ex = 0;
      const double f = frexp(nrm / 0.5, &ex);
      nsq = f == 0.5 ? ex - 1 : ex;
    }
    const double scale = ldexp(1.0, -nsq);
    if (t < M) {
      dg[t] = (t == 0 ? 0.0 : hc + hg * a.xi[t - 1]) * scale;
      sd[t] = (t == 0 ? 0.0 : (t == 1 ? 1.0 : hg)) * scale;
    }
    __syncthreads();
    double* E = sA;
    double* T = sB;
    // Taylor polynomial by Horner's rule, E <- I + X E / k, on the lower
    // triangle
    for (int k = kTaylorDegree; k >= 1; --k) {
      const double ik = inv[k];
#pragma unroll
      for (int ra = 0; ra < RB; ++ra) {
        const int i = ty + 16 * ra;
        if (i >= M) break;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int j = tx + 16 * rb;
          if (j > i) break;
          double v = i == 0 ? dg[0] * E[0] * ik
                            : (dg[i] * E[i * kCoefLd + j] + sd[i] * E[(i - 1) * kCoefLd + j]) * ik;
          if (i == j) v += 1.0;
          T[i * kCoefLd + j] = v;
        }
      }
      __syncthreads();
      double* x = E;
      E = T;
      T = x;
    }
    // Squaring; the last square forms the first column only.  A thread's
    // sums run over every k < 16 RB in order: the products outside
    // j <= k <= i hold a zero of the upper triangle or of the rows and
    // columns past M and add nothing, so each sum equals the host's over
    // k = j .. i.
    for (int q = 0; q < nsq; ++q) {
      if (q + 1 == nsq) {
        if (t < M) {
          double acc = 0.0;
          for (int k = 0; k <= t; ++k) acc += E[t * kCoefLd + k] * E[k * kCoefLd];
          T[t * kCoefLd] = acc;
        }
      } else {
        double acc[RB][RB];
#pragma unroll
        for (int ra = 0; ra < RB; ++ra)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[ra][rb] = 0.0;
#pragma unroll
        for (int k = 0; k < 16 * RB; ++k) {
          double ar[RB], br[RB];
#pragma unroll
          for (int ra = 0; ra < RB; ++ra) ar[ra] = E[(ty + 16 * ra) * kCoefLd + k];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) br[rb] = E[k * kCoefLd + tx + 16 * rb];
#pragma unroll
          for (int ra = 0; ra < RB; ++ra)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[ra][rb] += ar[ra] * br[rb];
        }
#pragma unroll
        for (int ra = 0; ra < RB; ++ra) {
          const int i = ty + 16 * ra;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const int j = tx + 16 * rb;
            if (i < M && j <= i) T[i * kCoefLd + j] = acc[ra][rb];
          }
        }
      }
      __syncthreads();
      double* x = E;
      E = T;
      T = x;
    }
    if (t < n) {
      const double v = E[(t + 1) * kCoefLd];
      dd[t] = v;
      a.cache->d[t] = v;
    }
    if (t == 0) {
      a.cache->hc = hc;
      a.cache->hg = hg;
      a.cache->n = n;
    }
  }
  __syncthreads();
  const double cc = bc[0], gg = bc[1], delta = bc[2], scal = bc[5];
  if (t < n) {
    const double d = dd[t];
    a.cf->dk[t] = d;
    a.cf->shift[t] = t > 0 ? cc / gg + a.xi[t - 1] : 0.0;
    a.cf->estf[t] = fabs(delta * d) / (a.rootN * scal);
  }
  if (t == 0) {
    a.cf->inv_g = 1.0 / gg;
    a.cf->thresh = a.thresh;
  }
}

}  // namespace

int leja_num_blocks(const Dims& d) {
  const dim3 g = cell_grid(d);
  return static_cast<int>(g.x * g.y * g.z);
}

hipError_t launch_leja_reset(LejaState* st, int nslots, int nterms, hipStream_t s) {
  hipLaunchKernelGGL(k_leja_reset, dim3(nslots < 64 ? nslots : 64), dim3(256), 0, s, st, nslots, nterms);
  return hipGetLastError();
}

template <class V>
hipError_t launch_leja_init(const Dims& d, const LejaCoef* cf, const double* v, V* q0, V* p, double* part,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_leja_init<V>, cell_grid(d), cell_block(), 0, s, d, cf, v, q0, p, part);
  return hipGetLastError();
}

template <class V>
hipError_t launch_leja_term(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout, V* p,
                            const LejaState* st, double* part, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int nb = leja_num_blocks(d);
  if (d.dim == 3)
    launch_timed(k_leja_term<3, V>, cell_grid(d), cell_block(), 0, s, e0, e1, d, cf, coef, qin, qout, p, st, part,
                 nb, k);
  else
    launch_timed(k_leja_term<2, V>, cell_grid(d), cell_block(), 0, s, e0, e1, d, cf, coef, qin, qout, p, st, part,
                 nb, k);
  return hipGetLastError();
}

template <class V>
hipError_t launch_leja_terms(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout, V* p,
                             const LejaState* st, double* part, int k, int nterms, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  if (d.dim != 2) return hipErrorInvalidValue;
  const dim3 g((d.nx + kBX - 1) / kBX, (d.ny + kLejaTileRows - 1) / kLejaTileRows, 1);
  const dim3 blk(kBX, kLejaThreadRows, 1);
  if (nterms == 4)
    launch_timed(k_leja_terms<4, kLejaTileRows, kLejaThreadRows, V>, g, blk, 0, s, e0, e1, d, cf, coef, qin, qout, p,
                 st, part, leja_num_blocks(d), k);
  else if (nterms == 2)
    launch_timed(k_leja_terms<2, kLejaTileRows, kLejaThreadRows, V>, g, blk, 0, s, e0, e1, d, cf, coef, qin, qout, p,
                 st, part, leja_num_blocks(d), k);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_leja_check(const Dims& d, const LejaCoef* cf, LejaState* st, const double* part, int k1, int k2,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_leja_check, dim3(1), dim3(kCheckThreads), 0, s, cf, st, part, leja_num_blocks(d), k1, k2);
  return hipGetLastError();
}

template <class V>
hipError_t launch_substep_update(const Dims& d, double* u, const V* p, double delta, int first, hipStream_t s,
                                 const double* zt) {
  hipLaunchKernelGGL(k_substep_update<V>, cell_grid(d), cell_block(), 0, s, d, u, p, delta, first, zt);
  return hipGetLastError();
}

hipError_t launch_leja_coef(const LejaCoefArgs& a, hipStream_t s) {
  if (a.n < 1 || a.n > kCoefMaxN || a.s < 1 || a.s > a.smax) return hipErrorInvalidValue;
  if (a.n + 1 <= 16)  // 16-row blocks of the order n + 1 matrix
    hipLaunchKernelGGL(k_leja_coef<1>, dim3(1), dim3(kCoefThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_leja_coef<2>, dim3(1), dim3(kCoefThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* a, float* b, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cast_f32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

template hipError_t launch_leja_init<double>(const Dims&, const LejaCoef*, const double*, double*, double*,
                                             double*, hipStream_t);
template hipError_t launch_leja_init<float>(const Dims&, const LejaCoef*, const double*, float*, float*, double*,
                                            hipStream_t);
template hipError_t launch_leja_term<double>(const Dims&, const LejaCoef*, const double*, const double*, double*,
                                             double*, const LejaState*, double*, int, hipStream_t, hipEvent_t,
                                             hipEvent_t);
template hipError_t launch_leja_term<float>(const Dims&, const LejaCoef*, const float*, const float*, float*, float*,
                                            const LejaState*, double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_substep_update<double>(const Dims&, double*, const double*, double, int, hipStream_t,
                                                  const double*);
template hipError_t launch_substep_update<float>(const Dims&, double*, const float*, double, int, hipStream_t,
                                                 const double*);

template hipError_t launch_leja_terms<double>(const Dims&, const LejaCoef*, const double*, const double*, double*,
                                              double*, const LejaState*, double*, int, int, hipStream_t, hipEvent_t,
                                              hipEvent_t);
template hipError_t launch_leja_terms<float>(const Dims&, const LejaCoef*, const float*, const float*, float*, float*,
                                             const LejaState*, double*, int, int, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace erem
