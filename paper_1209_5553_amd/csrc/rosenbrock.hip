// Shifted solves (sigma I - J) x = b for the Rosenbrock-type steps (Eq. ROS,
// Eq. ROSMh) and the Newton iterations of theta-Euler (Eq. temscheme): the
// paper solves these systems with BiCGSTAB; here BiCGSTAB runs with Jacobi
// right preconditioning, M = diag(sigma - J_ii), three kernels per iteration,
// every inner product reduced into a ring of slotted partial sums that the
// next kernel folds with one wavefront (no host round trip per iteration).
//
// With y = M^{-1} p and z = M^{-1} s, one iteration `it` is
//   K1: p = r + beta (p_old - omega_old v_old),  v = A y,  (rhat, v)
//   K2: alpha = (rhat, r) / (rhat, v),  s = r - alpha v,  t = A z,  (t, s), (t, t)
//   K3: omega = (t, s) / (t, t),  x += alpha y + omega z,  r = s - omega t,
//       (rhat, r), (r, r)
// where A = sigma I - J; a kernel that needs a neighbour's p (or s) forms it
// from the neighbour's operands, so p and v alternate between two buffers.
#include <hip/hip_runtime.h>

#include "rosenbrock.h"

namespace erem {

namespace {

__device__ inline int rb_tid() { return threadIdx.x + threadIdx.y * kBX; }
__device__ inline int rb_bid() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

// Sum of NV values over the 256-thread block; valid in thread 0.
template <int NV>
__device__ inline void rb_block_sum(double (&v)[NV]) {
  __shared__ double sh[kThreads / 64][NV];
#pragma unroll
  for (int n = 0; n < NV; ++n)
    for (int off = 32; off > 0; off >>= 1) v[n] += __shfl_down(v[n], off, 64);
  const int t = rb_tid();
  if ((t & 63) == 0) {
#pragma unroll
    for (int n = 0; n < NV; ++n) sh[t >> 6][n] = v[n];
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int n = 0; n < NV; ++n) v[n] = sh[0][n] + sh[1][n] + sh[2][n] + sh[3][n];
  }
}

// First slot of iteration it's partials in a ring of four.
__device__ inline int slot_of(const BicgState* st, int it) { return (it & 3) * st->nb; }

// Neighbour k of cell (x, y, z) in the stencil's order (-x, +x, -y, +y, -z,
// +z); a missing neighbour maps to the cell itself (its coefficient is 0).
template <int NB>
struct Nbrs {
  int idx[NB];
  __device__ Nbrs(const Dims& d, int x, int y, int z, int i) {
    const int pl = d.nx * d.ny;
    idx[0] = x > 0 ? i - 1 : i;
    idx[1] = x + 1 < d.nx ? i + 1 : i;
    idx[2] = y > 0 ? i - d.nx : i;
    idx[3] = y + 1 < d.ny ? i + d.nx : i;
    if (NB == 6) {
      idx[NB == 6 ? 4 : 0] = z > 0 ? i - pl : i;
      idx[NB == 6 ? 5 : 0] = z + 1 < d.nz ? i + pl : i;
    }
  }
};

// Scalars of a new solve (every producer overwrites the partial slots of
// all bands, so they need no clearing).
__global__ void k_bicg_reset(BicgState* st, double tol2) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->it_done = 0;
    st->breakdown = 0;
    st->tol2 = tol2;
  }
}

__global__ __launch_bounds__(kThreads) void k_bicg_start(Dims d, const double* __restrict__ b,
                                               double* __restrict__ xv, double* __restrict__ r,
                                               double* __restrict__ rhat, BicgState* st) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s[1] = {0.0};
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const double bi = b[i];
    r[i] = bi;
    rhat[i] = bi;
    xv[i] = 0.0;
    s[0] = bi * bi;
  }
  rb_block_sum<1>(s);
  if (rb_tid() == 0) {
    const int b = rb_bid();  // the block's band
    st->bb_sl[b] = s[0];
    st->rho[slot_of(st, 0) + b] = s[0];
    st->rr[slot_of(st, 0) + b] = s[0];
  }
}

// K1 of iteration `it`: convergence test on (r_it, r_it), beta, p, v = A y.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_bicg_pv(Dims d, double sigma, const double* __restrict__ coef,
                                            const double* __restrict__ r, const double* __restrict__ pold,
                                            const double* __restrict__ vold, double* __restrict__ pnew,
                                            double* __restrict__ vnew, const double* __restrict__ rhat,
                                            BicgState* st, int it) {
  __shared__ double beta_sh, om_sh;
  __shared__ int stop_sh;
  const int t = rb_tid();
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int N = d.N;
  const int i = in ? x + d.nx * (y + d.ny * z) : 0;
  const Nbrs<NB> nb(d, x, y, z, i);
  // operands first, so that their loads overlap the scalar decision below
  // (the diagonal of J is needed only at the neighbours: the preconditioned
  // operator's own-cell term is p itself)
  double rc = 0.0, pc = 0.0, vc = 0.0, rh = 0.0;
  double rn[NB], pn[NB], vn[NB], cn0[NB], ck[NB];
  if (in) {
    rc = r[i]; pc = pold[i]; vc = vold[i]; rh = rhat[i];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = nb.idx[k];
      rn[k] = r[j]; pn[k] = pold[j]; vn[k] = vold[j]; cn0[k] = coef[j];
      ck[k] = coef[(k + 1) * N + i];
    }
  }
  if (t < 64) {  // the first wavefront decides
    int stop = *(volatile int*)&st->done;
    double beta = 0.0, om = 0.0;
    if (!stop) {
      const double rr = wave_part_sum(st->rr + slot_of(st, it), st->nb);
      const double bb = wave_part_sum(st->bb_sl, st->nb);
      bool bad = !isfinite(rr);
      if (!bad && rr <= st->tol2 * bb) {
        stop = 1;
        if (rb_bid() == 0 && t == 0) { st->it_done = it; st->done = 1; }
      } else if (!bad && it > 0) {
        const double rho = wave_part_sum(st->rho + slot_of(st, it), st->nb);
        const double rho_p = wave_part_sum(st->rho + slot_of(st, it - 1), st->nb);
        const double rv_p = wave_part_sum(st->rv + slot_of(st, it - 1), st->nb);
        const double ts_p = wave_part_sum(st->ts + slot_of(st, it - 1), st->nb);
        const double tt_p = wave_part_sum(st->tt + slot_of(st, it - 1), st->nb);
        const double alpha_p = rho_p / rv_p;
        om = tt_p > 0.0 ? ts_p / tt_p : 0.0;
        beta = (rho / rho_p) * (alpha_p / om);
        bad = rho == 0.0 || !isfinite(beta);
      }
      if (bad) {
        stop = 1;
        if (rb_bid() == 0 && t == 0) { st->breakdown = 1; st->it_done = it; st->done = 1; }
      }
    }
    if (t == 0) { stop_sh = stop; beta_sh = beta; om_sh = om; }

  }
  __syncthreads();
  if (stop_sh) return;
  const double beta = beta_sh, om = om_sh;
  double s[1] = {0.0};
  if (in) {
    const double p = it == 0 ? rc : rc + beta * (pc - om * vc);
    double v = p;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const double pk = it == 0 ? rn[k] : rn[k] + beta * (pn[k] - om * vn[k]);
      v -= ck[k] * (pk / (sigma - cn0[k]));
    }
    pnew[i] = p;
    vnew[i] = v;
    s[0] = rh * v;
  }
  rb_block_sum<1>(s);
  if (t == 0) st->rv[slot_of(st, it) + rb_bid()] = s[0];
}

// K2: alpha, s = r - alpha v, t = A z, (t, s), (t, t).
template <int NB>
__global__ __launch_bounds__(kThreads) void k_bicg_st(Dims d, double sigma, const double* __restrict__ coef,
                                            const double* __restrict__ r, const double* __restrict__ v,
                                            double* __restrict__ sv, double* __restrict__ tv, BicgState* st,
                                            int it) {
  __shared__ double alpha_sh;
  __shared__ int stop_sh;
  const int t = rb_tid();
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int N = d.N;
  const int i = in ? x + d.nx * (y + d.ny * z) : 0;
  const Nbrs<NB> nb(d, x, y, z, i);
  double rc = 0.0, vc = 0.0;
  double rn[NB], vn[NB], cn0[NB], ck[NB];
  if (in) {
    rc = r[i]; vc = v[i];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = nb.idx[k];
      rn[k] = r[j]; vn[k] = v[j]; cn0[k] = coef[j];
      ck[k] = coef[(k + 1) * N + i];
    }
  }
  if (t < 64) {
    int stop = *(volatile int*)&st->done;
    double alpha = 0.0;
    if (!stop) {
      alpha = wave_part_sum(st->rho + slot_of(st, it), st->nb) / wave_part_sum(st->rv + slot_of(st, it), st->nb);
      if (!isfinite(alpha)) {
        stop = 1;
        if (rb_bid() == 0 && t == 0) { st->breakdown = 1; st->it_done = it; st->done = 1; }
      }
    }
    if (t == 0) { stop_sh = stop; alpha_sh = alpha; }

  }
  __syncthreads();
  if (stop_sh) return;
  const double alpha = alpha_sh;
  double s[2] = {0.0, 0.0};
  if (in) {
    const double si = rc - alpha * vc;
    double ti = si;
#pragma unroll
    for (int k = 0; k < NB; ++k) ti -= ck[k] * ((rn[k] - alpha * vn[k]) / (sigma - cn0[k]));
    sv[i] = si;
    tv[i] = ti;
    s[0] = ti * si;
    s[1] = ti * ti;
  }
  rb_block_sum<2>(s);
  if (t == 0) {
    const int b = rb_bid();
    st->ts[slot_of(st, it) + b] = s[0];
    st->tt[slot_of(st, it) + b] = s[1];
  }
}

// K3: omega, x += alpha y + omega z, r = s - omega t, (rhat, r), (r, r).
__global__ __launch_bounds__(kThreads) void k_bicg_xr(Dims d, double sigma, const double* __restrict__ coef,
                                            double* __restrict__ xv, double* __restrict__ r,
                                            const double* __restrict__ p, const double* __restrict__ sv,
                                            const double* __restrict__ tv, const double* __restrict__ rhat,
                                            BicgState* st, int it) {
  __shared__ double alpha_sh, om_sh;
  __shared__ int stop_sh;
  const int t = rb_tid();
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int i = in ? x + d.nx * (y + d.ny * z) : 0;
  double xc = 0.0, pc = 0.0, sc = 0.0, tc = 0.0, c0 = 0.0, rh = 0.0;
  if (in) {
    xc = xv[i]; pc = p[i]; sc = sv[i]; tc = tv[i]; c0 = coef[i]; rh = rhat[i];
  }
  if (t < 64) {
    const int stop = *(volatile int*)&st->done;
    double alpha = 0.0, om = 0.0;
    if (!stop) {
      alpha = wave_part_sum(st->rho + slot_of(st, it), st->nb) / wave_part_sum(st->rv + slot_of(st, it), st->nb);
      const double tt = wave_part_sum(st->tt + slot_of(st, it), st->nb);
      om = tt > 0.0 ? wave_part_sum(st->ts + slot_of(st, it), st->nb) / tt : 0.0;

    }
    if (t == 0) { stop_sh = stop; alpha_sh = alpha; om_sh = om; }
  }
  __syncthreads();
  if (stop_sh) return;
  const double alpha = alpha_sh, om = om_sh;
  double s[2] = {0.0, 0.0};
  if (in) {
    xv[i] = xc + (alpha * pc + om * sc) / (sigma - c0);
    const double rn = sc - om * tc;
    r[i] = rn;
    s[0] = rh * rn;
    s[1] = rn * rn;
  }
  rb_block_sum<2>(s);
  if (t == 0) {
    const int b = rb_bid();
    st->rho[slot_of(st, it + 1) + b] = s[0];
    st->rr[slot_of(st, it + 1) + b] = s[1];
  }
}

__global__ __launch_bounds__(kThreads) void k_lincomb(Dims d, double* out, LinComb lc) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < 4; ++m)
    if (m < lc.n) a[m] = lc.in[m][i];
  double s = lc.w[0] * a[0];
#pragma unroll
  for (int m = 1; m < 4; ++m)
    if (m < lc.n) s += lc.w[m] * a[m];
  out[i] = s;
}

}  // namespace

hipError_t launch_bicg_reset(BicgState* st, double tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_reset, dim3(1), dim3(256), 0, s, st, tol2);
  return hipGetLastError();
}

hipError_t launch_bicg_start(const Dims& d, const double* b, double* x, const BicgBufs& B, BicgState* st,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_start, cell_grid(d), cell_block(), 0, s, d, b, x, B.r, B.rhat, st);
  return hipGetLastError();
}

hipError_t launch_bicg_iteration(const Dims& d, double sigma, const double* coef, double* x,
                                 const BicgBufs& B, BicgState* st, int it, hipStream_t s, const hipEvent_t* e) {
  const double* pold = B.p[(it + 1) & 1];
  const double* vold = B.v[(it + 1) & 1];
  double* pnew = B.p[it & 1];
  double* vnew = B.v[it & 1];
  const hipEvent_t n = nullptr;
  if (d.dim == 3) {
    launch_timed(k_bicg_pv<6>, cell_grid(d), cell_block(), 0, s, e ? e[0] : n, e ? e[1] : n, d, sigma, coef, B.r,
                 pold, vold, pnew, vnew, B.rhat, st, it);
    launch_timed(k_bicg_st<6>, cell_grid(d), cell_block(), 0, s, e ? e[2] : n, e ? e[3] : n, d, sigma, coef, B.r,
                 static_cast<const double*>(vnew), B.s, B.t, st, it);
  } else {
    launch_timed(k_bicg_pv<4>, cell_grid(d), cell_block(), 0, s, e ? e[0] : n, e ? e[1] : n, d, sigma, coef, B.r,
                 pold, vold, pnew, vnew, B.rhat, st, it);
    launch_timed(k_bicg_st<4>, cell_grid(d), cell_block(), 0, s, e ? e[2] : n, e ? e[3] : n, d, sigma, coef, B.r,
                 static_cast<const double*>(vnew), B.s, B.t, st, it);
  }
  launch_timed(k_bicg_xr, cell_grid(d), cell_block(), 0, s, e ? e[4] : n, e ? e[5] : n, d, sigma, coef, x, B.r,
               static_cast<const double*>(pnew), static_cast<const double*>(B.s),
               static_cast<const double*>(B.t), static_cast<const double*>(B.rhat), st, it);
  return hipGetLastError();
}

hipError_t launch_lincomb(const Dims& d, double* out, const LinComb& lc, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, cell_grid(d), cell_block(), 0, s, d, out, lc);
  return hipGetLastError();
}

}  // namespace erem
