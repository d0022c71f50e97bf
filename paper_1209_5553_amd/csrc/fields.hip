// HIP kernels of the EREM path for gfx950 (MI355X): TPFA transmissibilities,
// face fluxes, Jacobian / G assembly, Gershgorin interval and the pressure
// conjugate gradients.
//
// Every cell kernel runs one thread per cell on a (64 x 4) block: one
// 64-lane wavefront per grid row segment, so loads along x are fully
// coalesced; +-y / +-z neighbours come from the same block's other rows or
// from L2.  Reductions: wavefront shuffles, then the four wavefront partials
// through LDS; the conjugate-gradient inner products then go to the block's
// own partial slot, which consumers add up in a fixed order (PcgState), and
// the assembly's min / max targets take an atomic min / max over kSlots
// slots (order-free); the consumer of a sum is always a later kernel, so
// kernel boundaries order every producer/consumer pair.
#include "device.h"

#include <cmath>

namespace erem {

namespace {

__device__ inline int tid_lin() { return threadIdx.x + threadIdx.y * kBX; }
__device__ inline int bid_lin() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// Sum of NV values over the 256-thread block; the result is valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV]) {
  __shared__ double sh[kThreads / 64][NV];
#pragma unroll
  for (int n = 0; n < NV; ++n)
    for (int off = 32; off > 0; off >>= 1) v[n] += __shfl_down(v[n], off, 64);
  const int t = tid_lin();
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

__device__ inline double rho_of(double T, const Phys& ph) {
  return ph.law == 1 ? 1000.0 * (1.0 - 3.0e-4 * (T - 20.0)) : ph.rho0;
}
__device__ inline double drho_of(const Phys& ph) { return ph.law == 1 ? -0.3 : 0.0; }
__device__ inline double mu_of(double T, const Phys& ph) {
  return ph.law == 1 ? 2.414e-5 * pow(10.0, 247.8 / (T + 133.0)) : ph.mu0;
}

// Mass mobility rho(T) K / mu(T) of one cell.
__device__ inline double mobility(const Phys& ph, const double* logk, const double* T, int i) {
  const double Ti = T ? T[i] : 20.0;
  return rho_of(Ti, ph) * exp(logk[i]) / mu_of(Ti, ph);
}

// Flat indices of the face arrays (boundary faces included).
__device__ inline int fx_idx(const Dims& d, int x, int y, int z) { return (z * d.ny + y) * (d.nx + 1) + x; }
__device__ inline int fy_idx(const Dims& d, int x, int y, int z) { return (z * (d.ny + 1) + y) * d.nx + x; }
__device__ inline int fz_idx(const Dims& d, int x, int y, int z) { return (z * d.ny + y) * d.nx + x; }

// ---------------------------------------------------------------------------
// TPFA transmissibilities (Sec. 3.1): harmonic mean on interior faces,
// Dirichlet half-cell on x faces, zero on the closed y / z boundary faces.
// Each cell writes its +x, +y, +z faces, and the cells of the first layer
// also write the -x / -y / -z boundary faces.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_transmissibility(Dims d, Phys ph, const double* __restrict__ logk,
                                                     const double* __restrict__ T, double* __restrict__ tx,
                                                     double* __restrict__ ty, double* __restrict__ tz) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const double ax = d.dy * d.dz, ay = d.dx * d.dz, az = d.dx * d.dy;
  const double hx = 0.5 * d.dx, hy = 0.5 * d.dy, hz = 0.5 * d.dz;
  const double ki = mobility(ph, logk, T, i);
  if (x + 1 < d.nx) {
    const double kj = mobility(ph, logk, T, i + 1);
    tx[fx_idx(d, x + 1, y, z)] = ax * ki * kj / (ki * hx + kj * hx);
  } else {
    tx[fx_idx(d, x + 1, y, z)] = ax * ki / hx;
  }
  if (x == 0) tx[fx_idx(d, 0, y, z)] = ax * ki / hx;
  if (y + 1 < d.ny) {
    const double kj = mobility(ph, logk, T, i + d.nx);
    ty[fy_idx(d, x, y + 1, z)] = ay * ki * kj / (ki * hy + kj * hy);
  } else {
    ty[fy_idx(d, x, y + 1, z)] = 0.0;
  }
  if (y == 0) ty[fy_idx(d, x, 0, z)] = 0.0;
  if (z + 1 < d.nz) {
    const double kj = mobility(ph, logk, T, i + d.nx * d.ny);
    tz[fz_idx(d, x, y, z + 1)] = az * ki * kj / (ki * hz + kj * hz);
  } else {
    tz[fz_idx(d, x, y, z + 1)] = 0.0;
  }
  if (z == 0) tz[fz_idx(d, x, y, 0)] = 0.0;
}

// Face mass fluxes F = tau (p_i - p_j) (Darcy, TPFA), +axis orientation.
__global__ __launch_bounds__(kThreads) void k_face_fluxes(Dims d, Phys ph, const double* __restrict__ p,
                                                const double* __restrict__ tx, const double* __restrict__ ty,
                                                const double* __restrict__ tz, double* __restrict__ fx,
                                                double* __restrict__ fy, double* __restrict__ fz) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const double pi = p[i];
  {
    const int f = fx_idx(d, x + 1, y, z);
    fx[f] = (x + 1 < d.nx) ? tx[f] * (pi - p[i + 1]) : tx[f] * (pi - ph.p_right);
  }
  if (x == 0) {
    const int f = fx_idx(d, 0, y, z);
    fx[f] = tx[f] * (ph.p_left - pi);
  }
  {
    const int f = fy_idx(d, x, y + 1, z);
    fy[f] = (y + 1 < d.ny) ? ty[f] * (pi - p[i + d.nx]) : 0.0;
  }
  if (y == 0) fy[fy_idx(d, x, 0, z)] = 0.0;
  {
    const int f = fz_idx(d, x, y, z + 1);
    fz[f] = (z + 1 < d.nz) ? tz[f] * (pi - p[i + d.nx * d.ny]) : 0.0;
  }
  if (z == 0) fz[fz_idx(d, x, y, 0)] = 0.0;
}

__global__ void k_reset_reduce(AsmReduce* r) {
  for (int k = threadIdx.x; k < kSlots; k += blockDim.x) {
    r->lo[k] = ord_encode(INFINITY);
    r->hi[k] = ord_encode(-INFINITY);
    r->tmax[k] = ord_encode(0.0);
    r->vmax[k] = ord_encode(0.0);
  }
}

// slot of this block's atomics in AsmReduce
__device__ inline int red_slot() {
  return (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) & (kSlots - 1);
}

// ---------------------------------------------------------------------------
// Jacobian stencil and G(T) (Sec. 3.1 fluxes, Eq. linear), fused with the
// Gershgorin interval of the rows (Sec. 4.2) and max |T|.
//   R_i = sum_faces [conduction tau (T_nb - T_i)] - [advection c_f F_out T_up] + b_i
//   G_i = R_i / (V C_i),  J_ij = A_ij / (V C_i),
//   J_ii = A_ii / (V C_i) - R_i C'_i / (V C_i^2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_assemble(Dims d, Phys ph, const double* __restrict__ poro,
                                             const double* __restrict__ fx, const double* __restrict__ fy,
                                             const double* __restrict__ fz, const double* __restrict__ T,
                                             double* __restrict__ coef, double* __restrict__ F,
                                             AsmReduce* red) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double lo = INFINITY, hi = -INFINITY, tmax = 0.0;
  if (x < d.nx && y < d.ny) {
    const int N = d.N;
    const int i = x + d.nx * (y + d.ny * z);
    const double ax = d.dy * d.dz, ay = d.dx * d.dz, az = d.dx * d.dy;
    const double tcx = ph.lam * ax / d.dx, tcy = ph.lam * ay / d.dy, tcz = ph.lam * az / d.dz;
    const double tcb = ph.lam * ax / (0.5 * d.dx);
    const double cf = ph.c_f;
    const double Ti = T[i];
    // every load first (the cell itself where a neighbour is missing; the
    // face arrays hold the boundary faces), the arithmetic after
    const int pl = d.nx * d.ny;
    const bool hw = x > 0, he = x + 1 < d.nx, hs = y > 0, hn = y + 1 < d.ny;
    const bool hb = d.dim == 3 && z > 0, ht = d.dim == 3 && z + 1 < d.nz;
    const double Tw = T[hw ? i - 1 : i], Te = T[he ? i + 1 : i];
    const double Ts = T[hs ? i - d.nx : i], Tn = T[hn ? i + d.nx : i];
    const double Tb = T[hb ? i - pl : i], Tt = T[ht ? i + pl : i];
    const double fw = fx[fx_idx(d, x, y, z)], fe = fx[fx_idx(d, x + 1, y, z)];
    const double fs = fy[fy_idx(d, x, y, z)], fn = fy[fy_idx(d, x, y + 1, z)];
    const double fb = d.dim == 3 ? fz[fz_idx(d, x, y, z)] : 0.0;
    const double ft = d.dim == 3 ? fz[fz_idx(d, x, y, z + 1)] : 0.0;
    const double phi = poro[i];
    double diag = 0.0, b = 0.0, R = 0.0;
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    // -x face (flux > 0 enters the cell)
    if (hw) {
      a[1] = tcx + cf * fmax(fw, 0.0);
      diag -= tcx + cf * fmax(-fw, 0.0);
      R += a[1] * Tw;
    } else {
      if (ph.dirichlet_left) {
        diag -= tcb;
        b += tcb * ph.T_left;
      }
      if (fw > 0.0) b += cf * fw * ph.T_left; else diag -= cf * (-fw);
    }
    // +x face (flux > 0 leaves the cell)
    if (he) {
      a[2] = tcx + cf * fmax(-fe, 0.0);
      diag -= tcx + cf * fmax(fe, 0.0);
      R += a[2] * Te;
    } else {
      if (fe >= 0.0) diag -= cf * fe; else b += cf * (-fe) * ph.T_right;
    }
    // -y / +y faces (closed boundaries carry nothing)
    if (hs) {
      a[3] = tcy + cf * fmax(fs, 0.0);
      diag -= tcy + cf * fmax(-fs, 0.0);
      R += a[3] * Ts;
    }
    if (hn) {
      a[4] = tcy + cf * fmax(-fn, 0.0);
      diag -= tcy + cf * fmax(fn, 0.0);
      R += a[4] * Tn;
    }
    if (hb) {
      a[5] = tcz + cf * fmax(fb, 0.0);
      diag -= tcz + cf * fmax(-fb, 0.0);
      R += a[5] * Tb;
    }
    if (ht) {
      a[6] = tcz + cf * fmax(-ft, 0.0);
      diag -= tcz + cf * fmax(ft, 0.0);
      R += a[6] * Tt;
    }
    R += diag * Ti + b;
    const double V = d.dx * d.dy * d.dz;
    const double C = phi * rho_of(Ti, ph) * cf + (1.0 - phi) * ph.rhoc_s;
    const double dC = phi * drho_of(ph) * cf;
    const double inv = 1.0 / (V * C);
    const double jc = diag * inv - R * dC * inv / C;
    coef[i] = jc;
    double rad = 0.0;
    const int ndir = d.dim == 3 ? 7 : 5;
    for (int k = 1; k < ndir; ++k) {
      const double c = a[k] * inv;
      coef[k * N + i] = c;
      rad += fabs(c);
    }
    F[i] = R * inv;
    lo = jc - rad;
    hi = jc + rad;
    tmax = fabs(Ti);
  }
  // block min / max through wavefront shuffles and LDS
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
    tmax = fmax(tmax, __shfl_down(tmax, off, 64));
  }
  __shared__ double sh[3][kThreads / 64];
  const int t = tid_lin();
  if ((t & 63) == 0) {
    sh[0][t >> 6] = lo;
    sh[1][t >> 6] = hi;
    sh[2][t >> 6] = tmax;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      sh[0][0] = fmin(sh[0][0], sh[0][w]);
      sh[1][0] = fmax(sh[1][0], sh[1][w]);
      sh[2][0] = fmax(sh[2][0], sh[2][w]);
    }
    const int k = red_slot();
    atomicMin(&red->lo[k], ord_encode(sh[0][0]));
    atomicMax(&red->hi[k], ord_encode(sh[1][0]));
    atomicMax(&red->tmax[k], ord_encode(sh[2][0]));
  }
}

// Gershgorin interval of a given stencil (rows): [min (J_ii - R_i), max (J_ii + R_i)].
__global__ __launch_bounds__(kThreads) void k_gershgorin(Dims d, const double* __restrict__ coef, AsmReduce* red) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double lo = INFINITY, hi = -INFINITY;
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const int ndir = d.dim == 3 ? 7 : 5;
    double rad = 0.0;
    for (int k = 1; k < ndir; ++k) rad += fabs(coef[k * d.N + i]);
    lo = coef[i] - rad;
    hi = coef[i] + rad;
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  __shared__ double sh[2][kThreads / 64];
  const int t = tid_lin();
  if ((t & 63) == 0) {
    sh[0][t >> 6] = lo;
    sh[1][t >> 6] = hi;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      sh[0][0] = fmin(sh[0][0], sh[0][w]);
      sh[1][0] = fmax(sh[1][0], sh[1][w]);
    }
    const int k = red_slot();
    atomicMin(&red->lo[k], ord_encode(sh[0][0]));
    atomicMax(&red->hi[k], ord_encode(sh[1][0]));
  }
}

__global__ void k_reset_vmax(AsmReduce* r) {
  for (int k = threadIdx.x; k < kSlots; k += blockDim.x) r->vmax[k] = ord_encode(0.0);
}

__global__ __launch_bounds__(kThreads) void k_absmax(Dims d, const double* __restrict__ v, AsmReduce* red) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double m = 0.0;
  if (x < d.nx && y < d.ny) m = fabs(v[x + d.nx * (y + d.ny * z)]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __shared__ double sh[kThreads / 64];
  const int t = tid_lin();
  if ((t & 63) == 0) sh[t >> 6] = m;
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kThreads / 64; ++w) sh[0] = fmax(sh[0], sh[w]);
    atomicMax(&red->vmax[red_slot()], ord_encode(sh[0]));
  }
}

// J u at cell (x, y, z) from the SoA stencil.
__device__ inline double stencil_apply(const Dims& d, const double* __restrict__ coef,
                                       const double* __restrict__ u, int x, int y, int z, int i) {
  const int N = d.N;
  double s = coef[i] * u[i];
  s += coef[N + i] * u[x > 0 ? i - 1 : i];
  s += coef[2 * N + i] * u[x + 1 < d.nx ? i + 1 : i];
  s += coef[3 * N + i] * u[y > 0 ? i - d.nx : i];
  s += coef[4 * N + i] * u[y + 1 < d.ny ? i + d.nx : i];
  if (d.dim == 3) {
    const int pl = d.nx * d.ny;
    s += coef[5 * N + i] * u[z > 0 ? i - pl : i];
    s += coef[6 * N + i] * u[z + 1 < d.nz ? i + pl : i];
  }
  return s;
}

// w = v + tg g + J u  (g may be null: w = v + J u)
__global__ __launch_bounds__(kThreads) void k_stencil_axpy(Dims d, const double* __restrict__ coef,
                                                 const double* __restrict__ v, const double* __restrict__ u,
                                                 double* __restrict__ w, const double* __restrict__ g,
                                                 double tg) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  double a = v[i];
  if (g) a += tg * g[i];
  w[i] = a + stencil_apply(d, coef, u, x, y, z, i);
}

// ---------------------------------------------------------------------------
// D_t G for boundary temperatures moving at the rates dTl (x = 0) and dTr
// (x = nx): b enters R linearly and is itself linear in T_left and T_right,
// so D_t b is the boundary part of the assembly with the rates in place of
// the temperatures, and D_t G = D_t b / (V C(T)) (the non-autonomous step,
// Sec. 3.2.3, Eq. nEERMg).  Zero away from the two x boundaries.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_time_rate(Dims d, Phys ph, const double* __restrict__ poro,
                                              const double* __restrict__ fx, const double* __restrict__ T,
                                              double dTl, double dTr, double* __restrict__ Gt) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const double cf = ph.c_f;
  double bt = 0.0;
  if (x == 0) {
    const double fw = fx[fx_idx(d, 0, y, z)];
    if (ph.dirichlet_left) bt += ph.lam * (d.dy * d.dz) / (0.5 * d.dx) * dTl;
    if (fw > 0.0) bt += cf * fw * dTl;
  }
  if (x + 1 == d.nx) {
    const double fe = fx[fx_idx(d, x + 1, y, z)];
    if (fe < 0.0) bt += cf * (-fe) * dTr;
  }
  const double phi = poro[i];
  const double V = d.dx * d.dy * d.dz;
  const double C = phi * rho_of(T[i], ph) * cf + (1.0 - phi) * ph.rhoc_s;
  Gt[i] = bt * (1.0 / (V * C));
}

// y <- a*y + b*x
__global__ __launch_bounds__(kThreads) void k_axpby(Dims d, double* __restrict__ yv, double a,
                                          const double* __restrict__ xv, double b) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  yv[i] = (a == 0.0) ? b * xv[i] : a * yv[i] + b * xv[i];
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned conjugate gradients for the steady TPFA pressure.
//   (A p)_i = sum_faces t_f (p_i - p_nb), Dirichlet x faces add t_f p_i only,
//   b_i = t_left p_left [x = 0] + t_right p_right [x = nx-1].
// One iteration = two kernels; all scalars (alpha, beta, norms) stay on the
// device in a ring of four iterations.
// ---------------------------------------------------------------------------
struct FaceT {
  double w, e, s, n, b, t;  // transmissibility of the six faces
};

__device__ inline FaceT load_faces(const Dims& d, const double* tx, const double* ty, const double* tz,
                                   int x, int y, int z) {
  FaceT f;
  f.w = tx[fx_idx(d, x, y, z)];
  f.e = tx[fx_idx(d, x + 1, y, z)];
  f.s = ty[fy_idx(d, x, y, z)];
  f.n = ty[fy_idx(d, x, y + 1, z)];
  if (d.dim == 3) {
    f.b = tz[fz_idx(d, x, y, z)];
    f.t = tz[fz_idx(d, x, y, z + 1)];
  } else {
    f.b = 0.0;
    f.t = 0.0;
  }
  return f;
}

// Scalars of a new solve; the partial slots need no clearing, every
// producer overwrites the slots of all bands.
__global__ void k_pcg_reset(PcgState* st, double tol2) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->it_done = -1;
    st->nonfinite = 0;
    st->bb = 0.0;
    st->tol2 = tol2;
    for (int k = 0; k < 4; ++k) st->alpha[k] = 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_start(Dims d, Phys ph, const double* __restrict__ tx,
                                              const double* __restrict__ ty, const double* __restrict__ tz,
                                              const double* __restrict__ xv, double* __restrict__ r,
                                              double* __restrict__ zv, double* __restrict__ p0,
                                              double* __restrict__ diag, PcgState* st) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s[3] = {0.0, 0.0, 0.0};
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const FaceT f = load_faces(d, tx, ty, tz, x, y, z);
    const double dg = f.w + f.e + f.s + f.n + f.b + f.t;
    const int pl = d.nx * d.ny;
    double Ax = dg * xv[i];
    if (x > 0) Ax -= f.w * xv[i - 1];
    if (x + 1 < d.nx) Ax -= f.e * xv[i + 1];
    if (y > 0) Ax -= f.s * xv[i - d.nx];
    if (y + 1 < d.ny) Ax -= f.n * xv[i + d.nx];
    if (z > 0) Ax -= f.b * xv[i - pl];
    if (z + 1 < d.nz) Ax -= f.t * xv[i + pl];
    double bi = 0.0;
    if (x == 0) bi += f.w * ph.p_left;
    if (x + 1 == d.nx) bi += f.e * ph.p_right;
    const double ri = bi - Ax;
    const double zi = ri / dg;
    r[i] = ri;
    zv[i] = zi;
    p0[i] = 0.0;
    diag[i] = dg;
    s[0] = ri * zi;
    s[1] = ri * ri;
    s[2] = bi * bi;
  }
  block_sum<3>(s);
  if (tid_lin() == 0) {
    const int b = bid_lin();  // the block's band
    st->rz[b] = s[0];
    st->rr[b] = s[1];
    st->bb_sl[b] = s[2];
  }
}

// Start of a correction solve A x = rhs from x = 0.
__global__ __launch_bounds__(kThreads) void k_pcg_start_rhs(Dims d, const double* __restrict__ tx,
                                                  const double* __restrict__ ty, const double* __restrict__ tz,
                                                  const double* __restrict__ rhs, double* __restrict__ xv,
                                                  double* __restrict__ r, double* __restrict__ zv,
                                                  double* __restrict__ p0, double* __restrict__ diag, PcgState* st,
                                                  int jacobi) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s[2] = {0.0, 0.0};
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const FaceT f = load_faces(d, tx, ty, tz, x, y, z);
    const double dg = f.w + f.e + f.s + f.n + f.b + f.t;
    const double ri = rhs[i];
    const double zi = ri / dg;
    xv[i] = 0.0;
    r[i] = ri;
    if (jacobi) zv[i] = zi;
    p0[i] = 0.0;
    diag[i] = dg;
    s[0] = ri * zi;
    s[1] = ri * ri;
  }
  block_sum<2>(s);
  if (tid_lin() == 0) {
    const int b = bid_lin();
    if (jacobi) st->rz[b] = s[0];  // otherwise the preconditioner writes r.z
    st->rr[b] = s[1];
    st->bb_sl[b] = s[1];
  }
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (error-free sum and fma product) for residuals
// and pressure differences: the pressure is held as p_hi + p_lo.
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};
__device__ inline DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline DD quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ inline DD dd_sub(DD a, DD b) { return dd_add(a, DD{-b.hi, -b.lo}); }
__device__ inline DD dd_mul(DD a, double t) {
  const double p = a.hi * t;
  double e = fma(a.hi, t, -p);
  e += a.lo * t;
  return quick_two_sum(p, e);
}

// r = b - A p in double-double, rounded; sums r^2 and b^2.
__global__ __launch_bounds__(kThreads) void k_dd_residual(Dims d, Phys ph, const double* __restrict__ tx,
                                                const double* __restrict__ ty, const double* __restrict__ tz,
                                                const double* __restrict__ phi, const double* __restrict__ plo,
                                                double* __restrict__ r, PcgState* st) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s[2] = {0.0, 0.0};
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const int pl = d.nx * d.ny;
    const FaceT f = load_faces(d, tx, ty, tz, x, y, z);
    // neighbour pressures first (the cell itself where a neighbour is
    // missing), so that every load issues before the arithmetic
    const bool hw = x > 0, he = x + 1 < d.nx, hs = y > 0, hn = y + 1 < d.ny, hb = z > 0, ht = z + 1 < d.nz;
    const int iw = hw ? i - 1 : i, ie = he ? i + 1 : i, is = hs ? i - d.nx : i, in = hn ? i + d.nx : i;
    const int ib = hb ? i - pl : i, it = ht ? i + pl : i;
    const DD pi{phi[i], plo[i]};
    const DD pw{phi[iw], plo[iw]}, pe{phi[ie], plo[ie]}, ps{phi[is], plo[is]}, pn{phi[in], plo[in]};
    const DD pb{phi[ib], plo[ib]}, pt{phi[it], plo[it]};
    DD acc{0.0, 0.0};  // sum t (p_i - p_nb)
    double bi = 0.0;
    acc = dd_add(acc, dd_mul(dd_sub(pi, hw ? pw : DD{ph.p_left, 0.0}), f.w));
    if (!hw) bi += f.w * ph.p_left;
    acc = dd_add(acc, dd_mul(dd_sub(pi, he ? pe : DD{ph.p_right, 0.0}), f.e));
    if (!he) bi += f.e * ph.p_right;
    if (hs) acc = dd_add(acc, dd_mul(dd_sub(pi, ps), f.s));
    if (hn) acc = dd_add(acc, dd_mul(dd_sub(pi, pn), f.n));
    if (hb) acc = dd_add(acc, dd_mul(dd_sub(pi, pb), f.b));
    if (ht) acc = dd_add(acc, dd_mul(dd_sub(pi, pt), f.t));
    // residual of sum t (p_i - p_nb) = 0 with Dirichlet neighbours folded in
    const double ri = -(acc.hi + acc.lo);
    r[i] = ri;
    s[0] = ri * ri;
    s[1] = bi * bi;
  }
  block_sum<2>(s);
  if (tid_lin() == 0) {
    const int b = bid_lin();
    st->rr[b] = s[0];
    st->bb_sl[b] = s[1];
  }
}

// Warm start of the next pressure solve from the last two solutions: the
// previous one (prev) and the current double-double one (hi + lo).  With
// extrapolate, hi = 2 p - prev and lo = 0; prev takes the current p.
__global__ __launch_bounds__(kThreads) void k_pressure_extrapolate(Dims d, double* __restrict__ phi,
                                                         double* __restrict__ plo, double* __restrict__ prev,
                                                         int extrapolate) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const double cur = phi[i] + plo[i];
  if (extrapolate) {
    phi[i] = 2.0 * cur - prev[i];
    plo[i] = 0.0;
  }
  prev[i] = cur;
}

// p_hi + p_lo += delta (double-double)
__global__ __launch_bounds__(kThreads) void k_dd_update(Dims d, double* __restrict__ phi, double* __restrict__ plo,
                                              const double* __restrict__ delta) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const DD s = dd_add(DD{phi[i], plo[i]}, DD{delta[i], 0.0});
  phi[i] = s.hi;
  plo[i] = s.lo;
}

// Face mass fluxes from the double-double pressure: F = t (p_i - p_j)
// with the difference formed before rounding.
__global__ __launch_bounds__(kThreads) void k_face_fluxes_dd(Dims d, Phys ph, const double* __restrict__ phi,
                                                   const double* __restrict__ plo, const double* __restrict__ tx,
                                                   const double* __restrict__ ty, const double* __restrict__ tz,
                                                   double* __restrict__ fx, double* __restrict__ fy,
                                                   double* __restrict__ fz) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const DD pi{phi[i], plo[i]};
  auto diff = [&](DD a, DD b) {
    const DD s = dd_sub(a, b);
    return s.hi + s.lo;
  };
  {
    const int f = fx_idx(d, x + 1, y, z);
    fx[f] = (x + 1 < d.nx) ? tx[f] * diff(pi, DD{phi[i + 1], plo[i + 1]}) : tx[f] * diff(pi, DD{ph.p_right, 0.0});
  }
  if (x == 0) {
    const int f = fx_idx(d, 0, y, z);
    fx[f] = tx[f] * diff(DD{ph.p_left, 0.0}, pi);
  }
  {
    const int f = fy_idx(d, x, y + 1, z);
    fy[f] = (y + 1 < d.ny) ? ty[f] * diff(pi, DD{phi[i + d.nx], plo[i + d.nx]}) : 0.0;
  }
  if (y == 0) fy[fy_idx(d, x, 0, z)] = 0.0;
  {
    const int f = fz_idx(d, x, y, z + 1);
    fz[f] = (z + 1 < d.nz) ? tz[f] * diff(pi, DD{phi[i + d.nx * d.ny], plo[i + d.nx * d.ny]}) : 0.0;
  }
  if (z == 0) fz[fz_idx(d, x, y, 0)] = 0.0;
}

// Iteration `it`, first half: convergence test on rr[it], beta, p_new =
// z + beta p_old (own and neighbour values), q = A p_new, pq[it].
__global__ __launch_bounds__(kThreads) void k_pcg_a(Dims d, const double* __restrict__ tx,
                                          const double* __restrict__ ty, const double* __restrict__ tz,
                                          const double* __restrict__ zv, const double* __restrict__ pold,
                                          double* __restrict__ pnew, double* __restrict__ q,
                                          PcgState* st, int it) {
  __shared__ double beta_sh;
  __shared__ int stop_sh;
  const int t = tid_lin();
  // operands first, so that their loads overlap the scalar decision below
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int i = x + d.nx * (y + d.ny * z);
  const int pl = d.nx * d.ny;
  FaceT f{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double zc = 0.0, pc = 0.0;
  double zn[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, pn[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool has[6] = {x > 0, x + 1 < d.nx, y > 0, y + 1 < d.ny, z > 0, z + 1 < d.nz};
  const int nbi[6] = {i - 1, i + 1, i - d.nx, i + d.nx, i - pl, i + pl};
  if (in) {
    f = load_faces(d, tx, ty, tz, x, y, z);
    zc = zv[i];
    pc = pold[i];
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (has[k]) {
        zn[k] = zv[nbi[k]];
        pn[k] = pold[nbi[k]];
      }
  }
  if (t < 64) {  // the first wavefront decides
    int stop = *(volatile int*)&st->done;
    double beta = 0.0;
    if (!stop) {
      const int nb = st->nb;
      const double rr = wave_part_sum(st->rr + (it & 3) * nb, nb);
      const double bb = wave_part_sum(st->bb_sl, nb);
      const double rz1 = wave_part_sum(st->rz + (it & 3) * nb, nb);
      const double rz0 = it > 0 ? wave_part_sum(st->rz + ((it - 1) & 3) * nb, nb) : 1.0;
      if (!isfinite(rr)) {
        stop = 1;
        if (bid_lin() == 0 && t == 0) { st->nonfinite = 1; st->done = 1; st->it_done = it; }
      } else if (rr <= st->tol2 * bb) {
        stop = 1;
        if (bid_lin() == 0 && t == 0) { st->done = 1; st->it_done = it; st->bb = bb; }
      } else if (it > 0) {
        beta = rz1 / rz0;
      }
    }
    if (t == 0) {
      stop_sh = stop;
      beta_sh = beta;
    }
  }
  __syncthreads();
  if (stop_sh) return;
  const double beta = beta_sh;
  double s[1] = {0.0};
  if (in) {
    const double fk[6] = {f.w, f.e, f.s, f.n, f.b, f.t};
    const double dg = f.w + f.e + f.s + f.n + f.b + f.t;
    const double pi = zc + beta * pc;
    double Ap = dg * pi;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (has[k]) Ap -= fk[k] * (zn[k] + beta * pn[k]);
    pnew[i] = pi;
    q[i] = Ap;
    s[0] = pi * Ap;
  }
  block_sum<1>(s);
  if (t == 0) st->pq[(it & 3) * st->nb + bid_lin()] = s[0];
}

// Iteration `it`, second half: alpha = rz/pq, x += alpha p, r -= alpha q,
// z = r / diag, rz[it+1], rr[it+1].
__global__ __launch_bounds__(kThreads) void k_pcg_b(Dims d, double* __restrict__ xv, double* __restrict__ r,
                                          double* __restrict__ zv, const double* __restrict__ pnew,
                                          const double* __restrict__ q, const double* __restrict__ diag,
                                          PcgState* st, int it, int jacobi) {
  __shared__ double alpha_sh;
  __shared__ int stop_sh;
  const int t = tid_lin();
  // operands first, so that their loads overlap the scalar decision below
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int i = x + d.nx * (y + d.ny * z);
  double xi = 0.0, pi = 0.0, ri = 0.0, qi = 0.0, di = 1.0;
  if (in) {
    xi = xv[i];
    pi = pnew[i];
    ri = r[i];
    qi = q[i];
    if (jacobi) di = diag[i];
  }
  if (t < 64) {  // the first wavefront decides
    const int stop = *(volatile int*)&st->done;
    if (t == 0) stop_sh = stop;
    if (!stop) {
      const int nb = st->nb;
      const double alpha = wave_part_sum(st->rz + (it & 3) * nb, nb) / wave_part_sum(st->pq + (it & 3) * nb, nb);
      if (t == 0) alpha_sh = alpha;
    }
  }
  __syncthreads();
  if (stop_sh) return;
  const double alpha = alpha_sh;
  double s[2] = {0.0, 0.0};
  if (in) {
    xv[i] = xi + alpha * pi;
    const double rn = ri - alpha * qi;
    r[i] = rn;
    if (jacobi) {
      const double zi = rn / di;
      zv[i] = zi;
      s[0] = rn * zi;
    }
    s[1] = rn * rn;
  }
  block_sum<2>(s);
  if (t == 0) {
    const int sl = ((it + 1) & 3) * st->nb + bid_lin();
    if (jacobi) st->rz[sl] = s[0];  // otherwise the preconditioner writes r.z
    st->rr[sl] = s[1];
  }
}

// ---------------------------------------------------------------------------
// The transient pressure ODE of a slightly compressible fluid in a slightly
// compressible rock (Eq. masscon4, Eq. spaceheat3), per cell:
//   D dp/dt = -(A p - b) + D (phi alpha_f / S) G2,   D = V rho(T) S,
//   S = phi (beta_f + alpha_b),  alpha_f = -rho'(T) / rho(T),
// A p = b the TPFA pressure system at the mobility of the last assembly
// (faces, Dirichlet x faces), G2 = dT/dt.  Writes J_p = -D^{-1} A as a
// stencil, G4 = dp/dt over G2 (in place), the Gershgorin interval of J_p
// and max |p|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_pressure_ode(Dims d, Phys ph, const double* __restrict__ poro,
                                                 const double* __restrict__ T, const double* __restrict__ p,
                                                 const double* __restrict__ tx, const double* __restrict__ ty,
                                                 const double* __restrict__ tz, double alpha_b, double beta_f,
                                                 double* __restrict__ coef, double* G, AsmReduce* red) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double lo = INFINITY, hi = -INFINITY, pmax = 0.0;
  if (x < d.nx && y < d.ny) {
    const int N = d.N;
    const int i = x + d.nx * (y + d.ny * z);
    const int pl = d.nx * d.ny;
    const bool has[6] = {x > 0, x + 1 < d.nx, y > 0, y + 1 < d.ny, d.dim == 3 && z > 0, d.dim == 3 && z + 1 < d.nz};
    const int nbi[6] = {has[0] ? i - 1 : i, has[1] ? i + 1 : i, has[2] ? i - d.nx : i,
                        has[3] ? i + d.nx : i, has[4] ? i - pl : i, has[5] ? i + pl : i};
    const FaceT f = load_faces(d, tx, ty, tz, x, y, z);
    const double pc = p[i];
    double pn[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pn[k] = p[nbi[k]];
    const double Ti = T[i], phi = poro[i], g2 = G[i];
    const double fk[6] = {f.w, f.e, f.s, f.n, f.b, f.t};
    const double dg = f.w + f.e + f.s + f.n + f.b + f.t;
    double r = -dg * pc;  // b - A p
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (has[k]) r += fk[k] * pn[k];
    if (x == 0) r += f.w * ph.p_left;
    if (x + 1 == d.nx) r += f.e * ph.p_right;
    const double rho = rho_of(Ti, ph);
    const double S = phi * (beta_f + alpha_b);
    const double inv = 1.0 / (d.dx * d.dy * d.dz * rho * S);
    const double af = -drho_of(ph) / rho;
    G[i] = r * inv + phi * af / S * g2;
    const double jc = -dg * inv;
    coef[i] = jc;
    double rad = 0.0;
    const int ndir = d.dim == 3 ? 7 : 5;
    for (int k = 1; k < ndir; ++k) {
      const double c = has[k - 1] ? fk[k - 1] * inv : 0.0;
      coef[k * N + i] = c;
      rad += c;
    }
    lo = jc - rad;
    hi = jc + rad;
    pmax = fabs(pc);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
    pmax = fmax(pmax, __shfl_down(pmax, off, 64));
  }
  __shared__ double sh[3][kThreads / 64];
  const int t = tid_lin();
  if ((t & 63) == 0) {
    sh[0][t >> 6] = lo;
    sh[1][t >> 6] = hi;
    sh[2][t >> 6] = pmax;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      sh[0][0] = fmin(sh[0][0], sh[0][w]);
      sh[1][0] = fmax(sh[1][0], sh[1][w]);
      sh[2][0] = fmax(sh[2][0], sh[2][w]);
    }
    const int k = red_slot();
    atomicMin(&red->lo[k], ord_encode(sh[0][0]));
    atomicMax(&red->hi[k], ord_encode(sh[1][0]));
    atomicMax(&red->tmax[k], ord_encode(sh[2][0]));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
hipError_t launch_transmissibility(const Dims& d, const Phys& ph, const double* logk, const double* T,
                                   double* tx, double* ty, double* tz, hipStream_t s) {
  hipLaunchKernelGGL(k_transmissibility, cell_grid(d), cell_block(), 0, s, d, ph, logk, T, tx, ty, tz);
  return hipGetLastError();
}

hipError_t launch_face_fluxes(const Dims& d, const Phys& ph, const double* p, const double* tx,
                              const double* ty, const double* tz, double* fx, double* fy, double* fz,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_face_fluxes, cell_grid(d), cell_block(), 0, s, d, ph, p, tx, ty, tz, fx, fy, fz);
  return hipGetLastError();
}

hipError_t launch_reset_reduce(AsmReduce* r, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_reduce, dim3(1), dim3(64), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_assemble(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                           const double* fy, const double* fz, const double* T, double* coef, double* F,
                           AsmReduce* red, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, cell_grid(d), cell_block(), 0, s, d, ph, poro, fx, fy, fz, T, coef, F, red);
  return hipGetLastError();
}

hipError_t launch_gershgorin(const Dims& d, const double* coef, AsmReduce* red, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_reduce, dim3(1), dim3(64), 0, s, red);
  hipLaunchKernelGGL(k_gershgorin, cell_grid(d), cell_block(), 0, s, d, coef, red);
  return hipGetLastError();
}

hipError_t launch_absmax(const Dims& d, const double* v, AsmReduce* red, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_vmax, dim3(1), dim3(64), 0, s, red);
  hipLaunchKernelGGL(k_absmax, cell_grid(d), cell_block(), 0, s, d, v, red);
  return hipGetLastError();
}

hipError_t launch_stencil_axpy(const Dims& d, const double* coef, const double* v, const double* u,
                               double* w, hipStream_t s, const double* g, double tg) {
  hipLaunchKernelGGL(k_stencil_axpy, cell_grid(d), cell_block(), 0, s, d, coef, v, u, w, g, tg);
  return hipGetLastError();
}

hipError_t launch_pressure_ode(const Dims& d, const Phys& ph, const double* poro, const double* T, const double* p,
                               const double* tx, const double* ty, const double* tz, double alpha_b, double beta_f,
                               double* coef, double* G, AsmReduce* red, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_reduce, dim3(1), dim3(64), 0, s, red);
  hipLaunchKernelGGL(k_pressure_ode, cell_grid(d), cell_block(), 0, s, d, ph, poro, T, p, tx, ty, tz, alpha_b, beta_f,
                     coef, G, red);
  return hipGetLastError();
}

hipError_t launch_time_rate(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                            const double* T, double dTl, double dTr, double* Gt, hipStream_t s) {
  hipLaunchKernelGGL(k_time_rate, cell_grid(d), cell_block(), 0, s, d, ph, poro, fx, T, dTl, dTr, Gt);
  return hipGetLastError();
}

hipError_t launch_axpby(const Dims& d, double* y, double a, const double* x, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, cell_grid(d), cell_block(), 0, s, d, y, a, x, b);
  return hipGetLastError();
}

hipError_t launch_pcg_reset(PcgState* st, double tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_reset, dim3(1), dim3(256), 0, s, st, tol2);
  return hipGetLastError();
}

hipError_t launch_pcg_start(const Dims& d, const Phys& ph, const double* tx, const double* ty,
                            const double* tz, const double* x, double* r, double* z, double* p0,
                            double* diag, PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start, cell_grid(d), cell_block(), 0, s, d, ph, tx, ty, tz, x, r, z, p0, diag, st);
  return hipGetLastError();
}

hipError_t launch_pcg_start_rhs(const Dims& d, const double* tx, const double* ty, const double* tz,
                                const double* rhs, double* x, double* r, double* z, double* p0, double* diag,
                                PcgState* st, int jacobi, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start_rhs, cell_grid(d), cell_block(), 0, s, d, tx, ty, tz, rhs, x, r, z, p0, diag, st,
                     jacobi);
  return hipGetLastError();
}

hipError_t launch_dd_residual(const Dims& d, const Phys& ph, const double* tx, const double* ty,
                              const double* tz, const double* phi, const double* plo, double* r, PcgState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_dd_residual, cell_grid(d), cell_block(), 0, s, d, ph, tx, ty, tz, phi, plo, r, st);
  return hipGetLastError();
}

hipError_t launch_pressure_extrapolate(const Dims& d, double* phi, double* plo, double* prev, int extrapolate,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_pressure_extrapolate, cell_grid(d), cell_block(), 0, s, d, phi, plo, prev, extrapolate);
  return hipGetLastError();
}

hipError_t launch_dd_update(const Dims& d, double* phi, double* plo, const double* delta, hipStream_t s) {
  hipLaunchKernelGGL(k_dd_update, cell_grid(d), cell_block(), 0, s, d, phi, plo, delta);
  return hipGetLastError();
}

hipError_t launch_face_fluxes_dd(const Dims& d, const Phys& ph, const double* phi, const double* plo,
                                 const double* tx, const double* ty, const double* tz, double* fx, double* fy,
                                 double* fz, hipStream_t s) {
  hipLaunchKernelGGL(k_face_fluxes_dd, cell_grid(d), cell_block(), 0, s, d, ph, phi, plo, tx, ty, tz, fx, fy, fz);
  return hipGetLastError();
}

hipError_t launch_pcg_a(const Dims& d, const double* tx, const double* ty, const double* tz, const double* z,
                        const double* pold, double* pnew, double* q, PcgState* st, int it, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1) {
  launch_timed(k_pcg_a, cell_grid(d), cell_block(), 0, s, e0, e1, d, tx, ty, tz, z, pold, pnew, q, st, it);
  return hipGetLastError();
}

hipError_t launch_pcg_b(const Dims& d, double* x, double* r, double* z, const double* pnew, const double* q,
                        const double* diag, PcgState* st, int it, int jacobi, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  launch_timed(k_pcg_b, cell_grid(d), cell_block(), 0, s, e0, e1, d, x, r, z, pnew, q, diag, st, it, jacobi);
  return hipGetLastError();
}

}  // namespace erem
