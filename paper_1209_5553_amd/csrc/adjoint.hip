// Adjoint kernels of the coupled EREM step on 2D grids (reverse mode of
// the forward path in fields.hip and leja.hip).
//
// Forward step (Sec. 3.1 discretisation, Sec. 3.2.2 sequential coupling,
// Eq. EERM with the Newton-Leja form of Sec. 4.2, Eq. newt):
//   m = rho(T) e^{logK} / mu(T);  t = TPFA(m);  A_p(t) p = r(t);  F = t dp
//   R = A_h(F) T + b(F);  G = R / (V C(T));  J = D_T G
//   u_{j+1} = u_j + delta sum_k d_k q_k,  q_0 = G + J u_j,
//   q_k = (J / gamma - shift_k) q_{k-1},  T+ = T + u_s
// The reverse sweep runs the recurrence backwards with the transposed
// stencil (s_m = d_m ybar, s_{k-1} = d_{k-1} ybar + (J/gamma - shift_k)^T s_k)
// and accumulates Jbar += s_k q_{k-1}^T / gamma on the stencil pattern; then
// it goes back through G and J to R, C(T) and the heat-operator rows, from
// the rows to the face fluxes (upwind directions fixed), from the fluxes to
// p and t, through the pressure system (adjoint solve with the same SPD
// matrix), the harmonic means and the mobility law.
//
// All kernels: one thread per cell, 64 x 4 blocks (a wavefront per row
// segment, coalesced along x).  Every output element has exactly one writer.
#include "adjoint.h"

#include <cmath>

namespace erem {

namespace {

__device__ inline int fxi(const Dims& d, int x, int y) { return y * (d.nx + 1) + x; }
__device__ inline int fyi(const Dims& d, int x, int y) { return y * d.nx + x; }

// J^T s at cell (x, y): the coefficient of each neighbour's row toward i.
// Neighbour indices of cell i, the cell itself where the neighbour is
// missing: every load below is in bounds and issued without a branch, and
// the missing neighbours' terms are dropped by a select.
struct Nbrs {
  bool hw, he, hs, hn;
  int w, e, s, n;
};
__device__ inline Nbrs nbrs(const Dims& d, int x, int y, int i) {
  Nbrs b;
  b.hw = x > 0;
  b.he = x + 1 < d.nx;
  b.hs = y > 0;
  b.hn = y + 1 < d.ny;
  b.w = b.hw ? i - 1 : i;
  b.e = b.he ? i + 1 : i;
  b.s = b.hs ? i - d.nx : i;
  b.n = b.hn ? i + d.nx : i;
  return b;
}

__device__ inline double jt_apply(const Dims& d, const double* __restrict__ coef, const double* __restrict__ s,
                                  int x, int y, int i) {
  const int N = d.N;
  const Nbrs b = nbrs(d, x, y, i);
  const double tw = coef[2 * N + b.w] * s[b.w], te = coef[N + b.e] * s[b.e];
  const double ts = coef[4 * N + b.s] * s[b.s], tn = coef[3 * N + b.n] * s[b.n];
  double v = coef[i] * s[i];
  v += b.hw ? tw : 0.0;
  v += b.he ? te : 0.0;
  v += b.hs ? ts : 0.0;
  v += b.hn ? tn : 0.0;
  return v;
}

// One row of the heat operator R = A_h T + b (conduction with the uniform
// conductivity's TPFA transmissibility, upwind advection c_f F T_upwind).
struct HeatRow {
  double diag, b;
  double a[4];  // -x, +x, -y, +y neighbours
};

__device__ inline HeatRow heat_row(const Dims& d, const Phys& ph, const double* __restrict__ fx,
                                   const double* __restrict__ fy, int x, int y) {
  HeatRow r{0.0, 0.0, {0.0, 0.0, 0.0, 0.0}};
  const double ax = d.dy * d.dz, ay = d.dx * d.dz;
  const double tcx = ph.lam * ax / d.dx, tcy = ph.lam * ay / d.dy;
  const double tcb = ph.lam * ax / (0.5 * d.dx);
  const double cf = ph.c_f;
  {
    const double f = fx[fxi(d, x, y)];  // > 0 enters the cell
    if (x > 0) {
      r.a[0] = tcx + cf * fmax(f, 0.0);
      r.diag -= tcx + cf * fmax(-f, 0.0);
    } else {
      if (ph.dirichlet_left) {
        r.diag -= tcb;
        r.b += tcb * ph.T_left;
      }
      if (f > 0.0) r.b += cf * f * ph.T_left; else r.diag -= cf * (-f);
    }
  }
  {
    const double f = fx[fxi(d, x + 1, y)];  // > 0 leaves the cell
    if (x + 1 < d.nx) {
      r.a[1] = tcx + cf * fmax(-f, 0.0);
      r.diag -= tcx + cf * fmax(f, 0.0);
    } else {
      if (f >= 0.0) r.diag -= cf * f; else r.b += cf * (-f) * ph.T_right;
    }
  }
  if (y > 0) {
    const double f = fy[fyi(d, x, y)];
    r.a[2] = tcy + cf * fmax(f, 0.0);
    r.diag -= tcy + cf * fmax(-f, 0.0);
  }
  if (y + 1 < d.ny) {
    const double f = fy[fyi(d, x, y + 1)];
    r.a[3] = tcy + cf * fmax(-f, 0.0);
    r.diag -= tcy + cf * fmax(f, 0.0);
  }
  return r;
}

__device__ inline double rho_law(double T, const Phys& ph) {
  return ph.law == 1 ? 1000.0 * (1.0 - 3.0e-4 * (T - 20.0)) : ph.rho0;
}
__device__ inline double mu_law(double T, const Phys& ph) {
  return ph.law == 1 ? 2.414e-5 * pow(10.0, 247.8 / (T + 133.0)) : ph.mu0;
}
__device__ inline double mob(const Phys& ph, const double* logk, const double* T, int i) {
  const double Ti = T[i];
  return rho_law(Ti, ph) * exp(logk[i]) / mu_law(Ti, ph);
}

#define CELL_INDEX                                   \
  const int x = blockIdx.x * kBX + threadIdx.x;      \
  const int y = blockIdx.y * kBY + threadIdx.y;      \
  if (x >= d.nx || y >= d.ny) return;                \
  const int i = x + d.nx * y;

__global__ __launch_bounds__(kThreads) void k_adj_scale(Dims d, const double* __restrict__ ubar, double scale,
                                              double* __restrict__ s_out) {
  CELL_INDEX
  s_out[i] = scale * ubar[i];
}

__global__ __launch_bounds__(kThreads) void k_adj_rev_term(Dims d, const double* __restrict__ coef,
                                                 const double* __restrict__ s_in,
                                                 const double* __restrict__ q, const double* __restrict__ ubar,
                                                 double yscale, double inv_g, double shift_k,
                                                 double* __restrict__ jbar, double* __restrict__ s_out) {
  CELL_INDEX
  const int N = d.N;
  // every load first (jbar too), then the stores: the loads issue together
  const Nbrs b = nbrs(d, x, y, i);
  const double si = s_in[i];
  const double jt = jt_apply(d, coef, s_in, x, y, i);
  const double ub = ubar[i];
  const double qc = q[i], qw = q[b.w], qe = q[b.e], qs = q[b.s], qn = q[b.n];
  double jb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) jb[k] = jbar[k * N + i];
  s_out[i] = yscale * ub + inv_g * jt - shift_k * si;
  const double g = inv_g * si;
  // a missing neighbour's entry of jbar is never read; it gets 0 added
  jbar[i] = jb[0] + g * qc;
  jbar[N + i] = jb[1] + (b.hw ? g * qw : 0.0);
  jbar[2 * N + i] = jb[2] + (b.he ? g * qe : 0.0);
  jbar[3 * N + i] = jb[3] + (b.hs ? g * qs : 0.0);
  jbar[4 * N + i] = jb[4] + (b.hn ? g * qn : 0.0);
}

__global__ __launch_bounds__(kThreads) void k_adj_substep(Dims d, const double* __restrict__ coef,
                                                const double* __restrict__ r, const double* __restrict__ u,
                                                double* __restrict__ wbar, double* __restrict__ ubar,
                                                double* __restrict__ jbar) {
  CELL_INDEX
  const int N = d.N;
  const double ri = r[i];
  const double wb = wbar[i];
  if (u) {
    // every load first (jbar too), then the stores
    const Nbrs b = nbrs(d, x, y, i);
    const double jt = jt_apply(d, coef, r, x, y, i);
    const double ub = ubar[i];
    const double uc = u[i], uw = u[b.w], ue = u[b.e], us = u[b.s], un = u[b.n];
    double jb[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) jb[k] = jbar[k * N + i];
    wbar[i] = wb + ri;
    ubar[i] = ub + jt;
    jbar[i] = jb[0] + ri * uc;
    jbar[N + i] = jb[1] + (b.hw ? ri * uw : 0.0);
    jbar[2 * N + i] = jb[2] + (b.he ? ri * ue : 0.0);
    jbar[3 * N + i] = jb[3] + (b.hs ? ri * us : 0.0);
    jbar[4 * N + i] = jb[4] + (b.hn ? ri * un : 0.0);
  } else {
    wbar[i] = wb + ri;
  }
}

// G = R inv, J_ii = diag inv - R C' inv / C, J_ik = a_k inv, inv = 1/(V C).
__global__ __launch_bounds__(kThreads) void k_adj_heat_cell(Dims d, Phys ph, const double* __restrict__ poro,
                                                  const double* __restrict__ fx, const double* __restrict__ fy,
                                                  const double* __restrict__ T, const double* __restrict__ jbar,
                                                  const double* __restrict__ wbar, double* __restrict__ Tbar,
                                                  double* __restrict__ rbar, double* __restrict__ dbar,
                                                  double* __restrict__ abar) {
  CELL_INDEX
  const int N = d.N;
  const HeatRow hr = heat_row(d, ph, fx, fy, x, y);
  const double Ti = T[i];
  double tn[4] = {0.0, 0.0, 0.0, 0.0};
  if (x > 0) tn[0] = T[i - 1];
  if (x + 1 < d.nx) tn[1] = T[i + 1];
  if (y > 0) tn[2] = T[i - d.nx];
  if (y + 1 < d.ny) tn[3] = T[i + d.nx];
  double R = hr.diag * Ti + hr.b;
  for (int k = 0; k < 4; ++k) R += hr.a[k] * tn[k];
  const double V = d.dx * d.dy * d.dz;
  const double phi = poro[i];
  const double C = phi * rho_law(Ti, ph) * ph.c_f + (1.0 - phi) * ph.rhoc_s;
  const double dC = phi * (ph.law == 1 ? -0.3 : 0.0) * ph.c_f;
  const double inv = 1.0 / (V * C);
  const double jb0 = jbar[i];
  const double wb = wbar[i];
  const double Rb = wb * inv - jb0 * dC * inv / C;
  double invb = wb * R + jb0 * (hr.diag - R * dC / C);
  for (int k = 0; k < 4; ++k) invb += jbar[(k + 1) * N + i] * hr.a[k];
  const double Cb = jb0 * R * dC * inv / (C * C) - invb * inv / C;
  Tbar[i] += Cb * dC;
  rbar[i] = Rb;
  dbar[i] = jb0 * inv + Rb * Ti;
  for (int k = 0; k < 4; ++k) abar[k * N + i] = jbar[(k + 1) * N + i] * inv + Rb * tn[k];
}

__global__ __launch_bounds__(kThreads) void k_adj_heat_face(Dims d, Phys ph, const double* __restrict__ fx,
                                                  const double* __restrict__ fy, const double* __restrict__ rbar,
                                                  const double* __restrict__ dbar, const double* __restrict__ abar,
                                                  double* __restrict__ Tbar, double* __restrict__ fxbar,
                                                  double* __restrict__ fybar) {
  CELL_INDEX
  const int N = d.N;
  const double ax = d.dy * d.dz, ay = d.dx * d.dz;
  const double tcx = ph.lam * ax / d.dx, tcy = ph.lam * ay / d.dy;
  const double cf = ph.c_f;
  const HeatRow hr = heat_row(d, ph, fx, fy, x, y);
  // Tbar_i += sum_j A_ji Rbar_j
  double tb = hr.diag * rbar[i];
  if (x > 0) tb += (tcx + cf * fmax(-fx[fxi(d, x, y)], 0.0)) * rbar[i - 1];          // row i-1, +x entry
  if (x + 1 < d.nx) tb += (tcx + cf * fmax(fx[fxi(d, x + 1, y)], 0.0)) * rbar[i + 1];  // row i+1, -x entry
  if (y > 0) tb += (tcy + cf * fmax(-fy[fyi(d, x, y)], 0.0)) * rbar[i - d.nx];       // row i-nx, +y entry
  if (y + 1 < d.ny) tb += (tcy + cf * fmax(fy[fyi(d, x, y + 1)], 0.0)) * rbar[i + d.nx];
  Tbar[i] += tb;
  // -x face of this cell
  {
    const double f = fx[fxi(d, x, y)];
    double fb;
    if (x > 0) {
      fb = (f > 0.0 ? cf * abar[i] : 0.0) + (f < 0.0 ? cf * dbar[i] : 0.0)                 // this cell's row
           + (f < 0.0 ? -cf * abar[N + i - 1] : 0.0) + (f > 0.0 ? -cf * dbar[i - 1] : 0.0);  // the left cell's row
    } else {
      fb = f > 0.0 ? cf * ph.T_left * rbar[i] : cf * dbar[i];
    }
    fxbar[fxi(d, x, y)] = fb;
  }
  if (x + 1 == d.nx) {
    const double f = fx[fxi(d, x + 1, y)];
    fxbar[fxi(d, x + 1, y)] = f >= 0.0 ? -cf * dbar[i] : -cf * ph.T_right * rbar[i];
  }
  // -y face of this cell (closed boundary faces carry no flux)
  if (y > 0) {
    const double f = fy[fyi(d, x, y)];
    fybar[fyi(d, x, y)] = (f > 0.0 ? cf * abar[2 * N + i] : 0.0) + (f < 0.0 ? cf * dbar[i] : 0.0) +
                          (f < 0.0 ? -cf * abar[3 * N + i - d.nx] : 0.0) + (f > 0.0 ? -cf * dbar[i - d.nx] : 0.0);
  } else {
    fybar[fyi(d, x, 0)] = 0.0;
  }
  if (y + 1 == d.ny) fybar[fyi(d, x, y + 1)] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_adj_flux_p(Dims d, const double* __restrict__ tx,
                                               const double* __restrict__ ty, const double* __restrict__ fxbar,
                                               const double* __restrict__ fybar, double* __restrict__ pbar) {
  CELL_INDEX
  // F on the -x / -y face is t (p_nb - p_i), on the +x / +y face t (p_i - p_nb);
  // the Dirichlet x faces have the same form with the boundary pressure.
  double pb = fxbar[fxi(d, x + 1, y)] * tx[fxi(d, x + 1, y)] - fxbar[fxi(d, x, y)] * tx[fxi(d, x, y)];
  if (y > 0) pb -= fybar[fyi(d, x, y)] * ty[fyi(d, x, y)];
  if (y + 1 < d.ny) pb += fybar[fyi(d, x, y + 1)] * ty[fyi(d, x, y + 1)];
  pbar[i] = pb;
}

__device__ inline void band_store(PcgState* st, double rr, double bb) {
  __shared__ double sh[kThreads / 64][2];
  for (int off = 32; off > 0; off >>= 1) {
    rr += __shfl_down(rr, off, 64);
    bb += __shfl_down(bb, off, 64);
  }
  const int t = threadIdx.x + threadIdx.y * kBX;
  if ((t & 63) == 0) {
    sh[t >> 6][0] = rr;
    sh[t >> 6][1] = bb;
  }
  __syncthreads();
  if (t == 0) {
    const int b = blockIdx.x + gridDim.x * blockIdx.y;  // the block's band
    st->rr[b] = sh[0][0] + sh[1][0] + sh[2][0] + sh[3][0];
    st->bb_sl[b] = sh[0][1] + sh[1][1] + sh[2][1] + sh[3][1];
  }
}

__global__ __launch_bounds__(kThreads) void k_spd_residual(Dims d, const double* __restrict__ tx,
                                                 const double* __restrict__ ty, const double* __restrict__ xv,
                                                 const double* __restrict__ b, double* __restrict__ r,
                                                 PcgState* st) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  double rr = 0.0, bb = 0.0;
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * y;
    const double xi = xv[i];
    double ax = 0.0;
    ax += tx[fxi(d, x, y)] * (xi - (x > 0 ? xv[i - 1] : 0.0));
    ax += tx[fxi(d, x + 1, y)] * (xi - (x + 1 < d.nx ? xv[i + 1] : 0.0));
    if (y > 0) ax += ty[fyi(d, x, y)] * (xi - xv[i - d.nx]);
    if (y + 1 < d.ny) ax += ty[fyi(d, x, y + 1)] * (xi - xv[i + d.nx]);
    const double bi = b[i];
    const double ri = bi - ax;
    r[i] = ri;
    rr = ri * ri;
    bb = bi * bi;
  }
  band_store(st, rr, bb);
}

__global__ __launch_bounds__(kThreads) void k_adj_trans(Dims d, Phys ph, const double* __restrict__ logk,
                                              const double* __restrict__ T, const double* __restrict__ phi,
                                              const double* __restrict__ plo, const double* __restrict__ fxbar,
                                              const double* __restrict__ fybar, const double* __restrict__ lam,
                                              double* __restrict__ Tbar, double* __restrict__ logkbar) {
  CELL_INDEX
  const double ax = d.dy * d.dz, ay = d.dx * d.dz;
  const double hx = 0.5 * d.dx, hy = 0.5 * d.dy;
  const double mi = mob(ph, logk, T, i);
  auto dp = [&](int a, int b) { return (phi[a] - phi[b]) + (plo[a] - plo[b]); };
  // d t / d m_i of a harmonic-mean face with neighbour mobility mj
  auto dharm = [&](double area, double h, double mj) {
    const double s = mi + mj;
    return area * mj * mj / (h * s * s);
  };
  double mb = 0.0;
  if (x > 0) {
    const int j = i - 1;
    const double tb = (fxbar[fxi(d, x, y)] - (lam[j] - lam[i])) * dp(j, i);
    mb += tb * dharm(ax, hx, mob(ph, logk, T, j));
  } else {
    const double pdiff = (ph.p_left - phi[i]) - plo[i];
    mb += (fxbar[fxi(d, 0, y)] + lam[i]) * pdiff * (ax / hx);
  }
  if (x + 1 < d.nx) {
    const int j = i + 1;
    const double tb = (fxbar[fxi(d, x + 1, y)] - (lam[i] - lam[j])) * dp(i, j);
    mb += tb * dharm(ax, hx, mob(ph, logk, T, j));
  } else {
    const double pdiff = (phi[i] - ph.p_right) + plo[i];
    mb += (fxbar[fxi(d, x + 1, y)] - lam[i]) * pdiff * (ax / hx);
  }
  if (y > 0) {
    const int j = i - d.nx;
    const double tb = (fybar[fyi(d, x, y)] - (lam[j] - lam[i])) * dp(j, i);
    mb += tb * dharm(ay, hy, mob(ph, logk, T, j));
  }
  if (y + 1 < d.ny) {
    const int j = i + d.nx;
    const double tb = (fybar[fyi(d, x, y + 1)] - (lam[i] - lam[j])) * dp(i, j);
    mb += tb * dharm(ay, hy, mob(ph, logk, T, j));
  }
  logkbar[i] += mb * mi;
  if (ph.law == 1) {
    const double Ti = T[i];
    const double dlog_rho = -0.3 / rho_law(Ti, ph);
    const double dlog_mu = -247.8 * 2.302585092994045684 / ((Ti + 133.0) * (Ti + 133.0));
    Tbar[i] += mb * mi * (dlog_rho - dlog_mu);
  }
}

#undef CELL_INDEX

inline dim3 grid2(const Dims& d) { return dim3((d.nx + kBX - 1) / kBX, (d.ny + kBY - 1) / kBY, 1); }
inline dim3 block2() { return dim3(kBX, kBY, 1); }

}  // namespace

hipError_t launch_adj_scale(const Dims& d, const double* ubar, double scale, double* s_out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_scale, grid2(d), block2(), 0, s, d, ubar, scale, s_out);
  return hipGetLastError();
}

hipError_t launch_adj_rev_term(const Dims& d, const double* coef, const double* s_in, const double* q_prev,
                               const double* ubar, double yscale, double inv_g, double shift_k, double* jbar,
                               double* s_out, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_timed(k_adj_rev_term, grid2(d), block2(), 0, s, e0, e1, d, coef, s_in, q_prev, ubar, yscale, inv_g,
               shift_k, jbar, s_out);
  return hipGetLastError();
}

hipError_t launch_adj_substep(const Dims& d, const double* coef, const double* rbar, const double* u, double* wbar,
                              double* ubar, double* jbar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_substep, grid2(d), block2(), 0, s, d, coef, rbar, u, wbar, ubar, jbar);
  return hipGetLastError();
}

hipError_t launch_adj_heat_cell(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                                const double* fy, const double* T, const double* jbar, const double* wbar,
                                double* Tbar, double* rbar, double* dbar, double* abar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_heat_cell, grid2(d), block2(), 0, s, d, ph, poro, fx, fy, T, jbar, wbar, Tbar, rbar,
                     dbar, abar);
  return hipGetLastError();
}

hipError_t launch_adj_heat_face(const Dims& d, const Phys& ph, const double* fx, const double* fy,
                                const double* rbar, const double* dbar, const double* abar, double* Tbar,
                                double* fxbar, double* fybar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_heat_face, grid2(d), block2(), 0, s, d, ph, fx, fy, rbar, dbar, abar, Tbar, fxbar,
                     fybar);
  return hipGetLastError();
}

hipError_t launch_adj_flux_p(const Dims& d, const double* tx, const double* ty, const double* fxbar,
                             const double* fybar, double* pbar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_flux_p, grid2(d), block2(), 0, s, d, tx, ty, fxbar, fybar, pbar);
  return hipGetLastError();
}

hipError_t launch_spd_residual(const Dims& d, const double* tx, const double* ty, const double* x, const double* b,
                               double* r, PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_spd_residual, grid2(d), block2(), 0, s, d, tx, ty, x, b, r, st);
  return hipGetLastError();
}

hipError_t launch_adj_trans(const Dims& d, const Phys& ph, const double* logk, const double* T, const double* phi,
                            const double* plo, const double* fxbar, const double* fybar, const double* lam,
                            double* Tbar, double* logkbar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_trans, grid2(d), block2(), 0, s, d, ph, logk, T, phi, plo, fxbar, fybar, lam,
                     Tbar, logkbar);
  return hipGetLastError();
}

}  // namespace erem
