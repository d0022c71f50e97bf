// Aggregation multigrid preconditioner for the TPFA pressure operator.
//
// Levels: cells aggregated 2 x 2 (x 2 in 3D).  With piecewise-constant
// prolongation P the Galerkin operator P^T A P of a two-point-flux matrix is
// again a two-point-flux matrix whose face transmissibility is the sum of the
// fine transmissibilities crossing the coarse face (Dirichlet faces included),
// so every level keeps the same face-array layout as the fine grid.
// Smoother: damped Jacobi (omega 0.8), the same sweeps before and after the
// coarse correction; the coarse correction is over-relaxed by omega_c; the
// cycle is symmetric, so it is a valid conjugate-gradient preconditioner.
// Fine levels run one kernel per operation; the levels with at most
// kMgLdsCells cells run inside one workgroup with everything in LDS.
#include "device.h"
#include "mg.h"

namespace erem {

namespace {

constexpr double kOmega = 0.8;

__device__ inline int fxi(int nx, int ny, int x, int y, int z) { return (z * ny + y) * (nx + 1) + x; }
__device__ inline int fyi(int nx, int ny, int x, int y, int z) { return (z * (ny + 1) + y) * nx + x; }
__device__ inline int fzi(int nx, int ny, int x, int y, int z) { return (z * ny + y) * nx + x; }

__device__ inline bool pcg_done(const PcgState* st) { return st && *(volatile const int*)&st->done; }

// (A v)_i without the diagonal: sum over interior faces of t * v_nb.
__device__ inline double offdiag_sum(const MgLevelDev& L, const double* __restrict__ tx,
                                     const double* __restrict__ ty, const double* __restrict__ tz,
                                     const double* __restrict__ v, int x, int y, int z, int i) {
  double s = 0.0;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  if (x > 0) s += tx[fxi(nx, ny, x, y, z)] * v[i - 1];
  if (x + 1 < nx) s += tx[fxi(nx, ny, x + 1, y, z)] * v[i + 1];
  if (y > 0) s += ty[fyi(nx, ny, x, y, z)] * v[i - nx];
  if (y + 1 < ny) s += ty[fyi(nx, ny, x, y + 1, z)] * v[i + nx];
  if (z > 0) s += tz[fzi(nx, ny, x, y, z)] * v[i - nx * ny];
  if (z + 1 < nz) s += tz[fzi(nx, ny, x, y, z + 1)] * v[i + nx * ny];
  return s;
}

// ---------------------------------------------------------------------------
// Setup: coarse faces and diagonal from the fine faces.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mg_coarsen(MgLevelDev F, MgLevelDev C) {
  const int X = blockIdx.x * kBX + threadIdx.x;
  const int Y = blockIdx.y * kBY + threadIdx.y;
  const int Z = blockIdx.z;
  if (X >= C.nx || Y >= C.ny) return;
  const int fnx = F.nx, fny = F.ny, fnz = F.nz;
  const int y0 = 2 * Y, y1 = min(2 * Y + 1, fny - 1);
  const int x0 = 2 * X, x1 = min(2 * X + 1, fnx - 1);
  const int z0 = C.nz > 1 || fnz > 1 ? 2 * Z : 0;
  const int z1 = fnz > 1 ? min(2 * Z + 1, fnz - 1) : 0;
  // sum of fine x faces at fine face index xf over the rows / layers of this aggregate
  auto sum_x = [&](int xf) {
    double s = 0.0;
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) s += F.tx[fxi(fnx, fny, xf, y, z)];
    return s;
  };
  auto sum_y = [&](int yf) {
    double s = 0.0;
    for (int z = z0; z <= z1; ++z)
      for (int x = x0; x <= x1; ++x) s += F.ty[fyi(fnx, fny, x, yf, z)];
    return s;
  };
  auto sum_z = [&](int zf) {
    double s = 0.0;
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) s += F.tz[fzi(fnx, fny, x, y, zf)];
    return s;
  };
  const double w = sum_x(2 * X);
  const double e = sum_x(min(2 * X + 2, fnx));
  const double s = sum_y(2 * Y);
  const double n = sum_y(min(2 * Y + 2, fny));
  double b = 0.0, t = 0.0;
  if (F.nz > 1) {
    b = sum_z(2 * Z);
    t = sum_z(min(2 * Z + 2, fnz));
  }
  const int cnx = C.nx, cny = C.ny;
  C.tx[fxi(cnx, cny, X + 1, Y, Z)] = e;
  if (X == 0) C.tx[fxi(cnx, cny, 0, Y, Z)] = w;
  C.ty[fyi(cnx, cny, X, Y + 1, Z)] = n;
  if (Y == 0) C.ty[fyi(cnx, cny, X, 0, Z)] = s;
  C.tz[fzi(cnx, cny, X, Y, Z + 1)] = t;
  if (Z == 0) C.tz[fzi(cnx, cny, X, Y, 0)] = b;
  C.diag[X + cnx * (Y + cny * Z)] = w + e + s + n + b + t;
}

// Two damped-Jacobi sweeps from zero: x1 = w b / D, x2 = x1 + w (b - A x1) / D.
__global__ __launch_bounds__(kThreads) void k_mg_smooth_down(MgLevelDev L, const double* __restrict__ b,
                                                   double* __restrict__ xout, const PcgState* st) {
  if (pcg_done(st)) return;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const int i = x + L.nx * (y + L.ny * z);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  auto x1 = [&](int j) { return kOmega * b[j] / L.diag[j]; };
  double s = 0.0;
  if (x > 0) s += L.tx[fxi(nx, ny, x, y, z)] * x1(i - 1);
  if (x + 1 < nx) s += L.tx[fxi(nx, ny, x + 1, y, z)] * x1(i + 1);
  if (y > 0) s += L.ty[fyi(nx, ny, x, y, z)] * x1(i - nx);
  if (y + 1 < ny) s += L.ty[fyi(nx, ny, x, y + 1, z)] * x1(i + nx);
  if (z > 0) s += L.tz[fzi(nx, ny, x, y, z)] * x1(i - nx * ny);
  if (z + 1 < nz) s += L.tz[fzi(nx, ny, x, y, z + 1)] * x1(i + nx * ny);
  const double D = L.diag[i];
  const double xi = kOmega * b[i] / D;
  // b - A x1 = b - D x1 + sum t x1_nb
  xout[i] = xi + kOmega * (b[i] - D * xi + s) / D;
}

// Residual b - A x of the fine cells of one aggregate, summed into the coarse rhs.
__global__ __launch_bounds__(kThreads) void k_mg_restrict(MgLevelDev F, MgLevelDev C, const double* __restrict__ b,
                                                const double* __restrict__ xv, double* __restrict__ bc,
                                                const PcgState* st) {
  if (pcg_done(st)) return;
  const int X = blockIdx.x * kBX + threadIdx.x;
  const int Y = blockIdx.y * kBY + threadIdx.y;
  const int Z = blockIdx.z;
  if (X >= C.nx || Y >= C.ny) return;
  const int x1 = min(2 * X + 1, F.nx - 1), y1 = min(2 * Y + 1, F.ny - 1);
  const int z0 = F.nz > 1 ? 2 * Z : 0, z1 = F.nz > 1 ? min(2 * Z + 1, F.nz - 1) : 0;
  double acc = 0.0;
  for (int z = z0; z <= z1; ++z)
    for (int y = 2 * Y; y <= y1; ++y)
      for (int x = 2 * X; x <= x1; ++x) {
        const int i = x + F.nx * (y + F.ny * z);
        acc += b[i] - F.diag[i] * xv[i] + offdiag_sum(F, F.tx, F.ty, F.tz, xv, x, y, z, i);
      }
  bc[X + C.nx * (Y + C.ny * Z)] = acc;
}

// y = xc + w (b - A xc) / D with xc = x + omega_c e[parent] (own and neighbour values).
__global__ __launch_bounds__(kThreads) void k_mg_prolong_smooth(MgLevelDev F, MgLevelDev C, const double* __restrict__ b,
                                                      const double* __restrict__ xv, const double* __restrict__ ec,
                                                      double omega_c, double* __restrict__ yout, const PcgState* st) {
  if (pcg_done(st)) return;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= F.nx || y >= F.ny) return;
  const int nx = F.nx, ny = F.ny, nz = F.nz;
  const int i = x + nx * (y + ny * z);
  const int cz = nz > 1 ? 1 : 0;
  auto xc = [&](int xx, int yy, int zz, int j) {
    return xv[j] + omega_c * ec[(xx >> 1) + C.nx * ((yy >> 1) + C.ny * (zz >> cz))];
  };
  double s = 0.0;
  if (x > 0) s += F.tx[fxi(nx, ny, x, y, z)] * xc(x - 1, y, z, i - 1);
  if (x + 1 < nx) s += F.tx[fxi(nx, ny, x + 1, y, z)] * xc(x + 1, y, z, i + 1);
  if (y > 0) s += F.ty[fyi(nx, ny, x, y, z)] * xc(x, y - 1, z, i - nx);
  if (y + 1 < ny) s += F.ty[fyi(nx, ny, x, y + 1, z)] * xc(x, y + 1, z, i + nx);
  if (z > 0) s += F.tz[fzi(nx, ny, x, y, z)] * xc(x, y, z - 1, i - nx * ny);
  if (z + 1 < nz) s += F.tz[fzi(nx, ny, x, y, z + 1)] * xc(x, y, z + 1, i + nx * ny);
  const double D = F.diag[i];
  const double xi = xc(x, y, z, i);
  yout[i] = xi + kOmega * (b[i] - D * xi + s) / D;
}

// Last Jacobi sweep: out = y + w (b - A y) / D.  With rz != nullptr (the
// finest level, b = r) also accumulates r . out into the CG ring slot.
__global__ __launch_bounds__(kThreads) void k_mg_smooth_final(MgLevelDev L, const double* __restrict__ b,
                                                    const double* __restrict__ yv, double* __restrict__ out,
                                                    PcgState* st, int rz_slot) {
  if (pcg_done(st)) return;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double part = 0.0;
  if (x < L.nx && y < L.ny) {
    const int i = x + L.nx * (y + L.ny * z);
    const double D = L.diag[i];
    const double v = yv[i] + kOmega * (b[i] - D * yv[i] + offdiag_sum(L, L.tx, L.ty, L.tz, yv, x, y, z, i)) / D;
    out[i] = v;
    part = b[i] * v;
  }
  if (rz_slot < 0) return;
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  __shared__ double sh[kThreads / 64];
  const int t = threadIdx.x + threadIdx.y * kBX;
  if ((t & 63) == 0) sh[t >> 6] = part;
  __syncthreads();
  if (t == 0) {
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    atomicAdd(&st->rz[rz_slot * kSlots + (bid & (kSlots - 1))], sh[0] + sh[1] + sh[2] + sh[3]);
  }
}

// ---------------------------------------------------------------------------
// Coarse levels in one workgroup: `ninner` V-cycles of levels lc..end
// (everything in LDS), from x = 0, on rhs b (global).  Writes x to out; with
// rz_slot >= 0 also b . out into the CG ring.
// ---------------------------------------------------------------------------
struct LdsLevel {
  double *tx, *ty, *tz, *diag, *B, *E, *T;
};

__device__ void lds_apply_smooth(const MgLevelDev& L, const LdsLevel& S, int sweeps, bool from_zero,
                                 double omega) {
  const int n = L.nx * L.ny * L.nz;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
      const double D = S.diag[c];
      double v;
      if (from_zero && sw == 0) {
        v = omega * S.B[c] / D;
      } else {
        const double e = S.E[c];
        v = e + omega * (S.B[c] - D * e + offdiag_sum(L, S.tx, S.ty, S.tz, S.E, x, y, z, c)) / D;
      }
      S.T[c] = v;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) S.E[c] = S.T[c];
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_mg_coarse_lds(MgCoarseArgs a, const double* __restrict__ bglob,
                                              double* __restrict__ out, PcgState* st, int rz_slot) {
  if (pcg_done(st)) return;
  extern __shared__ double smem[];
  LdsLevel S[kMgMaxLevels];
  // carve LDS and load faces / diagonal of every coarse level
  {
    double* p = smem;
    for (int l = 0; l < a.nlev; ++l) {
      const MgLevelDev& L = a.lev[l];
      const int n = L.nx * L.ny * L.nz;
      const int nfx = (L.nx + 1) * L.ny * L.nz, nfy = L.nx * (L.ny + 1) * L.nz;
      const int nfz = L.nz > 1 ? L.nx * L.ny * (L.nz + 1) : 0;  // 2D: z faces never read
      S[l].tx = p; p += nfx;
      S[l].ty = p; p += nfy;
      S[l].tz = p; p += nfz;
      S[l].diag = p; p += n;
      S[l].B = p; p += n;
      S[l].E = p; p += n;
      S[l].T = p; p += n;
      for (int j = threadIdx.x; j < nfx; j += blockDim.x) S[l].tx[j] = L.tx[j];
      for (int j = threadIdx.x; j < nfy; j += blockDim.x) S[l].ty[j] = L.ty[j];
      for (int j = threadIdx.x; j < nfz; j += blockDim.x) S[l].tz[j] = L.tz[j];
      for (int j = threadIdx.x; j < n; j += blockDim.x) S[l].diag[j] = L.diag[j];
    }
  }
  double* X = smem + a.lds_words;            // accumulated solution on the first coarse level
  double* R0 = X + a.n0;                      // original right-hand side
  const MgLevelDev& L0 = a.lev[0];
  const int n0 = a.n0;
  for (int j = threadIdx.x; j < n0; j += blockDim.x) {
    R0[j] = bglob[j];
    X[j] = 0.0;
  }
  __syncthreads();
  for (int cyc = 0; cyc < a.ninner; ++cyc) {
    // B_0 = R0 - A X
    for (int c = threadIdx.x; c < n0; c += blockDim.x) {
      const int x = c % L0.nx, y = (c / L0.nx) % L0.ny, z = c / (L0.nx * L0.ny);
      S[0].B[c] = R0[c] - S[0].diag[c] * X[c] + offdiag_sum(L0, S[0].tx, S[0].ty, S[0].tz, X, x, y, z, c);
    }
    __syncthreads();
    // down
    for (int l = 0; l + 1 < a.nlev; ++l) {
      const MgLevelDev& F = a.lev[l];
      const MgLevelDev& C = a.lev[l + 1];
      lds_apply_smooth(F, S[l], a.nu, true, kOmega);
      const int nc = C.nx * C.ny * C.nz;
      for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int X0 = c % C.nx, Y0 = (c / C.nx) % C.ny, Z0 = c / (C.nx * C.ny);
        const int x1 = min(2 * X0 + 1, F.nx - 1), y1 = min(2 * Y0 + 1, F.ny - 1);
        const int z0 = F.nz > 1 ? 2 * Z0 : 0, z1 = F.nz > 1 ? min(2 * Z0 + 1, F.nz - 1) : 0;
        double acc = 0.0;
        for (int z = z0; z <= z1; ++z)
          for (int y = 2 * Y0; y <= y1; ++y)
            for (int x = 2 * X0; x <= x1; ++x) {
              const int i = x + F.nx * (y + F.ny * z);
              acc += S[l].B[i] - S[l].diag[i] * S[l].E[i] +
                     offdiag_sum(F, S[l].tx, S[l].ty, S[l].tz, S[l].E, x, y, z, i);
            }
        S[l + 1].B[c] = acc;
      }
      __syncthreads();
    }
    // coarsest level: a single cell, solved exactly (undamped Jacobi)
    {
      const int l = a.nlev - 1;
      lds_apply_smooth(a.lev[l], S[l], a.nu_bottom, true, 1.0);
    }
    // up
    for (int l = a.nlev - 2; l >= 0; --l) {
      const MgLevelDev& F = a.lev[l];
      const MgLevelDev& C = a.lev[l + 1];
      const int n = F.nx * F.ny * F.nz;
      const int cz = F.nz > 1 ? 1 : 0;
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int x = c % F.nx, y = (c / F.nx) % F.ny, z = c / (F.nx * F.ny);
        S[l].E[c] += a.omega_c * S[l + 1].E[(x >> 1) + C.nx * ((y >> 1) + C.ny * (z >> cz))];
      }
      __syncthreads();
      lds_apply_smooth(F, S[l], a.nu, false, kOmega);
    }
    for (int c = threadIdx.x; c < n0; c += blockDim.x) X[c] += S[0].E[c];
    __syncthreads();
  }
  double part = 0.0;
  for (int c = threadIdx.x; c < n0; c += blockDim.x) {
    out[c] = X[c];
    part += R0[c] * X[c];
  }
  if (rz_slot < 0) return;
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x + 63) / 64; ++w) s += sh[w];
    atomicAdd(&st->rz[rz_slot * kSlots], s);
  }
}

}  // namespace

hipError_t mg_setup(const MgHierarchy& h, hipStream_t s) {
  for (int l = 1; l < h.nlev; ++l) {
    const MgLevelDev& F = h.lev[l - 1];
    const MgLevelDev& C = h.lev[l];
    const dim3 grid((C.nx + kBX - 1) / kBX, (C.ny + kBY - 1) / kBY, C.nz);
    hipLaunchKernelGGL(k_mg_coarsen, grid, cell_block(), 0, s, F, C);
  }
  return hipGetLastError();
}

// z = M^{-1} r for the finest level (r = lev[0].b); with rz_slot >= 0 also
// accumulates r . z into the CG ring.
hipError_t mg_apply(const MgHierarchy& h, const double* r, double* z, PcgState* st, int rz_slot, hipStream_t s) {
  const int lc = h.lc;
  auto grid_of = [](const MgLevelDev& L) {
    return dim3((L.nx + kBX - 1) / kBX, (L.ny + kBY - 1) / kBY, L.nz);
  };
  // down the fine levels
  for (int l = 0; l < lc; ++l) {
    const MgLevelDev& F = h.lev[l];
    const MgLevelDev& C = h.lev[l + 1];
    const double* b = l == 0 ? r : F.b;
    hipLaunchKernelGGL(k_mg_smooth_down, grid_of(F), cell_block(), 0, s, F, b, F.x, st);
    hipLaunchKernelGGL(k_mg_restrict, grid_of(C), cell_block(), 0, s, F, C, b, F.x, C.b, st);
  }
  // coarse levels in LDS
  {
    const double* b = lc == 0 ? r : h.lev[lc].b;
    double* out = lc == 0 ? z : h.lev[lc].x;
    hipLaunchKernelGGL(k_mg_coarse_lds, dim3(1), dim3(h.coarse_threads), h.lds_bytes, s, h.coarse, b, out,
                       st, lc == 0 ? rz_slot : -1);
  }
  // up the fine levels
  for (int l = lc - 1; l >= 0; --l) {
    const MgLevelDev& F = h.lev[l];
    const MgLevelDev& C = h.lev[l + 1];
    const double* b = l == 0 ? r : F.b;
    double* out = l == 0 ? z : F.x;
    hipLaunchKernelGGL(k_mg_prolong_smooth, grid_of(F), cell_block(), 0, s, F, C, b, F.x, C.x, h.omega_c, F.y, st);
    hipLaunchKernelGGL(k_mg_smooth_final, grid_of(F), cell_block(), 0, s, F, b, F.y, out, st, l == 0 ? rz_slot : -1);
  }
  return hipGetLastError();
}

// The attribute belongs to the kernel, not to a context: keep the largest
// size any context asked for.
hipError_t mg_set_lds_limit(int bytes) {
  static int granted = 0;
  if (bytes <= granted) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_coarse_lds),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) granted = bytes;
  return e;
}

}  // namespace erem
