// Aggregation multigrid preconditioner for the TPFA pressure operator.
//
// Levels: cells aggregated 2 x 2 (x 2 in 3D).  With piecewise-constant
// prolongation P the Galerkin operator P^T A P of a two-point-flux matrix is
// again a two-point-flux matrix whose face transmissibility is the sum of the
// fine transmissibilities crossing the coarse face (Dirichlet faces included),
// so every level keeps the same face-array layout as the fine grid.
// Smoother: on the 2D grid levels three Jacobi-type sweeps weighted by the
// reciprocals of the Chebyshev points of [2/3, 2] (the degree-3 Chebyshev
// polynomial in D^-1 A, whose spectrum these diagonally dominant M-matrices
// keep inside (0, 2]); on the 3D grid levels and the LDS-resident levels two
// damped-Jacobi sweeps (omega 0.8); the same sweeps before and after the
// coarse correction, which is over-relaxed by omega_c.  The bottom level (at
// most kMgBottomCells cells) is solved exactly with a dense inverse formed
// once per setup.  The cycle is symmetric, so it is a valid
// conjugate-gradient preconditioner.  Each grid level runs two kernels: the
// down leg (sweeps from zero + restricted residual) and the up leg (coarse
// correction + sweeps), each recomputing its neighbours' intermediate sweeps
// on shrinking halos instead of waiting for a grid-wide pass; the levels with
// at most kMgLdsCells cells run inside one workgroup with everything in LDS.
#include "device.h"
#include "mg.h"

namespace erem {

namespace {

constexpr double kOmega = 0.8;

// Weights of the sweeps on the 2D grid levels: the reciprocals of the
// Chebyshev points of [lmax / 3, lmax] for lmax = 2 (the Gershgorin bound of
// D^-1 A for these operators), so the smoother is the degree-NU Chebyshev
// polynomial in D^-1 A.  Any order gives the same polynomial, so the cycle
// stays symmetric.
template <int NU>
__device__ inline double sweep_weight(int k) {
  const double lmax = 2.0, lmin = lmax / 3.0;
  const double z = 0.5 * (lmax + lmin) + 0.5 * (lmax - lmin) * cos(M_PI * (2 * k + 1) / (2.0 * NU));
  return 1.0 / z;
}

__device__ inline int fxi(int nx, int ny, int x, int y, int z) { return (z * ny + y) * (nx + 1) + x; }
__device__ inline int fyi(int nx, int ny, int x, int y, int z) { return (z * (ny + 1) + y) * nx + x; }
__device__ inline int fzi(int nx, int ny, int x, int y, int z) { return (z * ny + y) * nx + x; }

__device__ inline bool pcg_done(const PcgState* st) { return st && *(volatile const int*)&st->done; }


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
  const int z0 = fnz > 1 ? 2 * Z : 0;
  const int z1 = fnz > 1 ? min(2 * Z + 1, fnz - 1) : 0;
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
  if (fnz > 1) {
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

// Dense inverse of the bottom-level operator (SPD, diagonally dominant, so
// Gauss-Jordan without pivoting is stable), one workgroup of 1024 threads
// holding the matrix in registers (assembled in LDS).
static_assert(kMgBottomCells <= 64, "the bottom inverse maps 64 rows x 16 column groups of 4 onto 1024 threads");
__global__ __launch_bounds__(1024) void k_mg_bottom_inverse(MgLevelDev L, double* __restrict__ inv) {
  __shared__ double M[kMgBottomCells * kMgBottomCells];
  __shared__ double prow[2][kMgBottomCells];
  __shared__ double pcol[2][kMgBottomCells];
  const int n = L.nx * L.ny * L.nz;
  for (int j = threadIdx.x; j < n * n; j += blockDim.x) M[j] = 0.0;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
    // diagonal = sum of the cell's face transmissibilities (Dirichlet faces
    // included), formed here so that the finest level needs no other setup
    double dg = L.tx[fxi(L.nx, L.ny, x, y, z)] + L.tx[fxi(L.nx, L.ny, x + 1, y, z)] +
                L.ty[fyi(L.nx, L.ny, x, y, z)] + L.ty[fyi(L.nx, L.ny, x, y + 1, z)];
    if (L.nz > 1) dg += L.tz[fzi(L.nx, L.ny, x, y, z)] + L.tz[fzi(L.nx, L.ny, x, y, z + 1)];
    M[c * n + c] = dg;
    if (x > 0) M[c * n + c - 1] = -L.tx[fxi(L.nx, L.ny, x, y, z)];
    if (x + 1 < L.nx) M[c * n + c + 1] = -L.tx[fxi(L.nx, L.ny, x + 1, y, z)];
    if (y > 0) M[c * n + c - L.nx] = -L.ty[fyi(L.nx, L.ny, x, y, z)];
    if (y + 1 < L.ny) M[c * n + c + L.nx] = -L.ty[fyi(L.nx, L.ny, x, y + 1, z)];
    if (z > 0) M[c * n + c - L.nx * L.ny] = -L.tz[fzi(L.nx, L.ny, x, y, z)];
    if (z + 1 < L.nz) M[c * n + c + L.nx * L.ny] = -L.tz[fzi(L.nx, L.ny, x, y, z + 1)];
  }
  __syncthreads();
  // Gauss-Jordan in place, no pivoting (the operator is SPD).  Thread t keeps
  // row t / 16, columns 4 (t % 16) .. 4 (t % 16) + 3 in registers; the pivot
  // row and column go through LDS, double-buffered so that one barrier per
  // pivot suffices.  Rows and columns past n carry values that are never
  // stored, so the update runs without branches (selects only).
  const int t = threadIdx.x;
  const int i = t >> 4, j0 = (t & 15) * 4;
  double m[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) m[u] = (i < n && j0 + u < n) ? M[i * n + j0 + u] : 0.0;
  for (int k = 0; k < n; ++k) {
    const int b = k & 1;
    if (i == k) {
#pragma unroll
      for (int u = 0; u < 4; ++u) prow[b][j0 + u] = m[u];
    }
    if ((k >> 2) == (t & 15)) {
      const int u = k & 3;
      pcol[b][i] = u == 0 ? m[0] : u == 1 ? m[1] : u == 2 ? m[2] : m[3];
    }
    __syncthreads();
    const double piv = 1.0 / prow[b][k];
    const double ci = pcol[b][i];
    double rj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) rj[u] = prow[b][j0 + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      const double pr = j == k ? piv : rj[u] * piv;  // new pivot row
      const double upd = m[u] - ci * pr;
      m[u] = i == k ? pr : (j == k ? -ci * piv : upd);
    }
  }
  if (i < n) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + u < n) inv[i * n + j0 + u] = m[u];
  }
}

// Cell index and the neighbour sum of one level; the neighbour order (-x, +x,
// -y, +y, -z, +z) is the same everywhere, so fused and unfused forms of a
// sweep round identically.
__device__ inline int cidx(const MgLevelDev& L, int x, int y, int z) { return x + L.nx * (y + L.ny * z); }

template <class F>
__device__ inline double nb_sum(const MgLevelDev& L, int x, int y, int z, F&& v) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  double s = 0.0;
  if (x > 0) s += L.tx[fxi(nx, ny, x, y, z)] * v(x - 1, y, z);
  if (x + 1 < nx) s += L.tx[fxi(nx, ny, x + 1, y, z)] * v(x + 1, y, z);
  if (y > 0) s += L.ty[fyi(nx, ny, x, y, z)] * v(x, y - 1, z);
  if (y + 1 < ny) s += L.ty[fyi(nx, ny, x, y + 1, z)] * v(x, y + 1, z);
  if (z > 0) s += L.tz[fzi(nx, ny, x, y, z)] * v(x, y, z - 1);
  if (z + 1 < nz) s += L.tz[fzi(nx, ny, x, y, z + 1)] * v(x, y, z + 1);
  return s;
}

// Two damped-Jacobi sweeps from zero at one cell: x1 = w b / D,
// x2 = x1 + w (b - A x1) / D.
__device__ inline double sweep2_from_zero(const MgLevelDev& L, const double* __restrict__ b, int x, int y, int z) {
  auto x1 = [&](int xx, int yy, int zz) {
    const int j = cidx(L, xx, yy, zz);
    return kOmega * b[j] / L.diag[j];
  };
  const int i = cidx(L, x, y, z);
  const double D = L.diag[i];
  const double xi = kOmega * b[i] / D;
  return xi + kOmega * (b[i] - D * xi + nb_sum(L, x, y, z, x1)) / D;
}

// Down leg of one level, fused: the two pre-smoothing sweeps (x written for
// the up leg) and the restricted residual b - A x summed over each 2 x 2
// (x 2) aggregate.  One thread per fine cell of a column pair in z; the
// neighbours' sweeps are recomputed, so no grid-wide dependency remains.
// x pairs are adjacent lanes, y pairs adjacent rows of the 64 x 4 block.
__global__ __launch_bounds__(kThreads) void k_mg_down_restrict(MgLevelDev F, MgLevelDev C,
                                                     const double* __restrict__ b, double* __restrict__ xout,
                                                     double* __restrict__ bc, const PcgState* st) {
  if (pcg_done(st)) return;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int Z = blockIdx.z;
  const int z0 = F.nz > 1 ? 2 * Z : 0, z1 = F.nz > 1 ? min(2 * Z + 1, F.nz - 1) : 0;
  double acc = 0.0;
  if (x < F.nx && y < F.ny) {
    auto x2 = [&](int xx, int yy, int zz) { return sweep2_from_zero(F, b, xx, yy, zz); };
    for (int z = z0; z <= z1; ++z) {
      const int i = cidx(F, x, y, z);
      const double xi = x2(x, y, z);
      xout[i] = xi;
      acc += b[i] - F.diag[i] * xi + nb_sum(F, x, y, z, x2);
    }
  }
  acc += __shfl_xor(acc, 1, 64);
  __shared__ double sh[kBY][kBX];
  sh[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if ((threadIdx.x & 1) == 0 && (threadIdx.y & 1) == 0 && x < F.nx && y < F.ny) {
    const int X = x >> 1, Y = y >> 1;
    bc[X + C.nx * (Y + C.ny * Z)] = acc + sh[threadIdx.y + 1][threadIdx.x];
  }
}

// Up leg of one level, fused: coarse correction xc = x + omega_c e[parent],
// one damped-Jacobi sweep y = xc + w (b - A xc) / D, and the last sweep
// out = y + w (b - A y) / D, with the neighbours' y recomputed.  With
// rz_slot >= 0 (the finest level, b = r) also accumulates r . out into the
// CG ring slot.
__global__ __launch_bounds__(kThreads) void k_mg_up_smooth(MgLevelDev F, MgLevelDev C, const double* __restrict__ b,
                                                 const double* __restrict__ xv, const double* __restrict__ ec,
                                                 double omega_c, double* __restrict__ out, PcgState* st,
                                                 int rz_slot) {
  if (pcg_done(st)) return;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const int cz = F.nz > 1 ? 1 : 0;
  double part = 0.0;
  if (x < F.nx && y < F.ny) {
    auto xc = [&](int xx, int yy, int zz) {
      return xv[cidx(F, xx, yy, zz)] + omega_c * ec[(xx >> 1) + C.nx * ((yy >> 1) + C.ny * (zz >> cz))];
    };
    auto ys = [&](int xx, int yy, int zz) {
      const int j = cidx(F, xx, yy, zz);
      const double D = F.diag[j];
      const double v = xc(xx, yy, zz);
      return v + kOmega * (b[j] - D * v + nb_sum(F, xx, yy, zz, xc)) / D;
    };
    const int i = cidx(F, x, y, z);
    const double D = F.diag[i];
    const double yi = ys(x, y, z);
    const double v = yi + kOmega * (b[i] - D * yi + nb_sum(F, x, y, z, ys)) / D;
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
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);  // the block's band
    st->rz[rz_slot * st->nb + bid] = sh[0] + sh[1] + sh[2] + sh[3];
  }
}

// ---------------------------------------------------------------------------
// 2D forms of the two legs.  A block of 64 x 4 threads owns a tile of 64 x 8
// cells (two rows per thread, so each thread holds a whole y pair of
// aggregates).  Every global operand of the tile and its halo (two cells for
// the first sweep, one for the second) is loaded into LDS in one phase, so the
// chain of dependent memory latencies is a single one; the sweeps then run
// from LDS.  Same arithmetic, in the same order, as the generic forms above.
// ---------------------------------------------------------------------------
constexpr int kTY = 8;           // tile rows (two per thread)

// A 64 x kTY tile covers the 64 x 4 bands (bx, 2 by) and (bx, 2 by + 1) of
// the finest grid: its partial goes to the first, zero to the second.
__device__ inline void tile_band_store(double* slots, int nx, int ny, double v) {
  const int gx = (nx + kBX - 1) / kBX, gyb = (ny + kBY - 1) / kBY;
  const int b0 = blockIdx.x + gx * (2 * blockIdx.y);
  slots[b0] = v;
  if (2 * static_cast<int>(blockIdx.y) + 1 < gyb) slots[b0 + gx] = 0.0;
}

// Faces of the halo-H region: x faces of its rows (face gx of cell gx is its
// -x face) and y faces of its columns.
template <int H>
struct TileFacesH {
  double tx[kTY + 2 * H][kBX + 2 * H + 1];
  double ty[kTY + 2 * H + 1][kBX + 2 * H];
};
using TileFaces = TileFacesH<1>;

// Faces of a tile staged through registers: fetch issues every load (a
// fixed number per thread), store writes them to LDS, so the loads of all
// the tile's operands are in flight together instead of one loop trip after
// another.
template <int H>
struct FaceRegs {
  static constexpr int W = kBX + 2 * H, HH = kTY + 2 * H;
  static constexpr int NX = HH * (W + 1), NY = (HH + 1) * W;
  static constexpr int UX = (NX + kThreads - 1) / kThreads, UY = (NY + kThreads - 1) / kThreads;
  double tx[UX], ty[UY];
  __device__ inline void fetch(const MgLevelDev& L, int x0, int y0, int tid) {
    const int nx = L.nx, ny = L.ny;
#pragma unroll
    for (int u = 0; u < UX; ++u) {
      const int k = tid + u * kThreads;
      const int ly = k / (W + 1), lx = k - ly * (W + 1);
      const int gx = x0 - H + lx, gy = y0 - H + ly;
      tx[u] = (k < NX && gx >= 0 && gx <= nx && gy >= 0 && gy < ny) ? L.tx[fxi(nx, ny, gx, gy, 0)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UY; ++u) {
      const int k = tid + u * kThreads;
      const int ly = k / W, lx = k - ly * W;
      const int gx = x0 - H + lx, gy = y0 - H + ly;
      ty[u] = (k < NY && gx >= 0 && gx < nx && gy >= 0 && gy <= ny) ? L.ty[fyi(nx, ny, gx, gy, 0)] : 0.0;
    }
  }
  __device__ inline void store(TileFacesH<H>& F, int tid) const {
#pragma unroll
    for (int u = 0; u < UX; ++u) {
      const int k = tid + u * kThreads;
      if (k < NX) F.tx[k / (W + 1)][k % (W + 1)] = tx[u];
    }
#pragma unroll
    for (int u = 0; u < UY; ++u) {
      const int k = tid + u * kThreads;
      if (k < NY) F.ty[k / W][k % W] = ty[u];
    }
  }
};

// Neighbour sum of the halo-H cell (lx, ly) at (gx, gy), values v in a
// region whose element (sy, sx) is that cell.
template <int W, int H>
__device__ inline double nb_sum_tile(const TileFacesH<H>& F, int nx, int ny, int gx, int gy, int lx, int ly,
                                     const double (*v)[W], int sy, int sx) {
  double s = 0.0;
  if (gx > 0) s += F.tx[ly][lx] * v[sy][sx - 1];
  if (gx + 1 < nx) s += F.tx[ly][lx + 1] * v[sy][sx + 1];
  if (gy > 0) s += F.ty[ly][lx] * v[sy - 1][sx];
  if (gy + 1 < ny) s += F.ty[ly + 1][lx] * v[sy + 1][sx];
  return s;
}

// Tile arrays of the 2D legs: the 64 x 8 tile plus a halo of H cells.
template <int H>
struct Halo {
  static constexpr int W = kBX + 2 * H;
  static constexpr int R = kTY + 2 * H;
};

// One damped-Jacobi sweep, out = x + w (B - D x + sum t x_nb) / D, on the
// tile plus a halo of h (cells outside the grid get zero); arrays in
// halo-HA coordinates, faces of the halo-HF region (HF >= h, HA > h).
template <int HA, int HF>
__device__ inline void tile_sweep(int h, const TileFacesH<HF>& tf, const MgLevelDev& F, int x0, int y0, int tid,
                                  const double (*sb)[Halo<HA>::W], const double (*sd)[Halo<HA>::W],
                                  const double (*xin)[Halo<HA>::W], double (*xo)[Halo<HA>::W], double om) {
  constexpr int W = Halo<HA>::W;
  const int w = kBX + 2 * h, hh = kTY + 2 * h;
  for (int k = tid; k < w * hh; k += kThreads) {
    const int ry = k / w, rx = k - ry * w;
    const int ly = ry + HA - h, lx = rx + HA - h;
    const int gx = x0 - HA + lx, gy = y0 - HA + ly;
    double v = 0.0;
    if (gx >= 0 && gx < F.nx && gy >= 0 && gy < F.ny) {
      const double D = sd[ly][lx];
      const double xi = xin[ly][lx];
      v = xi + om * (sb[ly][lx] - D * xi +
                     nb_sum_tile<W>(tf, F.nx, F.ny, gx, gy, lx - (HA - HF), ly - (HA - HF), xin, ly, lx)) / D;
    }
    xo[ly][lx] = v;
  }
}

// Down leg of a 2D level, fused: NU damped-Jacobi sweeps from zero (the
// first, x1 = w B / D, needs no neighbours; sweep k runs on the tile plus a
// halo of NU - k + 1 so that the neighbours' values are recomputed instead of
// exchanged), then the restricted residual of the tile's aggregates.
//
// With CG, iteration it of Chronopoulos-Gear conjugate gradients (one
// reduction phase per iteration) is folded in front of the leg.  From the
// slot sums of the previous leg pair: the stop test on ||r_it||, then
// beta = g_it / g_{it-1}, alpha = g_it / (d_it - beta g_it / alpha_{it-1})
// with g = r.z, d = w.z, w = A z (alpha = g_0 / d_0, beta = 0 at it = 0);
// s = w + beta s_old and r_new = r - alpha s on the tile and its halo (the
// halo values recomputed, the tile's written); p = z + beta p and
// x += alpha p on the tile; the partial sums of r_new . r_new.
template <int NU, bool CG>
__global__ __launch_bounds__(kThreads) void k_mg_down_restrict_2d(MgLevelDev F, MgLevelDev C,
                                                        const double* __restrict__ b, double* __restrict__ xout,
                                                        double* __restrict__ bc, PcgState* st, CgFuse cg) {
  static_assert(NU >= 2, "two sweeps at least");
  constexpr int HA = NU;  // b, D (and the CG vectors) on the tile plus NU
  constexpr int W = Halo<HA>::W, R = Halo<HA>::R;
  const bool stop = pcg_done(st);
  __shared__ double sb[R][W], sd[R][W], sx[2][R][W];
  __shared__ double sw[CG ? R : 1][CG ? W : 1], ss[CG ? R : 1][CG ? W : 1];
  __shared__ double alpha_sh, beta_sh;
  __shared__ int stop_sh;
  __shared__ TileFacesH<NU - 1> tf;
  const int nx = F.nx, ny = F.ny;
  const int tile = xcd_tile_id();  // 2D grid: tile = bx + gridDim.x * by
  const int x0 = (tile % gridDim.x) * kBX, y0 = (tile / gridDim.x) * kTY;
  const int tid = threadIdx.x + threadIdx.y * kBX;
  const int it = cg.it;
  // every load of the tile is issued (into registers) before the first LDS
  // store: the cells' b, D (and w, s) on the tile plus NU, the faces, the
  // tile's own x, z, p
  constexpr int U = (R * W + kThreads - 1) / kThreads;
  double rb[U], rd[U], rw[CG ? U : 1], rs[CG ? U : 1];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = tid + u * kThreads;
    const int ly = k / W, lx = k - ly * W;
    const int gx = x0 - HA + lx, gy = y0 - HA + ly;
    const bool in = k < R * W && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int j = gx + nx * gy;
    rb[u] = in ? b[j] : 0.0;
    rd[u] = in ? F.diag[j] : 1.0;
    if (CG) {
      rw[u] = in ? cg.w[j] : 0.0;
      rs[u] = (in && it > 0) ? cg.s_old[j] : 0.0;
    }
  }
  FaceRegs<NU - 1> fr;
  fr.fetch(F, x0, y0, tid);
  // the tile's own cells (two rows per thread) for the p and x updates
  const int ox = x0 + threadIdx.x;
  double xo[2] = {0.0, 0.0}, po[2] = {0.0, 0.0}, zo[2] = {0.0, 0.0};
  if (CG) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int oy = y0 + 2 * threadIdx.y + r;
      if (ox < nx && oy < ny) {
        xo[r] = cg.x[ox + nx * oy];
        zo[r] = cg.z[ox + nx * oy];
        if (it > 0) po[r] = cg.p[ox + nx * oy];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = tid + u * kThreads;
    if (k >= R * W) continue;
    const int ly = k / W, lx = k - ly * W;
    sb[ly][lx] = rb[u];
    sd[ly][lx] = rd[u];
    if (CG) {
      sw[ly][lx] = rw[u];
      ss[ly][lx] = rs[u];
    } else {
      sx[0][ly][lx] = sweep_weight<NU>(0) * rb[u] / rd[u];  // first sweep from zero
    }
  }
  fr.store(tf, tid);
  if (CG && tid < 64) {  // the first wavefront decides for the block
    int halt = stop ? 1 : 0;
    double alpha = 0.0, beta = 0.0;
    const int nb = st->nb;
    const double rr = wave_part_sum(st->rr + (it & 3) * nb, nb);
    const double bb = wave_part_sum(st->bb_sl, nb);
    const double g1 = wave_part_sum(st->rz + (it & 3) * nb, nb);
    const double d1 = wave_part_sum(st->wz + (it & 3) * nb, nb);
    const double g0 = it > 0 ? wave_part_sum(st->rz + ((it - 1) & 3) * nb, nb) : 1.0;
    const bool lead = tile == 0;
    if (halt) {
      // an earlier iteration converged
    } else if (!isfinite(rr)) {
      halt = 1;
      if (lead && tid == 0) { st->nonfinite = 1; st->done = 1; st->it_done = it; }
    } else if (rr <= st->tol2 * bb) {
      halt = 1;
      if (lead && tid == 0) { st->done = 1; st->it_done = it; st->bb = bb; }
    } else if (it > 0) {
      beta = g1 / g0;
      alpha = g1 / (d1 - beta * g1 / st->alpha[(it - 1) & 3]);
    } else {
      alpha = g1 / d1;
    }
    if (tid == 0) {
      stop_sh = halt;
      alpha_sh = alpha;
      beta_sh = beta;
    }
    if (!halt && lead && tid == 0) st->alpha[it & 3] = alpha;
  }
  if (CG) {
    // block (0, 0) may set the stop flag while this kernel runs, so every
    // wavefront follows the first one's decision, not its own read
    __syncthreads();
    if (stop_sh) return;
    const double alpha = alpha_sh, beta = beta_sh;
    for (int k = tid; k < R * W; k += kThreads) {
      const int ly = k / W, lx = k - ly * W;
      const double sv = sw[ly][lx] + beta * ss[ly][lx];  // zero outside the grid stays zero
      const double rn = sb[ly][lx] - alpha * sv;
      ss[ly][lx] = sv;
      sb[ly][lx] = rn;
      sx[0][ly][lx] = sweep_weight<NU>(0) * rn / sd[ly][lx];  // first sweep from zero
    }
    __syncthreads();
    double rr = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int ly = 2 * threadIdx.y + r, oy = y0 + ly;
      if (ox < nx && oy < ny) {
        const int j = ox + nx * oy;
        const double rn = sb[ly + HA][threadIdx.x + HA];
        const double pn = zo[r] + beta * po[r];
        cg.r_new[j] = rn;
        cg.s_new[j] = ss[ly + HA][threadIdx.x + HA];
        cg.p[j] = pn;
        cg.x[j] = xo[r] + alpha * pn;
        rr += rn * rn;
      }
    }
    for (int off = 32; off > 0; off >>= 1) rr += __shfl_down(rr, off, 64);
    __shared__ double sh[kThreads / 64];
    if ((tid & 63) == 0) sh[tid >> 6] = rr;
    __syncthreads();
    if (tid == 0) tile_band_store(st->rr + ((it + 1) & 3) * st->nb, nx, ny, sh[0] + sh[1] + sh[2] + sh[3]);
  } else {
    if (stop) return;
    __syncthreads();
  }
#pragma unroll
  for (int k = 2; k <= NU; ++k) {
    tile_sweep<HA, NU - 1>(NU - k + 1, tf, F, x0, y0, tid, sb, sd, sx[(k - 2) & 1], sx[(k - 1) & 1],
                           sweep_weight<NU>(k - 1));
    __syncthreads();
  }
  const double(*fin)[W] = sx[(NU - 1) & 1];
  const int gx = x0 + threadIdx.x;
  double acc = 0.0;
  for (int r = 0; r < 2; ++r) {
    const int ly = 2 * threadIdx.y + r;
    const int gy = y0 + ly;
    if (gx < nx && gy < ny) {
      const int sy = ly + HA, sxx = threadIdx.x + HA;
      const double xi = fin[sy][sxx];
      xout[gx + nx * gy] = xi;
      acc += sb[sy][sxx] - sd[sy][sxx] * xi +
             nb_sum_tile<W>(tf, nx, ny, gx, gy, sxx - (HA - (NU - 1)), sy - (HA - (NU - 1)), fin, sy, sxx);
    }
  }
  acc += __shfl_xor(acc, 1, 64);
  const int gy = y0 + 2 * threadIdx.y;
  if ((threadIdx.x & 1) == 0 && gx < nx && gy < ny) bc[(gx >> 1) + C.nx * (gy >> 1)] = acc;
}

// Up leg of a 2D level, fused: the coarse correction v = x + w_c e[parent]
// on the tile plus a halo of HU, then NU damped-Jacobi sweeps on shrinking
// halos; the last lands on the tile (out = z) and, with rz_slot >= 0, b . z
// goes to the CG ring.  With CG (the finest level of the Chronopoulos-Gear
// form) every halo is one larger, so that the last sweep also covers the
// halo-one ring and w = A z follows on the tile (w_out); the partial sums of
// r.z and w.z go to the ring slot.
template <int NU, bool CG>
__global__ __launch_bounds__(kThreads) void k_mg_up_smooth_2d(MgLevelDev F, MgLevelDev C, const double* __restrict__ b,
                                                     const double* __restrict__ xv, const double* __restrict__ ec,
                                                     double omega_c, double* __restrict__ out,
                                                     double* __restrict__ w_out, PcgState* st, int rz_slot) {
  constexpr int HU = NU + (CG ? 1 : 0);
  constexpr int W = Halo<HU>::W, R = Halo<HU>::R;
  const bool stop = pcg_done(st);
  __shared__ double sxc[R][W], sb[R][W], sd[R][W], sy[2][R][W];
  __shared__ TileFacesH<HU - 1> tf;
  const int nx = F.nx, ny = F.ny;
  const int tile = xcd_tile_id();  // 2D grid: tile = bx + gridDim.x * by
  const int x0 = (tile % gridDim.x) * kBX, y0 = (tile / gridDim.x) * kTY;
  const int tid = threadIdx.x + threadIdx.y * kBX;
  // every load of the tile is issued (into registers) before the first LDS store
  constexpr int U = (R * W + kThreads - 1) / kThreads;
  double rx[U], re[U], rb[U], rd[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = tid + u * kThreads;
    const int ly = k / W, lx = k - ly * W;
    const int gx = x0 - HU + lx, gy = y0 - HU + ly;
    const bool in = k < R * W && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int j = gx + nx * gy;
    rx[u] = in ? xv[j] : 0.0;
    re[u] = in ? ec[(gx >> 1) + C.nx * (gy >> 1)] : 0.0;
    rb[u] = in ? b[j] : 0.0;
    rd[u] = in ? F.diag[j] : 1.0;
  }
  FaceRegs<HU - 1> fr;
  fr.fetch(F, x0, y0, tid);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = tid + u * kThreads;
    if (k >= R * W) continue;
    const int ly = k / W, lx = k - ly * W;
    const int gx = x0 - HU + lx, gy = y0 - HU + ly;
    const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    sxc[ly][lx] = in ? rx[u] + omega_c * re[u] : 0.0;
    sb[ly][lx] = rb[u];
    sd[ly][lx] = rd[u];
  }
  fr.store(tf, tid);
  if (stop) return;
  __syncthreads();
#pragma unroll
  for (int k = 1; k <= NU; ++k) {
    tile_sweep<HU, HU - 1>(HU - k, tf, F, x0, y0, tid, sb, sd, k == 1 ? sxc : sy[(k - 2) & 1], sy[(k - 1) & 1],
                           sweep_weight<NU>(NU - k));
    __syncthreads();
  }
  const double(*fin)[W] = sy[(NU - 1) & 1];
  const int gx = x0 + threadIdx.x;
  double g = 0.0, dz = 0.0;
  for (int r = 0; r < 2; ++r) {
    const int ly = 2 * threadIdx.y + r;
    const int gy = y0 + ly;
    if (gx < nx && gy < ny) {
      const int syy = ly + HU, sxx = threadIdx.x + HU;
      const double z = fin[syy][sxx];
      out[gx + nx * gy] = z;
      g += sb[syy][sxx] * z;
      if (CG) {
        const double w = sd[syy][sxx] * z - nb_sum_tile<W>(tf, nx, ny, gx, gy, sxx - 1, syy - 1, fin, syy, sxx);
        w_out[gx + nx * gy] = w;
        dz += w * z;
      }
    }
  }
  if (rz_slot < 0) return;
  for (int off = 32; off > 0; off >>= 1) {
    g += __shfl_down(g, off, 64);
    if (CG) dz += __shfl_down(dz, off, 64);
  }
  __shared__ double sh[2][kThreads / 64];
  if ((tid & 63) == 0) {
    sh[0][tid >> 6] = g;
    sh[1][tid >> 6] = dz;
  }
  __syncthreads();
  if (tid == 0) {
    tile_band_store(st->rz + rz_slot * st->nb, nx, ny, sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3]);
    if (CG) tile_band_store(st->wz + rz_slot * st->nb, nx, ny, sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
  }
}

// ---------------------------------------------------------------------------
// Coarse levels in one workgroup, everything in LDS: a.ncyc V-cycles over
// the levels first..bottom-1 with the exact dense solve on the bottom level,
// from x = 0, on rhs b (global).  Writes x to out; with rz_slot >= 0 also
// b . out into the CG ring.  LDS per smoothed level: faces, diagonal, its
// inverse and three vectors; bottom: two vectors, the partial products of
// the dense solve and the inverse.
// ---------------------------------------------------------------------------
struct LdsLevel {
  double *tx, *ty, *tz, *diag, *B, *E, *T, *dinv;
};

__device__ inline void lds_level(const MgCoarseArgs& a, double* smem, int l, LdsLevel& S) {
  S.tx = smem + a.off[l][0];
  S.ty = smem + a.off[l][1];
  S.tz = smem + a.off[l][2];
  S.diag = smem + a.off[l][3];
  S.B = smem + a.off[l][4];
  S.E = smem + a.off[l][5];
  S.T = smem + a.off[l][6];
  S.dinv = smem + a.off[l][7];
}

// (x, y, z) of cell c of a level
__device__ inline void cell_xyz(const MgLevelDev& L, int c, int& x, int& y, int& z) {
  if (L.nz == 1) {
    y = c / L.nx;
    x = c - y * L.nx;
    z = 0;
  } else {
    const int pl = L.nx * L.ny;
    z = c / pl;
    const int r = c - z * pl;
    y = r / L.nx;
    x = r - y * L.nx;
  }
}

// Neighbour sum of cell c of an LDS level with values v(j, x, y, z) of the
// neighbour j at (x, y, z).  Every face index is valid (boundary faces are
// stored); a missing neighbour is replaced by the cell itself and its term
// dropped by a select, so all loads issue without branches and wait once.
template <class V>
__device__ inline double lds_nb_sum(const MgLevelDev& L, const LdsLevel& S, int x, int y, int z, int c, V&& v) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const bool hw = x > 0, he = x + 1 < nx, hs = y > 0, hn = y + 1 < ny;
  const double tw = S.tx[fxi(nx, ny, x, y, z)], te = S.tx[fxi(nx, ny, x + 1, y, z)];
  const double ts = S.ty[fyi(nx, ny, x, y, z)], tn = S.ty[fyi(nx, ny, x, y + 1, z)];
  const double vw = v(hw ? c - 1 : c, hw ? x - 1 : x, y, z);
  const double ve = v(he ? c + 1 : c, he ? x + 1 : x, y, z);
  const double vs = v(hs ? c - nx : c, x, hs ? y - 1 : y, z);
  const double vn = v(hn ? c + nx : c, x, hn ? y + 1 : y, z);
  double s = (hw ? tw * vw : 0.0) + (he ? te * ve : 0.0) + (hs ? ts * vs : 0.0) + (hn ? tn * vn : 0.0);
  if (nz > 1) {  // uniform: 2D levels keep no z faces in LDS
    const bool hb = z > 0, ht = z + 1 < nz;
    const double tb = S.tz[fzi(nx, ny, x, y, z)], tt = S.tz[fzi(nx, ny, x, y, z + 1)];
    const double vb = v(hb ? c - nx * ny : c, x, y, hb ? z - 1 : z);
    const double vt = v(ht ? c + nx * ny : c, x, y, ht ? z + 1 : z);
    s += (hb ? tb * vb : 0.0) + (ht ? tt * vt : 0.0);
  }
  return s;
}

// One smoothed level's faces and diagonal (and 1/diagonal) into LDS, every
// load issued before the first store.  Two face values and one diagonal
// value per thread cover the level: it has at most blockDim cells and at
// most twice as many faces per direction.
__device__ inline void lds_load_level(const MgLevelDev& L, const LdsLevel& S) {
  const int bd = blockDim.x, t = threadIdx.x;
  const int n = L.nx * L.ny * L.nz;
  const int nfx = (L.nx + 1) * L.ny * L.nz, nfy = L.nx * (L.ny + 1) * L.nz;
  const int nfz = L.nz > 1 ? L.nx * L.ny * (L.nz + 1) : 0;  // 2D: z faces never read
  double fx[2], fy[2], fz[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = t + u * bd;
    fx[u] = j < nfx ? L.tx[j] : 0.0;
    fy[u] = j < nfy ? L.ty[j] : 0.0;
    fz[u] = j < nfz ? L.tz[j] : 0.0;
  }
  const double dg = t < n ? L.diag[t] : 1.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = t + u * bd;
    if (j < nfx) S.tx[j] = fx[u];
    if (j < nfy) S.ty[j] = fy[u];
    if (j < nfz) S.tz[j] = fz[u];
  }
  if (t < n) {
    S.diag[t] = dg;
    S.dinv[t] = 1.0 / dg;  // the sweeps multiply; one division per cell here
  }
}

// Phases of the LDS levels; each ends with a barrier.
// Down leg of level l: two damped-Jacobi sweeps from zero in one pass (E = x2,
// the first sweep's x1 = w B / D recomputed at the neighbours), then the
// restricted residual into the B of level l + 1: the sum over the (up to)
// 2 x 2 (x 2) fine cells of each coarse cell, a fine index past the edge
// clamped and its term dropped.
// One damped-Jacobi sweep of an LDS level from xin into xo (different arrays).
__device__ inline void lds_sweep(const MgLevelDev& F, const LdsLevel& S, const double* xin, double* xo) {
  const int bd = blockDim.x, t = threadIdx.x;
  const int n = F.nx * F.ny * F.nz;
  auto xv = [&](int j, int, int, int) { return xin[j]; };
  for (int c = t; c < n; c += bd) {
    int x, y, z;
    cell_xyz(F, c, x, y, z);
    const double di = S.dinv[c];
    const double v = xin[c];
    xo[c] = v + kOmega * ((S.B[c] + lds_nb_sum(F, S, x, y, z, c, xv)) * di - v);
  }
  __syncthreads();
}

__device__ inline void lds_down(const MgCoarseArgs& a, double* smem, int l) {
  const int bd = blockDim.x, t = threadIdx.x;
  const MgLevelDev& F = a.lev[l];
  const MgLevelDev& C = a.lev[l + 1];
  LdsLevel S, SC;
  lds_level(a, smem, l, S);
  lds_level(a, smem, l + 1, SC);
  {
    const int n = F.nx * F.ny * F.nz;
    auto x1 = [&](int j, int, int, int) { return kOmega * S.B[j] * S.dinv[j]; };
    for (int c = t; c < n; c += bd) {
      int x, y, z;
      cell_xyz(F, c, x, y, z);
      const double di = S.dinv[c];
      const double bi = S.B[c];
      const double xi = kOmega * bi * di;
      S.E[c] = xi + kOmega * ((bi + lds_nb_sum(F, S, x, y, z, c, x1)) * di - xi);
    }
    __syncthreads();
  }
  for (int k = 2; k < kMgLdsSweeps; k += 2) {  // further sweeps in pairs, ending in E
    lds_sweep(F, S, S.E, S.T);
    lds_sweep(F, S, S.T, S.E);
  }
  const int nc = C.nx * C.ny * C.nz;
  auto ev = [&](int j, int, int, int) { return S.E[j]; };
  auto res = [&](int x, int y, int z) {
    const int i = x + F.nx * (y + F.ny * z);
    return S.B[i] - S.diag[i] * S.E[i] + lds_nb_sum(F, S, x, y, z, i, ev);
  };
  for (int c = t; c < nc; c += bd) {
    int X0, Y0, Z0;
    cell_xyz(C, c, X0, Y0, Z0);
    const int x0 = 2 * X0, y0 = 2 * Y0;
    const bool hx = x0 + 1 < F.nx, hy = y0 + 1 < F.ny;
    const int x1 = hx ? x0 + 1 : x0, y1 = hy ? y0 + 1 : y0;
    double acc;
    if (F.nz > 1) {
      const int z0 = 2 * Z0;
      const bool hz = z0 + 1 < F.nz;
      const int z1 = hz ? z0 + 1 : z0;
      const double r000 = res(x0, y0, z0), r100 = res(x1, y0, z0), r010 = res(x0, y1, z0), r110 = res(x1, y1, z0);
      const double r001 = res(x0, y0, z1), r101 = res(x1, y0, z1), r011 = res(x0, y1, z1), r111 = res(x1, y1, z1);
      acc = r000 + (hx ? r100 : 0.0) + (hy ? r010 : 0.0) + (hx && hy ? r110 : 0.0);
      if (hz) acc += r001 + (hx ? r101 : 0.0) + (hy ? r011 : 0.0) + (hx && hy ? r111 : 0.0);
    } else {
      const double r00 = res(x0, y0, 0), r10 = res(x1, y0, 0), r01 = res(x0, y1, 0), r11 = res(x1, y1, 0);
      acc = r00 + (hx ? r10 : 0.0) + (hy ? r01 : 0.0) + (hx && hy ? r11 : 0.0);
    }
    SC.B[c] = acc;
  }
  __syncthreads();
}

// Up leg of level l: coarse correction folded into the first sweep,
// T = y(E + w_c e[parent]), then E = T + w (B - A T) / D.
__device__ inline void lds_up(const MgCoarseArgs& a, double* smem, int l) {
  const int bd = blockDim.x, t = threadIdx.x;
  const MgLevelDev& F = a.lev[l];
  const MgLevelDev& C = a.lev[l + 1];
  LdsLevel S, SC;
  lds_level(a, smem, l, S);
  lds_level(a, smem, l + 1, SC);
  const int n = F.nx * F.ny * F.nz;
  const int cz = F.nz > 1 ? 1 : 0;
  auto xc = [&](int j, int x, int y, int z) {
    return S.E[j] + a.omega_c * SC.E[(x >> 1) + C.nx * ((y >> 1) + C.ny * (z >> cz))];
  };
  for (int c = t; c < n; c += bd) {
    int x, y, z;
    cell_xyz(F, c, x, y, z);
    const double di = S.dinv[c];
    const double v = xc(c, x, y, z);
    S.T[c] = v + kOmega * ((S.B[c] + lds_nb_sum(F, S, x, y, z, c, xc)) * di - v);
  }
  __syncthreads();
  lds_sweep(F, S, S.T, S.E);
  for (int k = 2; k < kMgLdsSweeps; k += 2) {  // further sweeps in pairs, ending in E
    lds_sweep(F, S, S.E, S.T);
    lds_sweep(F, S, S.T, S.E);
  }
}

// Bottom: E = inverse * B, the columns split over the wavefronts (partial
// products in T), then summed per row.  The inverse of the symmetric bottom
// operator is symmetric: it is read by columns so that consecutive threads
// hit consecutive banks.
__device__ inline void lds_bottom(const MgCoarseArgs& a, double* smem, const double* Binv, int nb) {
  const int bd = blockDim.x, t = threadIdx.x;
  LdsLevel S;
  lds_level(a, smem, a.nlev - 1, S);
  const int groups = (bd + 63) >> 6;
  const int chunk = (nb + groups - 1) / groups;
  const int r = t & 63, g = t >> 6;
  if (r < nb) {
    const int j0 = g * chunk, j1 = min(nb, j0 + chunk);
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) acc += Binv[j * nb + r] * S.B[j];
    S.T[g * nb + r] = acc;
  }
  __syncthreads();
  if (t < nb) {
    double acc = 0.0;
    for (int k = 0; k < groups; ++k) acc += S.T[k * nb + t];
    S.E[t] = acc;
  }
  __syncthreads();
}

// Residual of level l for the correction so far: B <- B - A E (in place: a
// cell writes only its own B, the neighbours' E are only read).  Thread t
// owns cell t (the level has at most blockDim cells); returns E of that cell.
__device__ inline double lds_residual(const MgCoarseArgs& a, double* smem, int l) {
  const int t = threadIdx.x;
  const MgLevelDev& F = a.lev[l];
  LdsLevel S;
  lds_level(a, smem, l, S);
  const int n = F.nx * F.ny * F.nz;
  double e = 0.0;
  if (t < n) {
    auto ev = [&](int j, int, int, int) { return S.E[j]; };
    int x, y, z;
    cell_xyz(F, t, x, y, z);
    e = S.E[t];
    S.B[t] += lds_nb_sum(F, S, x, y, z, t, ev) - S.diag[t] * e;
  }
  __syncthreads();
  return e;
}

// Coarse levels in one workgroup, everything in LDS: a.ncyc cycles on the
// first level; inside each, the coarse problem of the second level is solved
// by a.ncyc1 V-cycles over the levels below it (a W-shaped cycle with two
// visits under the first level), with the exact dense solve on the bottom
// level.  Later cycles on a level start from the residual the earlier ones
// left, and the corrections add up.  From x = 0, on rhs b (global); writes x
// to out; with rz_slot >= 0 also b . out into the CG ring.
__global__ __launch_bounds__(1024) void k_mg_coarse_lds(MgCoarseArgs a, const double* __restrict__ bglob,
                                              const double* __restrict__ binv, double* __restrict__ out,
                                              PcgState* st, int rz_slot) {
  const bool stop = pcg_done(st);  // checked once the level loads are in flight
  extern __shared__ double smem[];
  const int nl = a.nlev;          // levels in LDS, the last one is the bottom
  const int bd = blockDim.x, t = threadIdx.x;
  LdsLevel S0;
  lds_level(a, smem, 0, S0);
  const int n0 = a.n0;
  const double b0 = t < n0 ? bglob[t] : 0.0;
  // faces / diagonals of the smoothed levels, the bottom inverse, the rhs
  for (int l = 0; l + 1 < nl; ++l) {
    LdsLevel S;
    lds_level(a, smem, l, S);
    lds_load_level(a.lev[l], S);
  }
  const MgLevelDev& Lb = a.lev[nl - 1];
  const int nb = Lb.nx * Lb.ny * Lb.nz;
  double* Binv = smem + a.inv_off;
  for (int j0 = 0; j0 < nb * nb; j0 += 4 * bd) {
    double r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + t + u * bd;
      r[u] = j < nb * nb ? binv[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + t + u * bd;
      if (j < nb * nb) Binv[j] = r[u];
    }
  }
  if (t < n0) S0.B[t] = b0;
  if (stop) return;
  __syncthreads();
  double x0 = 0.0;  // accumulated correction of the first level, cell t
  for (int cyc = 0; cyc < a.ncyc; ++cyc) {
    if (cyc > 0) x0 += lds_residual(a, smem, 0);
    if (nl == 1) {
      lds_bottom(a, smem, Binv, nb);
      continue;
    }
    lds_down(a, smem, 0);
    double x1 = 0.0;  // accumulated correction of the second level, cell t
    for (int c1 = 0; c1 < a.ncyc1; ++c1) {
      if (c1 > 0) x1 += lds_residual(a, smem, 1);
      for (int l = 1; l + 1 < nl; ++l) lds_down(a, smem, l);
      lds_bottom(a, smem, Binv, nb);
      for (int l = nl - 2; l >= 1; --l) lds_up(a, smem, l);
    }
    if (a.ncyc1 > 1) {
      LdsLevel S1;
      lds_level(a, smem, 1, S1);
      const MgLevelDev& L1 = a.lev[1];
      if (t < L1.nx * L1.ny * L1.nz) S1.E[t] += x1;
      __syncthreads();
    }
    lds_up(a, smem, 0);
  }
  double part = 0.0;
  if (t < n0) {
    const double v = x0 + S0.E[t];
    out[t] = v;
    part = b0 * v;
  }
  if (rz_slot < 0) return;
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  __shared__ double sh[16];
  if ((t & 63) == 0) sh[t >> 6] = part;
  __syncthreads();
  // the whole grid is this workgroup's: its sum in the first band's slot,
  // zeros in the others
  double* slots = st->rz + rz_slot * st->nb;
  for (int k = t + 1; k < st->nb; k += bd) slots[k] = 0.0;
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < (bd + 63) / 64; ++w) s += sh[w];
    slots[0] = s;
  }
}

}  // namespace

hipError_t mg_setup(const MgHierarchy& h, hipStream_t s) {
  for (int l = 1; l <= h.lb; ++l) {
    const MgLevelDev& F = h.lev[l - 1];
    const MgLevelDev& C = h.lev[l];
    const dim3 grid((C.nx + kBX - 1) / kBX, (C.ny + kBY - 1) / kBY, C.nz);
    hipLaunchKernelGGL(k_mg_coarsen, grid, cell_block(), 0, s, F, C);
  }
  hipLaunchKernelGGL(k_mg_bottom_inverse, dim3(1), dim3(1024), 0, s, h.lev[h.lb], h.binv);
  return hipGetLastError();
}

// z = M^{-1} r on the finest level; with rz_slot >= 0 also accumulates r . z
// into the CG ring.
hipError_t mg_apply(const MgHierarchy& h, const double* r, double* z, PcgState* st, int rz_slot, hipStream_t s,
                    const CgFuse* cg) {
  if (cg && !mg_fuses_cg(h)) return hipErrorInvalidValue;
  const int lc = h.lc;
  auto grid_of = [](const MgLevelDev& L) {
    return dim3((L.nx + kBX - 1) / kBX, (L.ny + kBY - 1) / kBY, L.nz);
  };
  for (int l = 0; l < lc; ++l) {
    const MgLevelDev& F = h.lev[l];
    const MgLevelDev& C = h.lev[l + 1];
    const double* b = l == 0 ? r : F.b;
    if (F.nz == 1) {
      const dim3 g((F.nx + kBX - 1) / kBX, (F.ny + kTY - 1) / kTY, 1);
      if (l == 0 && cg && cg->update)
        hipLaunchKernelGGL((k_mg_down_restrict_2d<kMgSweeps, true>), g, cell_block(), 0, s, F, C, b, F.x, C.b, st,
                           *cg);
      else
        hipLaunchKernelGGL((k_mg_down_restrict_2d<kMgSweeps, false>), g, cell_block(), 0, s, F, C, b, F.x, C.b, st,
                           CgFuse{});
    } else {
      const dim3 g((F.nx + kBX - 1) / kBX, (F.ny + kBY - 1) / kBY, C.nz);
      hipLaunchKernelGGL(k_mg_down_restrict, g, cell_block(), 0, s, F, C, b, F.x, C.b, st);
    }
  }
  {
    const double* b = lc == 0 ? r : h.lev[lc].b;
    double* out = lc == 0 ? z : h.lev[lc].x;
    hipLaunchKernelGGL(k_mg_coarse_lds, dim3(1), dim3(h.coarse_threads), h.lds_bytes, s, h.coarse, b, h.binv,
                       out, st, lc == 0 ? rz_slot : -1);
  }
  // The up leg reads its level's x at the neighbours, so it writes its result
  // to y (z on the finest level); the LDS solve leaves its result in x.
  for (int l = lc - 1; l >= 0; --l) {
    const MgLevelDev& F = h.lev[l];
    const MgLevelDev& C = h.lev[l + 1];
    const double* b = l == 0 ? (cg && cg->update ? cg->r_new : r) : F.b;
    const double* ec = l + 1 == lc ? C.x : C.y;
    double* out = l == 0 ? z : F.y;
    if (F.nz == 1) {
      const dim3 g((F.nx + kBX - 1) / kBX, (F.ny + kTY - 1) / kTY, 1);
      if (l == 0 && cg)
        hipLaunchKernelGGL((k_mg_up_smooth_2d<kMgSweeps, true>), g, cell_block(), 0, s, F, C, b, F.x, ec, h.omega_c,
                           out, cg->w_out, st, rz_slot);
      else
        hipLaunchKernelGGL((k_mg_up_smooth_2d<kMgSweeps, false>), g, cell_block(), 0, s, F, C, b, F.x, ec, h.omega_c,
                           out, nullptr, st, l == 0 ? rz_slot : -1);
    } else {
      hipLaunchKernelGGL(k_mg_up_smooth, grid_of(F), cell_block(), 0, s, F, C, b, F.x, ec, h.omega_c, out, st,
                         l == 0 ? rz_slot : -1);
    }
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
