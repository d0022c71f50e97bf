// Shared declarations of the EREM device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

namespace erem {

constexpr int kBX = 64;        // threads along x per block (one wavefront)
constexpr int kBY = 4;         // rows per block -> 256 threads, 4 wavefronts
constexpr int kThreads = kBX * kBY;
constexpr int kSlots = 64;     // spread of the atomic min / max targets (AsmReduce)
constexpr int kMaxTerms = 1024;  // Leja degree cap per substep
// Widest substep interval h (beta - alpha) / s of the FP32 Newton passes: the
// terms grow to about e^(rho/10) times the result before they cancel, and in
// FP32 that growth is lost accuracy.
constexpr double kMixedRhoMax = 32.0;

struct Dims {
  int nx, ny, nz;      // cells
  int dim;             // 2 or 3
  int N;               // nx*ny*nz
  double dx, dy, dz;
};

struct Phys {
  int law;             // 0 constant, 1 water laws
  int dirichlet_left;  // conduction half-cell on x = 0
  double c_f, mu0, rho0, lam, rhoc_s;
  double p_left, p_right, T_left, T_right;
};

// Per-evaluation Leja coefficients (device resident).
struct LejaCoef {
  double inv_g;                 // 1 / gamma
  double thresh;                // 10^-p
  double shift[kMaxTerms + 1];  // c/gamma + xi_{k-1} for term k
  double dk[kMaxTerms + 1];     // divided differences d_k
  double estf[kMaxTerms + 1];   // |delta d_k| / (sqrt(N) scal)
};

// Per-substep Leja stop state (device resident).
struct LejaState {
  int stopped;     // -1 running, else the term at which the stop test passed
  int nonfinite;
  int checked;     // last term whose sum is final
  int pad;
  double sums[kMaxTerms + 1];  // sum q_k^2 (FP64)
};

// Divided differences of phi1 last formed on the device, with their key
// (the scaled interval centre hc, half-width hg and how many were formed):
// an evaluation with the same key reuses them.
struct DdCache {
  double hc, hg;
  int n, pad;
  double d[kMaxTerms + 1];
};

// Reduction targets of the assembly pass (ordered-integer encodings), one
// partial per slot: the blocks spread their atomics over kSlots addresses
// and the host folds the slots (slot_min / slot_max).
struct AsmReduce {
  unsigned long long lo[kSlots];    // min_i (J_ii - R_i)
  unsigned long long hi[kSlots];    // max_i (J_ii + R_i)
  unsigned long long tmax[kSlots];  // max_i |T_i|
  unsigned long long vmax[kSlots];  // max_i |v_i| (phi1_apply)
};

// Conjugate-gradient scalars.  The inner products are kept as partial sums,
// one per 64 x 4 cell band of the grid (the blocks of cell_grid), in a ring
// of four iterations: each band's slot is written by the block or tile that
// covers it (a tile of several bands writes its sum into its first band and
// zeros into the others), and every consumer sums the slots in band order
// (wave_part_sum), so the result does not depend on the order in which the
// blocks ran.  The arrays live in one device allocation of
// pcg_parts_words(nb) doubles.
struct PcgState {
  int done;        // 1 once converged
  int it_done;     // iteration count at convergence
  int nonfinite;
  int nb;          // partial slots per inner product (bands of the grid)
  double bb;       // ||b||^2 (reduced by the start kernel)
  double tol2;     // rtol^2
  double alpha[4];        // step lengths (Chronopoulos-Gear form)
  double* bb_sl;          // [nb]
  double* rz;             // [4][nb]
  double* rr;             // [4][nb]
  double* pq;             // [4][nb]
  double* wz;             // [4][nb] w.z (Chronopoulos-Gear form)
};
inline size_t pcg_parts_words(int nb) { return static_cast<size_t>(17) * nb; }
// The state's array pointers into a parts allocation of pcg_parts_words(nb).
inline void pcg_bind_parts(PcgState* st, double* parts, int nb) {
  st->nb = nb;
  st->bb_sl = parts;
  st->rz = parts + nb;
  st->rr = parts + 5 * static_cast<size_t>(nb);
  st->pq = parts + 9 * static_cast<size_t>(nb);
  st->wz = parts + 13 * static_cast<size_t>(nb);
}

inline dim3 cell_grid(const Dims& d) {
  return dim3((d.nx + kBX - 1) / kBX, (d.ny + kBY - 1) / kBY, d.nz);
}
// Number of 64 x 4 cell bands (the blocks of cell_grid).
inline int cell_bands(const Dims& d) {
  const dim3 g = cell_grid(d);
  return static_cast<int>(g.x * g.y * g.z);
}
inline dim3 cell_block() { return dim3(kBX, kBY, 1); }

// Host launchers (kernels.hip).  All enqueue on `s` and return hipGetLastError().
hipError_t launch_transmissibility(const Dims& d, const Phys& ph, const double* logk,
                                   const double* T, double* tx, double* ty, double* tz,
                                   hipStream_t s);
hipError_t launch_face_fluxes(const Dims& d, const Phys& ph, const double* p, const double* tx,
                              const double* ty, const double* tz, double* fx, double* fy,
                              double* fz, hipStream_t s);
hipError_t launch_reset_reduce(AsmReduce* r, hipStream_t s);
hipError_t launch_assemble(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                           const double* fy, const double* fz, const double* T, double* coef,
                           double* F, AsmReduce* red, hipStream_t s);
hipError_t launch_absmax(const Dims& d, const double* v, AsmReduce* red, hipStream_t s);
hipError_t launch_gershgorin(const Dims& d, const double* coef, AsmReduce* red, hipStream_t s);
// w = v + tg g + J u (g null: w = v + J u)
hipError_t launch_stencil_axpy(const Dims& d, const double* coef, const double* v,
                               const double* u, double* w, hipStream_t s,
                               const double* g = nullptr, double tg = 0.0);
// J_p stencil, G4 over G2 (in place), Gershgorin interval and max |p| of the
// transient pressure ODE at (T, p) with the current faces
hipError_t launch_pressure_ode(const Dims& d, const Phys& ph, const double* poro, const double* T, const double* p,
                               const double* tx, const double* ty, const double* tz, double alpha_b, double beta_f,
                               double* coef, double* G, AsmReduce* red, hipStream_t s);
// Gt = D_t G for boundary temperature rates dTl (x = 0) and dTr (x = nx)
hipError_t launch_time_rate(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                            const double* T, double dTl, double dTr, double* Gt, hipStream_t s);
hipError_t launch_axpby(const Dims& d, double* y, double a, const double* x, double b,
                        hipStream_t s);
hipError_t launch_pcg_reset(PcgState* st, double tol2, hipStream_t s);
hipError_t launch_pcg_start(const Dims& d, const Phys& ph, const double* tx, const double* ty,
                            const double* tz, const double* x, double* r, double* z, double* p0,
                            double* diag, PcgState* st, hipStream_t s);
hipError_t launch_pcg_start_rhs(const Dims& d, const double* tx, const double* ty, const double* tz,
                                const double* rhs, double* x, double* r, double* z, double* p0,
                                double* diag, PcgState* st, int jacobi, hipStream_t s);
hipError_t launch_dd_residual(const Dims& d, const Phys& ph, const double* tx, const double* ty,
                              const double* tz, const double* phi, const double* plo, double* r,
                              PcgState* st, hipStream_t s);
hipError_t launch_dd_update(const Dims& d, double* phi, double* plo, const double* delta,
                            hipStream_t s);
// Extrapolated warm start: prev <- p; with extrapolate, p <- 2 p - prev_old.
hipError_t launch_pressure_extrapolate(const Dims& d, double* phi, double* plo, double* prev, int extrapolate,
                                      hipStream_t s);
hipError_t launch_face_fluxes_dd(const Dims& d, const Phys& ph, const double* phi,
                                 const double* plo, const double* tx, const double* ty,
                                 const double* tz, double* fx, double* fy, double* fz,
                                 hipStream_t s);
hipError_t launch_pcg_a(const Dims& d, const double* tx, const double* ty, const double* tz,
                        const double* z, const double* pold, double* pnew, double* q,
                        PcgState* st, int it, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_pcg_b(const Dims& d, double* x, double* r, double* z, const double* pnew,
                        const double* q, const double* diag, PcgState* st, int it,
                        int jacobi, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Tile index of this block for grids whose neighbouring tiles share data:
// the hardware deals consecutive workgroups to the eight XCDs in turn
// (workgroup b to XCD b % 8), so tiles are handed out so that each XCD takes
// one contiguous range of them (x fastest), and the halos of a tile's
// neighbours are mostly in the same XCD's L2.  A bijection of the block
// index; only the placement changes.
#ifndef EREM_XCD_REMAP
#define EREM_XCD_REMAP 1
#endif
constexpr int kXcds = 8;
__device__ inline int xcd_tile_id() {
  const int nbk = gridDim.x * gridDim.y * gridDim.z;
  const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (!EREM_XCD_REMAP) return b;
  const int q = nbk / kXcds, r = nbk % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Launch; with events (sampled timing) they record the kernel's own start
// and stop, without the queue's gaps around it.
template <typename K, typename... A>
inline void launch_timed(K kernel, dim3 grid, dim3 block, unsigned shmem, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, A... args) {
  if (e0)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Sum of n partials at base in a fixed order, by one wavefront: lane l adds
// base[l], base[l + 64], ... in turn, a shuffle tree adds the lanes, and lane
// 0's result is broadcast so that every lane takes the same decisions.  The
// loads go sixteen at a time (a lane's share of 1024 partials is one memory
// latency), and are added in order after they arrive.
__device__ inline double wave_part_sum(const double* __restrict__ base, int n) {
  constexpr int kBatch = 16;
  const int lane = __lane_id();
  double s = 0.0;
  for (int k = lane; k < n; k += kBatch * 64) {
    double v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = k + j * 64 < n ? base[k + j * 64] : 0.0;
#pragma unroll
    for (int j = 0; j < kBatch; ++j) s += v[j];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return __shfl(s, 0, 64);
}

// Ordered encoding of doubles for atomic min/max on 64-bit unsigned integers.
__host__ __device__ inline unsigned long long ord_encode(double v) {
  union { double d; unsigned long long u; } c;
  c.d = v;
  return (c.u >> 63) ? ~c.u : (c.u | 0x8000000000000000ull);
}
__host__ __device__ inline double ord_decode(unsigned long long k) {
  union { double d; unsigned long long u; } c;
  c.u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return c.d;
}

// The encodings order like the values: fold the slots of one target.
inline double slot_min(const unsigned long long* v) {
  unsigned long long m = v[0];
  for (int k = 1; k < kSlots; ++k) m = v[k] < m ? v[k] : m;
  return ord_decode(m);
}
inline double slot_max(const unsigned long long* v) {
  unsigned long long m = v[0];
  for (int k = 1; k < kSlots; ++k) m = v[k] > m ? v[k] : m;
  return ord_decode(m);
}

}  // namespace erem
