// Batched EREM over many independent linear problems (batch.hip): shared
// structures and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

// Tile shapes of the work kernel: 64 x kBatchTileRows[shape] cells on 64 x
// kBatchThreadRows[shape] threads, kBatchPassTerms[shape] Newton terms per
// pass; shapes 2-7 place the tiles so that each XCD takes a contiguous range
// of them.
constexpr int kNumTileShapes = 8;
constexpr int kBatchTileRows[kNumTileShapes] = {8, 16, 8, 16, 32, 16, 8, 32};
constexpr int kBatchThreadRows[kNumTileShapes] = {8, 16, 8, 8, 8, 8, 8, 8};
constexpr int kBatchPassTerms[kNumTileShapes] = {4, 4, 4, 4, 4, 8, 8, 8};
constexpr int kBatchTileX = 64;
constexpr int kBatchPartStride = 8;  // partials per tile (one per term of a pass)

// Static description of one problem of the batch.
struct BProb {
  int nx, ny;
  int s;          // substeps per step
  int coef_off;   // first divided difference / shift of this problem
  long long off;  // first cell in the packed vectors
  double inv_g;   // 1 / gamma
  double delta;   // substep length h / s
  double rootN;   // sqrt(nx ny)
  int tile0;      // first tile of the problem in the tile list
  int ntiles;     // its tiles (tiles_x rows of 64 x rows cells)
  int tiles_x;
  int pad;
};

// Tile list entry: the problem and the tile's first cell.
struct BTile {
  int pid, x0, y0;
  int done;  // set by the control kernel once the problem is done: the tile returns at entry
};

// Phases of a problem; every work launch advances each problem that is not
// done by one phase, and the control kernel that follows picks the next.
enum BPhase : int {
  kPhInit = 0,    // start of a substep: q_0, p = d_0 q_0 (and the end of the previous substep or step)
  kPhTerms = 1,   // Newton terms k .. k + nt - 1
  kPhFinish = 2,  // the last step's T update
  kPhDone = 3,
};

// Kinds of start pass.
enum BInit : int {
  kInitFirst = 0,  // first step: T^0 as given
  kInitSub = 1,    // substep j >= 1: u += delta p of substep j - 1
  kInitStep = 2,   // next step: T += u + delta p of the last substep
};

// Dynamic state of one problem, written only by the control kernel.
struct BState {
  int phase, kind;
  int step;   // steps completed
  int sub;    // current substep
  int k;      // first term of the next pass
  int terms;  // Newton terms applied
  int flags;  // 1: no convergence within m_max, 2: non-finite norm
  int tpar;   // buffer holding T^n: 0 the caller's array, 1 the internal copy
  int upar;   // buffer holding u (sum of the finished substeps' increments)
  int ppar;   // buffer holding p (the current substep's Newton sum)
  int phases; // work passes taken
  int pad;
  double scal;     // error scale tol_a + tol_r max|T^n|
  double ring[5];  // the last five scaled error estimates
};

struct BatchArgs {
  const BProb* prob;
  BTile* tile;
  BState* state;
  int* ndone;            // problems done (control kernel counts them)
  const double* coef64;  // 5-point stencil, SoA with stride ntot (FP64)
  const void* coef;      // stencil of the Newton terms (FP64 or FP32)
  const double* g;       // G(T) = J T + g
  double* T0;            // the caller's temperatures
  double* T1;            // internal temperature buffer
  double *u0, *u1;       // substep increment sums (ping-pong)
  double* v;             // G(T^n) of the current step
  void *q0, *q1;         // Newton vectors (FP64 or FP32)
  void *p0, *p1;         // Newton sums (ping-pong over substeps)
  const double* dk;      // divided differences, (m_max + 1) per problem
  const double* shift;   // c/gamma + xi_{k-1}, (m_max + 1) per problem
  double* part;          // kBatchPartStride partials per tile
  long long ntot;
  int nprob, ntiles, nsteps, m_max;
  int nt;                // Newton terms per pass of the tile shape
  double tol_a, tol_r, thresh;
};

hipError_t batch_pack(int nx, int ny, const double* coef, const double* F, const double* T0,
                      double* bcoef, double* g, long long ntot, long long off, hipStream_t s);
hipError_t batch_reset(const BatchArgs& a, hipStream_t s);
// One phase of every problem: the work pass over all tiles, then the control
// kernel.  e0 / e1 (optional) time the work pass alone.
hipError_t batch_phase(const BatchArgs& a, int shape, int fp32, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
size_t batch_lds_bytes(int shape, int fp32);

}  // namespace erem
