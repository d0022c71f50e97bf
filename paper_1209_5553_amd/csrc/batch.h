// Batched EREM kernel (batch.hip): shared structures.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kNumTileShapes = 5;
extern const int kTileShapes[kNumTileShapes][2];  // {threads per problem, cells loaded ahead per thread (0: fused terms)}

// Static description of one problem of the batch.
struct BProb {
  int nx, ny;
  int s;          // substeps per step
  int coef_off;   // first divided difference / shift of this problem
  long long off;  // first cell in the packed vectors
  double inv_g;   // 1 / gamma
  double delta;   // substep length h / s
};

// Outcome of one problem, written once by its workgroup.
struct BDyn {
  int step;   // steps completed
  int terms;  // Leja terms applied
  int flags;  // 1: no convergence within m_max, 2: non-finite norm
  int pad;
};

struct BatchArgs {
  const BProb* prob;
  BDyn* dyn;
  const int* order;     // problems in the order the workgroups take them
  const double* coef64; // 5-point stencil, SoA with stride ntot (FP64)
  const void* coef;     // stencil used by the Newton terms (FP64 or FP32)
  const double* g;      // G(T) = J T + g
  double* T;
  double* v;            // G(T^n) of the current step
  double* u;            // sum of the finished substeps' increments
  void *q0, *q1, *p;    // Newton vectors (FP64 or FP32)
  const double* dk;     // divided differences, (m_max + 1) per problem
  const double* shift;  // c/gamma + xi_{k-1}, (m_max + 1) per problem
  long long ntot;
  int nprob, nsteps, m_max;
  double tol_a, tol_r, thresh;
};

hipError_t batch_pack(int nx, int ny, const double* coef, const double* F, const double* T0,
                      double* bcoef, double* g, long long ntot, long long off, hipStream_t s);
hipError_t batch_launch(const BatchArgs& a, int shape, int fp32, int grid, hipStream_t s);

}  // namespace erem
