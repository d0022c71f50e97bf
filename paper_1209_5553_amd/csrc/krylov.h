// Device Arnoldi process for the Krylov evaluation of phi1 (krylov.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kMaxKrylov = 64;

int kry_num_blocks(const Dims& d);
// Arnoldi (CGS2) on the start vector in w[0, N): w holds 2N doubles, V
// (m + 1) N, H (m + 1) m, g m + 1 and part (m + 1) kry_num_blocks(d).
hipError_t arnoldi_cgs2(const Dims& d, const double* coef, double* V, double* w, double* H, double* beta,
                        double* g, double* part, int m, hipStream_t s);
hipError_t krylov_combine(const Dims& d, const double* V, int nvec, const double* c, double* u,
                          int first, hipStream_t s);

}  // namespace erem
