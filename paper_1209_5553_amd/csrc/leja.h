// Device Newton-Leja evaluation: launchers (leja.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kLejaRing = 16;       // terms whose block partials are kept
#ifndef EREM_LEJA_TILE_ROWS
#define EREM_LEJA_TILE_ROWS 8
#endif
constexpr int kLejaTileRows = EREM_LEJA_TILE_ROWS;  // rows of the multi-term tile (64 wide)
#ifndef EREM_LEJA_THREAD_ROWS
#define EREM_LEJA_THREAD_ROWS 8
#endif
constexpr int kLejaThreadRows = EREM_LEJA_THREAD_ROWS;  // thread rows of its block (64 wide)
constexpr int kCheckThreads = 1024;  // workgroup of the stop-test kernel
constexpr int kCheckEvery = 4;      // terms between stop tests

int leja_num_blocks(const Dims& d);

hipError_t launch_leja_reset(LejaState* st, int nslots, int nterms, hipStream_t s);
template <class V>
hipError_t launch_leja_init(const Dims& d, const LejaCoef* cf, const double* v, V* q0, V* p,
                            double* part, hipStream_t s);
template <class V>
hipError_t launch_leja_term(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout,
                            V* p, const LejaState* st, double* part, int k, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Terms k .. k + nterms - 1 in one launch (2D grids only, nterms 2 or 4):
// the last q to qout, p updated, every term's partial sums in its ring slot.
template <class V>
hipError_t launch_leja_terms(const Dims& d, const LejaCoef* cf, const V* coef, const V* qin, V* qout,
                             V* p, const LejaState* st, double* part, int k, int nterms, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_leja_check(const Dims& d, const LejaCoef* cf, LejaState* st, const double* part,
                             int k1, int k2, hipStream_t s);
// u = (first ? 0 : u) + delta p (+ zt when zt is not null)
template <class V>
hipError_t launch_substep_update(const Dims& d, double* u, const V* p, double delta, int first,
                                 hipStream_t s, const double* zt = nullptr);
hipError_t launch_cast_f32(const double* a, float* b, long long n, hipStream_t s);

}  // namespace erem
