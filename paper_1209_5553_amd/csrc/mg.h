// Aggregation multigrid preconditioner of the TPFA pressure operator.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kMgMaxLevels = 16;
constexpr int kMgLdsCells = 1024;   // levels at or below this size run in one workgroup
#ifndef EREM_MG_TOP_CYCLES
#define EREM_MG_TOP_CYCLES 2
#endif
#ifndef EREM_MG_SUB_CYCLES
#define EREM_MG_SUB_CYCLES 2
#endif
constexpr int kMgTopCycles = EREM_MG_TOP_CYCLES;  // cycles per coarse solve on the first LDS level
constexpr int kMgSubCycles = EREM_MG_SUB_CYCLES;  // V-cycles under the second LDS level per visit
constexpr int kMgBottomCells = 64;  // bottom level, solved with a dense inverse
#ifndef EREM_MG_SWEEPS
#define EREM_MG_SWEEPS 3
#endif
#ifndef EREM_MG_LDS_SWEEPS
#define EREM_MG_LDS_SWEEPS 2
#endif
constexpr int kMgSweeps = EREM_MG_SWEEPS;         // damped-Jacobi sweeps each way, 2D grid levels
constexpr int kMgLdsSweeps = EREM_MG_LDS_SWEEPS;  // the same on the LDS levels (even)
static_assert(kMgLdsSweeps % 2 == 0 && kMgLdsSweeps >= 2, "LDS sweeps come in pairs");

// One level: faces in the fine-grid layout (x faces (nz, ny, nx+1), y faces
// (nz, ny+1, nx), z faces (nz+1, ny, nx)), diagonal, and work vectors.
struct MgLevelDev {
  int nx, ny, nz;
  double *tx, *ty, *tz, *diag;
  double *b, *x, *y;  // rhs, down-leg iterate, up-leg result
};

// Arguments of the single-workgroup coarse solve over levels lc..lb.
struct MgCoarseArgs {
  int nlev;                    // levels handled in LDS (the last is the bottom)
  int n0;                      // cells of the first of them
  int nu;                      // Jacobi sweeps before and after the coarse correction (the kernels do two)
  int inv_off;                 // LDS offset of the bottom inverse
  int ncyc;                    // cycles on the first LDS level (1 when it is the bottom)
  int ncyc1;                   // V-cycles of the second level's coarse problem per visit (1 when it is the bottom)
  double omega_c;              // coarse-correction relaxation
  int off[kMgMaxLevels][8];    // LDS offsets: tx, ty, tz, diag, B, E, T, 1/diag per level
  MgLevelDev lev[kMgMaxLevels];
};

struct MgHierarchy {
  int nlev = 0;            // levels built (finest first), the last is the bottom
  int lc = 0;              // first level handled in LDS
  int lb = 0;              // bottom level (= nlev - 1)
  int coarse_threads = 0;
  size_t lds_bytes = 0;
  double omega_c = 2.1;
  double* binv = nullptr;  // dense inverse of the bottom operator (device)
  MgLevelDev lev[kMgMaxLevels];
  MgCoarseArgs coarse;
};

// Chronopoulos-Gear conjugate gradients folded into the finest legs of a
// 2D hierarchy.  With update, the first down leg runs iteration it (stop
// test; alpha, beta from the ring; s = w + beta s_old; r_new = r - alpha s;
// p = z + beta p; x += alpha p; r_new . r_new into the ring) and the cycle
// preconditions r_new; the last up leg also forms w_out = A z and puts r.z
// and w.z into the ring slot.  r_new and s_new are separate buffers from r
// and s_old: neighbouring tiles still read the old values.
struct CgFuse {
  int update;          // run iteration it in the first down leg
  int it;
  double* x;
  double* r_new;
  const double* z;     // z_it (read)
  const double* w;     // w_it = A z_it (read)
  double* p;           // p_{it-1} in, p_it out (own cells)
  const double* s_old;
  double* s_new;
  double* w_out;       // w of the new z
};

hipError_t mg_setup(const MgHierarchy& h, hipStream_t s);
// z = M^{-1} r.  With cg (only where mg_fuses_cg): see CgFuse; with
// cg->update, r is the residual before the update and z = M^{-1} r_new.
hipError_t mg_apply(const MgHierarchy& h, const double* r, double* z, PcgState* st, int rz_slot,
                    hipStream_t s, const CgFuse* cg = nullptr);
// True when the finest level is 2D and runs the global-memory legs.
inline bool mg_fuses_cg(const MgHierarchy& h) { return h.lc > 0 && h.lev[0].nz == 1; }
hipError_t mg_set_lds_limit(int bytes);

}  // namespace erem
