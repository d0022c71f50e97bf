// Aggregation multigrid preconditioner of the TPFA pressure operator.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

constexpr int kMgMaxLevels = 16;
constexpr int kMgLdsCells = 1024;   // levels at or below this size run in one workgroup

// One level: faces in the fine-grid layout (x faces (nz, ny, nx+1), y faces
// (nz, ny+1, nx), z faces (nz+1, ny, nx)), diagonal, and work vectors.
struct MgLevelDev {
  int nx, ny, nz;
  double *tx, *ty, *tz, *diag;
  double *b, *x, *y;
};

// Arguments of the single-workgroup coarse solve over levels lc..nlev-1.
struct MgCoarseArgs {
  int nlev;        // levels handled in LDS
  int n0;          // cells of the first of them
  int lds_words;   // LDS words taken by the level arrays
  int ninner;      // V-cycles of the coarse solve
  int nu;          // Jacobi sweeps before and after the coarse correction
  int nu_bottom;   // sweeps on the coarsest level
  double omega_c;  // coarse-correction relaxation
  MgLevelDev lev[kMgMaxLevels];
};

struct MgHierarchy {
  int nlev = 0;            // all levels, finest first
  int lc = 0;              // first level handled in LDS
  int coarse_threads = 0;
  size_t lds_bytes = 0;
  double omega_c = 1.6;
  MgLevelDev lev[kMgMaxLevels];
  MgCoarseArgs coarse;
};

hipError_t mg_setup(const MgHierarchy& h, hipStream_t s);
hipError_t mg_apply(const MgHierarchy& h, const double* r, double* z, PcgState* st, int rz_slot,
                    hipStream_t s);
hipError_t mg_set_lds_limit(int bytes);

}  // namespace erem
