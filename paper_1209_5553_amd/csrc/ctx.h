// Internal view of the EREM context shared by the library's translation
// units (erem_api.cpp, adjoint_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "device.h"
#include "rosenbrock.h"
#include "erem.h"
#include "mg.h"

struct DivDiffCache {
  double hc = NAN, hg = NAN;
  int n = 0;
  std::vector<double> d;
};

struct erem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  erem::Dims d{};
  erem::Phys ph{};
  bool rock_set = false, fluid_set = false, bc_set = false;
  bool trans_set = false, flux_set = false, jac_set = false;
  // coef and F hold the pressure operator J_p and G4 of erem_step_pressure
  // (false: the heat Jacobian J and G2 = dT/dt)
  bool op_pressure = false;

  // fields (device)
  double *logk = nullptr, *poro = nullptr;
  double *tx = nullptr, *ty = nullptr, *tz = nullptr;
  double *fx = nullptr, *fy = nullptr, *fz = nullptr;
  double *coef = nullptr, *F = nullptr;
  // non-autonomous step: D_t G and the phi2 term (allocated on first use)
  double *gt = nullptr, *zt = nullptr;
  // shifted solves (BiCGSTAB) and the Rosenbrock / theta-Euler stages
  // (allocated on first use): solver vectors, stage vectors k_1..k_3, the
  // stage state Y, G(Y), the right-hand side, and a scratch stencil
  double *bc_r = nullptr, *bc_rhat = nullptr, *bc_p0 = nullptr, *bc_p1 = nullptr, *bc_v0 = nullptr,
         *bc_v1 = nullptr, *bc_s = nullptr, *bc_t = nullptr;
  double *rs_k0 = nullptr, *rs_k1 = nullptr, *rs_k2 = nullptr, *rs_y = nullptr, *rs_g = nullptr,
         *rs_rhs = nullptr, *rs_coef = nullptr;
  erem::BicgState* bicg = nullptr;
  erem::BicgState* h_bicg = nullptr;
  double* bicg_parts = nullptr;  // the BiCGSTAB partial slots (erem::bicg_parts_words(cell bands))
  int bicg_last = 0;  // iterations of the last converged solve (poll placement)
  double *qa = nullptr, *qb = nullptr, *pacc = nullptr, *u = nullptr, *w = nullptr;
  double *pres = nullptr, *pr = nullptr, *pr2 = nullptr, *pz = nullptr, *pp0 = nullptr, *pp1 = nullptr;
  double *pw = nullptr, *ps0 = nullptr, *ps1 = nullptr;  // Chronopoulos-Gear w = A z and s
  double *pq = nullptr, *pdiag = nullptr, *pres_lo = nullptr, *pdelta = nullptr, *prhs = nullptr;
  double* pres_prev = nullptr;  // previous pressure for the extrapolated warm start (on first use)
  bool pres_prev_set = false;   // pres_prev holds the solution before the context's current one
  double* part = nullptr;  // Leja block partial sums (ring of kLejaRing terms)
  // FP32 copies for the mixed-precision Leja passes (allocated on first use)
  float *coef32 = nullptr, *qa32 = nullptr, *qb32 = nullptr, *p32 = nullptr;
  bool coef32_valid = false;
  // Krylov basis (m+1 vectors), work vector, Hessenberg matrix, norm, coefficients
  double *kV = nullptr, *kw = nullptr, *kH = nullptr, *kbeta = nullptr, *kc = nullptr, *kg = nullptr,
         *kpart = nullptr;
  int kry_m = 0;
  std::vector<double> hH;
  size_t nfx = 0, nfy = 0, nfz = 0;

  // device control blocks
  erem::LejaCoef* cf = nullptr;
  erem::LejaState* states = nullptr;
  int nstates = 0;
  erem::AsmReduce* red = nullptr;
  erem::PcgState* pcg = nullptr;

  // pinned host mirrors
  erem::LejaCoef* h_cf = nullptr;
  erem::LejaState* h_states = nullptr;
  erem::AsmReduce* h_red = nullptr;
  erem::PcgState* h_pcg = nullptr;
  double* pcg_parts = nullptr;    // the PCG partial slots (erem::pcg_parts_words(pcg_nb))
  double* h_pcg_parts = nullptr;  // pinned: ||b||^2 and r.r partials of a residual
  int pcg_nb = 0;

  std::vector<double> xi;  // Leja points
  DivDiffCache dd, dd2;  // phi1 and phi2 divided differences
  int last_m = 0;          // largest substep degree of the previous evaluation
  int last_m_p = 0;        // the same for the transient pressure (its own degree)
  // interval width beta - alpha of the previous Leja evaluation (0: none), which
  // predicts the next one's substep count; the same for the transient pressure
  double last_w = 0.0, last_w_p = 0.0;
  // coefficients formed on the device: the Leja points and the
  // divided-difference cache
  double* xi_dev = nullptr;
  erem::DdCache* ddc = nullptr;
  // profiling (HIP events around each Leja term and PCG half-iteration)
  // iterations of the last converged CG solve (poll placement), per kind of
  // solve (0: pressure, 1: other SPD right-hand sides) and refinement
  // correction (the first correction of a solve takes many more iterations
  // than the later ones)
  int pcg_last[2][4] = {};
  int prof = 0;  // per-launch event timing: 0 off, n > 0 one launch in n
  std::vector<hipEvent_t> ev;
  hipEvent_t ev_setup = nullptr;  // the first residual readback of a pressure solve
  double t_leja = 0.0, t_pcg_a = 0.0, t_pcg_b = 0.0, t_mg = 0.0;
  long long n_leja = 0, n_pcg_a = 0, n_pcg_b = 0, n_mg = 0;
  double t_adj = 0.0;
  long long n_adj = 0;
  double t_bicg = 0.0;
  long long n_bicg = 0;
  // multigrid preconditioner of the pressure operator
  erem::MgHierarchy mg;
  bool use_mg = true;
  std::vector<double*> mg_bufs;
  double alpha = 0.0, beta = 0.0, tmax = 0.0;
  std::vector<int> applied;  // Leja terms applied per substep by the last evaluation
  // adjoint storage (allocated on first use): stored Leja iterates, substep
  // sums u_j, a recomputed segment of iterates, and the per-cell / per-face
  // adjoint fields
  double* adj_q = nullptr;
  size_t adj_q_cap = 0;
  double* adj_u = nullptr;
  size_t adj_u_cap = 0;
  double* adj_seg = nullptr;
  size_t adj_seg_cap = 0;
  double* adj_block = nullptr;
  double *adj_sa = nullptr, *adj_sb = nullptr, *adj_jbar = nullptr, *adj_wbar = nullptr, *adj_ubar = nullptr;
  double *adj_rbar = nullptr, *adj_dbar = nullptr, *adj_abar = nullptr, *adj_fxbar = nullptr;
  double *adj_fybar = nullptr, *adj_pbar = nullptr, *adj_lam = nullptr, *adj_pscr = nullptr;
  std::string err;
};

namespace erem_internal {

int fail(erem_ctx* c, int code, const std::string& msg);

// Message of the calls that need the heat Jacobian and G2 while the context
// holds the pressure operator of erem_step_pressure.
constexpr const char* kHoldsPressure =
    "the context holds the pressure operator of erem_step_pressure: call erem_form_jacobian first";

#define HIP_TRY(ctx, expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess)                                                         \
      return erem_internal::fail((ctx), EREM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

template <class T>
int dev_alloc(erem_ctx* c, T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) return fail(c, EREM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return EREM_OK;
}

int check_opts(erem_ctx* c, const erem_opts* o);
int ensure_events(erem_ctx* c, size_t n);  // event pool of at least n events (profiling)
double elapsed_ms(hipEvent_t a, hipEvent_t b);
int ndir(const erem_ctx* c);
int read_reduce(erem_ctx* c);
const std::vector<double>& divided_differences(erem_ctx* c, double hc, double hg, int n, int ell = 1);
// x <- A^{-1} b for the TPFA pressure matrix A (Dirichlet x faces folded into
// the diagonal, no right-hand side from the boundary values): conjugate
// gradients with the context's preconditioner, refined in FP64 until
// ||b - A x|| <= rtol ||b||.  x and b are device arrays of N values.
int spd_solve(erem_ctx* c, const double* b, double* x, double rtol, int max_iter, int* iters);

}  // namespace erem_internal
