// Adjoint (reverse-mode) kernels of the coupled EREM step (adjoint.hip).
// 2D grids; cell arrays flat x + nx*y, stencils SoA [5][N] in the order
// centre, -x, +x, -y, +y; face arrays as the forward path's.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace erem {

// s_out = scale * ubar
hipError_t launch_adj_scale(const Dims& d, const double* ubar, double scale, double* s_out, hipStream_t s);

// One reverse Newton-Leja term (k from m down to 1), with s_in = s_k and
// q_prev = q_{k-1}:
//   s_out = yscale * ubar + inv_g * J^T s_in - shift_k * s_in
//   jbar[dir][i] += inv_g * s_in[i] * q_prev[neighbour(i, dir)]
hipError_t launch_adj_rev_term(const Dims& d, const double* coef, const double* s_in, const double* q_prev,
                               const double* ubar, double yscale, double inv_g, double shift_k, double* jbar,
                               double* s_out, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// End of a reversed substep with rbar = s_0: wbar += rbar; when u is given
// (substeps after the first), ubar += J^T rbar and jbar[dir][i] += rbar[i] u[nb].
hipError_t launch_adj_substep(const Dims& d, const double* coef, const double* rbar, const double* u,
                              double* wbar, double* ubar, double* jbar, hipStream_t s);

// Heat-operator adjoint, cell part: from Gbar (wbar) and Jbar, the bars of R,
// of the operator row (diagonal, four neighbours) and the capacity term of Tbar.
hipError_t launch_adj_heat_cell(const Dims& d, const Phys& ph, const double* poro, const double* fx,
                                const double* fy, const double* T, const double* jbar, const double* wbar,
                                double* Tbar, double* rbar, double* dbar, double* abar, hipStream_t s);

// Heat-operator adjoint, face part: Tbar += A_h^T Rbar and the face-flux bars.
hipError_t launch_adj_heat_face(const Dims& d, const Phys& ph, const double* fx, const double* fy,
                                const double* rbar, const double* dbar, const double* abar, double* Tbar,
                                double* fxbar, double* fybar, hipStream_t s);

// pbar from the face-flux bars (F = t (p_i - p_j), boundary half cells).
hipError_t launch_adj_flux_p(const Dims& d, const double* tx, const double* ty, const double* fxbar,
                             const double* fybar, double* pbar, hipStream_t s);

// r = b - A x for the pressure matrix (no boundary right-hand side); sums of
// r^2 and b^2 into the slots of st.
hipError_t launch_spd_residual(const Dims& d, const double* tx, const double* ty, const double* x,
                               const double* b, double* r, PcgState* st, hipStream_t s);

// Transmissibility and mobility adjoint: tbar per face from fbar, the
// pressure adjoint lambda and the (double-double) pressure; then
// logkbar += mbar m and Tbar += mbar m (rho'/rho - mu'/mu).
hipError_t launch_adj_trans(const Dims& d, const Phys& ph, const double* logk, const double* T,
                            const double* phi, const double* plo, const double* fxbar, const double* fybar,
                            const double* lam, double* Tbar, double* logkbar, hipStream_t s);

}  // namespace erem
