// Host launchers of the discrete-adjoint kernels (reverse of S9 .. S1).
#pragma once
#include "common.h"
#include "step.h"

namespace chns {

// A1: pbar = (dt/We) D(ubar' / rho_f')
// (also zeta = 0, the initial guess of the adjoint pressure solve)
void adj_p_rhs(int dim, const Geo &g, const StepConst &k, const double *phin, const double *const ubar[3],
               double *pbar, double *zeta, hipStream_t st);
// A3: ustar_bar = ubar' + (We/dt) G zeta; rho_f' bar from the projection and
// the pressure operator; zero the accumulators.
void adj_proj_faces(int dim, const Geo &g, const StepConst &k, const double *phin, const double *p, const double *zeta,
                    const double *const ubar[3], AdjBufs &A, double *const uout[3], hipStream_t st);
// A5 + A6 for component a (after K nu_a = ustar_bar_a)
void adj_mom(int dim, const Geo &g, const StepConst &k, int a, const double *phi, const double *phin,
             const double *mu, const double *const u[3], const double *const ustar[3], AdjBufs &A,
             double *const uout[3], hipStream_t st);
// A7 .. A9: density / viscosity, mass flux and phi update adjoints, mu_bar
void adj_rho_flux_mu(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phin,
                     const double *mu, const double *const u[3], const double *phibar_in, AdjBufs &A,
                     double *const uout[3], double *phibar_out, hipStream_t st);
// A10: rhs of the CH adjoint solve, L phihat, omega = 0
void adj_ch_rhs(int dim, const Geo &g, const StepConst &k, const double *phihat, AdjBufs &A, hipStream_t st);
// A12 .. A15 after M omega = chr
void adj_ch_post(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                 AdjBufs &A, double *const uout[3], double *phibar_out, hipStream_t st);
// final: out[0] = dL/dsigma, out[1] = dL/dM (sigma = 1/We, M = We/Pe),
// out[2] = dL/dk, out[3] = dL/ds_t of this step
void adj_params(int dim, const Geo &g, const StepConst &k, const AdjBufs &A, double *out, hipStream_t st);

}  // namespace chns
