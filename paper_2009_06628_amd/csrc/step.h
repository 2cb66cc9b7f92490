// Host launchers of the time-step kernels (S1..S9 and diagnostics).
#pragma once
#include "common.h"

namespace chns {

// Constants of one step, derived from chns_props on the host.
struct StepConst {
    double h, ih, ih2;
    double dt, S, Cn, Pe, kM;          // kM = 1/(Pe Cn)
    double alpha, beta, gamma, xi;     // mixture maps
    double inv_Re, inv_We, We, inv_Fr;
};

constexpr int kPCoef = 1, kPRhs = 2;

// Tangential velocities of moving walls: v[b][side][a] is a face array of
// component a whose layer next to wall (b, side) holds the wall speed, or
// null for a wall at rest.
struct WallVel {
    const double *v[3][2][3];
};

// Outputs of the set-up of every momentum component (component a: level-0
// coefficients s, cs[b] of its hierarchy, right-hand side, initial guess
// u_a; ustar null: the guess is left to the time-guess kernel).
struct MomOut {
    double *s[3];
    double *cs[3][3];   // [component][direction]
    double *rhs[3];
    double *ustar[3];
};

// Three-phase constants (TernConst, common.h) from the properties.
TernConst tern_const_of(const chns_props &p);

// The stored phase fields of a three-phase step (phases 1 and 2; phase 3 is
// -1 - phi_1 - phi_2): phi^n, phi^{n+1} and mu~^{n+1}.
struct Phases3 {
    const double *phi[2];
    double *phin[2];
    double *mu[2];
    double *mix[5];   // per-step mixture fields: rho^{n+1}, rho^n, eta^{n+1}, rho_lin^n, chi
};

// T1: r_i and phihat_i = phi_i for i = 1, 2 (hat1 / hat2 null: not written).
void launch_ch_rhs3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                    const double *const u[3], double *r1, double *r2, double *hat1, double *hat2, hipStream_t st);
// T3: mu~_i from phihat_i.
void launch_mu3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph, const double *hat1,
                const double *hat2, hipStream_t st);
// T4: phi_i^{n+1}, and the per-step mixture fields read by the set-up and
// projection (rho^{n+1}, rho^n, eta^{n+1}, rho_lin^n, chi), from the same pass.
void launch_phi_update3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                        const double *const u[3], hipStream_t st);
// T5-T7 set-up of every component in one pass (as launch_mom_setup_all).
// m: face mass-flux arrays of the step (written here first).
void launch_mom_setup3_all(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                           const double *const u[3], const MomOut &o, double *const m[3], hipStream_t st,
                           const WallVel *wv = nullptr);
// T8 set-up (parts as launch_p_setup).
void launch_p_setup3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                     const double *const ustar[3], double *s, double *const cs[3], double *rhs, hipStream_t st,
                     int part, double *rho_out = nullptr);
// T9: projection, phi_i = phi_i^{n+1}.
void launch_project3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                     const double *const ustar[3], const double *p, double *phi1, double *phi2, double *const u[3],
                     hipStream_t st);
// Diagnostics into out[0..8] = sum c_1, c_2, c_3, kinetic, sum (Sigma_i/2) psi,
// sum (Sigma_i/2) |G phi_i|^2, gravity, umax, divmax.
void launch_diagnostics3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const double *phi1,
                         const double *phi2, const double *const u[3], double *part, unsigned int *counter,
                         double *out, hipStream_t st);

// Energy-law monitor of one two-phase step (after S8, before S9): unscaled
// sums visc, chem, cubic, inert into out[0..3]; s[a], cs[a][b] the level-0
// momentum coefficients of component a.
void launch_energy_monitor(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phi_new,
                           const double *mu, const double *const u[3], const double *const ustar[3], const double *p,
                           const double *const s[3], const double *const cs[3][3], double *part,
                           unsigned int *counter, double *out, hipStream_t st);

// Crank-Nicolson variant (cn.hip): kh is the step constants with dt/2.
void launch_cn_ch_rhs(int dim, const Geo &g, const StepConst &kh, const double *phik, const double *phim,
                      const double *const vm[3], double *r, double *phihat, hipStream_t st);
void launch_cn_phi_update(int dim, const Geo &g, const StepConst &k, const double *phik, const double *phim,
                          const double *const vm[3], const double *mu, double *phin, double *phimid, hipStream_t st);
void launch_cn_mom_setup(int dim, const Geo &g, const StepConst &kh, int a, const double *phim,
                         const double *phimid, const double *mu, const double *const vm[3], double *s,
                         double *const cs[3], double *rhs, double *ustar, const double *vk, const double *pm,
                         const WallVel *wv, hipStream_t st);
void launch_cn_project(int dim, const Geo &g, const StepConst &kh, const double *phimid,
                       const double *const ustar[3], const double *dp, double *const vt[3], double *p, hipStream_t st);
void launch_cn_finish(int dim, const Geo &g, const double *const vt[3], double *const u[3], double *phi,
                      const double *phin, hipStream_t st);
void launch_cn_zero(const Geo &g, double *x, hipStream_t st);

// S1: r = phi - dt D(u A phi) + dt kM L(psi'(phi) - S phi); phihat = phi
// (phihat null: not written).
void launch_ch_rhs(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                   double *r, double *phihat, hipStream_t st);
// S3: mu = psi'(phi) + S (phihat - phi) - Cn^2 L phihat.
void launch_mu(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phihat, double *mu,
               hipStream_t st);
// S4: phi_new = phi - dt D(u A phi - kM G mu).
void launch_phi_update(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                       const double *mu, double *phi_new, hipStream_t st);
// S5-S7 set-up for component a: level-0 coefficients of the momentum slot,
// right-hand side, and initial guess ustar_a = u_a.
// wv: tangential velocities of moving walls (null: every wall at rest).
void launch_mom_setup(int dim, const Geo &g, const StepConst &k, int a, const double *phi, const double *phi_new,
                      const double *mu, const double *const u[3], double *s, double *const cs[3], double *rhs,
                      double *ustar, hipStream_t st, int coef_only = 0, const WallVel *wv = nullptr);
// S5-S7 set-up of all d components in one pass (each thread sets up the
// faces of every axis at its cell index): the components read the same
// mixture, flux and velocity fields, so one sweep over them replaces d.
void launch_mom_setup_all(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phi_new,
                          const double *mu, const double *const u[3], const MomOut &o, hipStream_t st,
                          const WallVel *wv = nullptr);
// S8 set-up: pressure coefficients 1/(rho_f h^2) from clamp(phi_new)
// (part & kPCoef) and rhs = -(We/dt) D ustar (part & kPRhs).  The
// coefficients need only phi_new, so the step sets them and the pressure
// hierarchy up while the momentum solves run.
void launch_p_setup(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    double *s, double *const cs[3], double *rhs, hipStream_t st, int part = kPCoef | kPRhs,
                    double *rho_out = nullptr);
// Pressure coefficients from a given cell density (stand-alone solve).
void launch_p_coef_from_rho(int dim, const Geo &g, double ih2, const double *rho, double *s, double *const cs[3],
                            hipStream_t st);
// S9: u = ustar - (dt/We) G p / rho_f; phi = phi_new.
void launch_project(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    const double *p, double *phi, double *const u[3], hipStream_t st);
// CH slot level-0 coefficients: s = 1, cs = c / h^2.
void launch_fill_ch(int dim, const Geo &g, double csval, double *s, double *const cs[3], hipStream_t st);
// S8 initial guess: where p equals h[0] (the handle's previous solution), p
// extrapolated in time from p and the older pressures h[1], h[2] (as many
// as are finite: quadratic, linear or p itself); then h[2] = h[1],
// h[1] = the incoming p.
void launch_pressure_guess(const Geo &g, double *p, double *const h[3], hipStream_t st);
// S7 initial guess of one component: where p equals plast, u extrapolated
// from its last solutions h[0], h[1], h[2] (as many as are finite), else u^n
// (un).  Writes every cell of u: the momentum set-up is then given no ustar.
void launch_velocity_guess(const Geo &g, double *u, double *const h[3], const double *un, const double *p,
                           const double *plast, hipStream_t st);
// Diagnostics into out[0..6] = mass+, mass-, kinetic, free, gravity, umax, divmax.
void launch_diagnostics(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                        double *part, unsigned int *counter, double *out, hipStream_t st);

}  // namespace chns
