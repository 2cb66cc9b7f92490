// Time-step kernels of the split CHNS step (gfx950).  One thread per cell
// (or face) in grid-stride loops; coalesced along x.  FP64 throughout.
//
// Grid conventions: cell c = i + nx (j + ny k); the face array of axis a
// stores at entry c the face between c - e_a and c; on a walled axis the
// entry with index 0 is the wall and the opposite wall face is not stored.
// The model follows the paper's governing equations: mixture maps with the
// pull-back phi* (remark on the pull-back), double-well psi, consistent
// flux J = (rho_- - rho_+)/(2 rho_+ Cn) grad mu, skew-symmetric advection
// (appendix remark), surface tension in the potential form phi grad mu /
// (We Cn) (lemma on the weak equivalence of the forcing), gravity along -y.
#include "stepdev.h"

namespace chns {

// ---------------------------------------------------------------------------
// S1
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_ch_rhs(Geo g, StepConst k, const double *__restrict__ phi, U3 u,
                                                   double *__restrict__ r, double *__restrict__ phihat) {
    CELL_LOOP(g.N) ch_rhs_cell<DIM>(g, k, phi, u, r, phihat, c);
}

// ---------------------------------------------------------------------------
// S3
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mu(Geo g, StepConst k, const double *__restrict__ phi,
                                               const double *__restrict__ ph, double *__restrict__ mu) {
    CELL_LOOP(g.N) mu_cell<DIM>(g, k, phi, ph, mu, c);
}

// ---------------------------------------------------------------------------
// S4: flux-form update; both cells of a face evaluate its flux with the same
// operands in the same order, so sum(phi) telescopes to round-off.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_phi_update(Geo g, StepConst k, const double *__restrict__ phi, U3 u,
                                                       const double *__restrict__ mu, double *__restrict__ phin) {
    CELL_LOOP(g.N) phi_update_cell<DIM>(g, k, phi, u, mu, phin, c);
}

// ---------------------------------------------------------------------------
// S5-S7 set-up for component a
// ---------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mom_setup(Geo g, StepConst k, int a, const double *__restrict__ phi,
                                                      const double *__restrict__ phin, const double *__restrict__ mu,
                                                      U3 u, double *__restrict__ s, W3 cs, double *__restrict__ rhs,
                                                      double *__restrict__ ustar, int coef_only) {
    CELL_LOOP(g.N) mom_setup_cell<DIM>(g, k, a, phi, phin, mu, u, s, cs, rhs, ustar, coef_only, c);
}

// The same with moving walls.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mom_setup_walls(Geo g, StepConst k, int a, const double *__restrict__ phi,
                                                            const double *__restrict__ phin,
                                                            const double *__restrict__ mu, U3 u,
                                                            double *__restrict__ s, W3 cs, double *__restrict__ rhs,
                                                            double *__restrict__ ustar, int coef_only, WallVel wv) {
    const Mix2 mx = mk_mix2(k, phi, phin, mu);
    CELL_LOOP(g.N) mom_setup_body<DIM, Mix2, true>(g, k, a, mx, u, s, cs, rhs, ustar, coef_only, c, &wv);
}

// All components in one pass.
template <int DIM, bool WALLS>
__global__ void __launch_bounds__(kBlock) k_mom_setup_all(Geo g, StepConst k, const double *__restrict__ phi,
                                                          const double *__restrict__ phin,
                                                          const double *__restrict__ mu, U3 u, MomOut o, WallVel wv) {
    const Mix2 mx = mk_mix2(k, phi, phin, mu);
    CELL_LOOP(g.N) mom_setup_all_body<DIM, Mix2, WALLS>(g, k, mx, u, o, c, &wv);
}

// ---------------------------------------------------------------------------
// S8 set-up
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_p_setup(Geo g, StepConst k, const double *__restrict__ phin, U3 us,
                                                    double *__restrict__ s, W3 cs, double *__restrict__ rhs, int part,
                                                    double *__restrict__ rho_out) {
    const Mix2 mx = mk_mix2(k, phin, phin, phin);
    CELL_LOOP(g.N) p_setup_body<DIM>(g, k, mx, us, s, cs, rhs, part, c, rho_out);
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_p_coef_rho(Geo g, double ih2, const double *__restrict__ rho,
                                                       double *__restrict__ s, W3 cs) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int lo = nb_lo(g, c, ia[b], b);
            cs.a[b][c] = lo >= 0 ? 1.0 / (0.5 * (rho[c] + rho[lo])) * ih2 : 0.0;
        }
        s[c] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// S9
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_project(Geo g, StepConst k, const double *__restrict__ phin, U3 us,
                                                    const double *__restrict__ p, double *__restrict__ phi, W3 u) {
    CELL_LOOP(g.N) project_cell<DIM>(g, k, phin, us, p, phi, u, c);
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_fill_ch(Geo g, double csval, double *__restrict__ s, W3 cs) {
    CELL_LOOP(g.N) {
        s[c] = 1.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) cs.a[b][c] = csval;
    }
}

// ---------------------------------------------------------------------------
// diagnostics (deterministic)
// ---------------------------------------------------------------------------
constexpr int kNDiag = 8;   // mass+, mass-, kinetic, psi-sum, grad2-sum, grav, umax, divmax

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_diag(Geo g, StepConst k, const double *__restrict__ phi, U3 u,
                                                 double *part, unsigned int *counter, double *out) {
    __shared__ double lds[kBlock / kWave];
    double acc[kNDiag] = {0, 0, 0, 0, 0, 0, 0, 0};
    CELL_LOOP(g.N) {
        int i, j, kk;
        if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double pc = phi[c];
        const double rc = k.alpha * pullback(pc) + k.beta;
        acc[0] += 0.5 * (1.0 + pc);
        acc[1] += 0.5 * (1.0 - pc);
        acc[3] += 0.25 * (pc * pc - 1.0) * (pc * pc - 1.0);
        if (k.inv_Fr != 0.0) acc[5] += rc * ((j + 0.5) * k.h);
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            const double uc = u.a[a][c];
            if (lo >= 0) {
                const double rf = 0.5 * (rc + (k.alpha * pullback(phi[lo]) + k.beta));
                acc[2] += 0.5 * rf * uc * uc;
                const double gp = (pc - phi[lo]) * k.ih;
                acc[4] += gp * gp;
                acc[6] = fmax(acc[6], fabs(uc));
            }
            div += (hi >= 0 ? u.a[a][hi] : 0.0) - (lo >= 0 ? uc : 0.0);
        }
        acc[7] = fmax(acc[7], fabs(div * k.ih));
    }
#pragma unroll
    for (int q = 0; q < kNDiag; ++q) {
        double v = (q >= 6) ? block_max(acc[q], lds) : block_sum(acc[q], lds);
        if (threadIdx.x == 0) part[q * kMaxBlocks + blockIdx.x] = v;
    }
    if (last_block(counter)) {
        for (int q = 0; q < kNDiag; ++q) {
            double v = 0.0;
            for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
                const double x = ((volatile double *)part)[q * kMaxBlocks + b];
                v = (q >= 6) ? fmax(v, x) : v + x;
            }
            v = (q >= 6) ? block_max(v, lds) : block_sum(v, lds);
            if (threadIdx.x == 0) out[q] = v;
        }
        if (threadIdx.x == 0) *counter = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)
// bytes: algorithmic (compulsory) traffic in units of one FP64 cell array
#define DISPATCH(cls, arrays, dim, kern, n, st, ...)                            \
    do {                                                                        \
        const double bytes_ = 8.0 * (double)(arrays) * (double)(n);              \
        if ((dim) == 2)                                                         \
            LAUNCH(cls, bytes_, (kern<2>), n, st, __VA_ARGS__);                 \
        else                                                                    \
            LAUNCH(cls, bytes_, (kern<3>), n, st, __VA_ARGS__);                 \
    } while (0)


void launch_ch_rhs(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3], double *r,
                   double *phihat, hipStream_t st) {
    DISPATCH(K_CH_RHS, (phihat ? 3 : 2) + dim, dim, k_ch_rhs, g.N, st, g, k, phi, mk_u3(u), r, phihat);
}
void launch_mu(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phihat, double *mu,
               hipStream_t st) {
    DISPATCH(K_MU, 3, dim, k_mu, g.N, st, g, k, phi, phihat, mu);
}
void launch_phi_update(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                       const double *mu, double *phi_new, hipStream_t st) {
    DISPATCH(K_PHI_UPDATE, 3 + dim, dim, k_phi_update, g.N, st, g, k, phi, mk_u3(u), mu, phi_new);
}
void launch_mom_setup(int dim, const Geo &g, const StepConst &k, int a, const double *phi, const double *phi_new,
                      const double *mu, const double *const u[3], double *s, double *const cs[3], double *rhs,
                      double *ustar, hipStream_t st, int coef_only, const WallVel *wv) {
    if (wv) {
        DISPATCH(K_MOM_SETUP, 6 + 2 * dim, dim, k_mom_setup_walls, g.N, st, g, k, a, phi, phi_new, mu, mk_u3(u), s,
                 mk_w3(cs), rhs, ustar, coef_only, *wv);
        return;
    }
    DISPATCH(K_MOM_SETUP, 6 + 2 * dim, dim, k_mom_setup, g.N, st, g, k, a, phi, phi_new, mu, mk_u3(u), s, mk_w3(cs), rhs,
             ustar, coef_only);
}
void launch_mom_setup_all(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phi_new,
                          const double *mu, const double *const u[3], const MomOut &o, hipStream_t st,
                          const WallVel *wv) {
    WallVel w{};
    if (wv) w = *wv;
    // phi, phi_new, mu and u[d] read; s, cs[d], rhs, ustar written per component
    const double bytes = 8.0 * (3 + dim + dim * (3 + dim) - (o.ustar[0] ? 0 : dim)) * g.N;
    const dim3 grid(grid_for(g.N)), block(kBlock);
    if (dim == 2) {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup_all<2, true>), grid, block, st, g, k, phi, phi_new, mu, mk_u3(u),
                    o, w);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup_all<2, false>), grid, block, st, g, k, phi, phi_new, mu, mk_u3(u),
                    o, w);
    } else {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup_all<3, true>), grid, block, st, g, k, phi, phi_new, mu, mk_u3(u),
                    o, w);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup_all<3, false>), grid, block, st, g, k, phi, phi_new, mu, mk_u3(u),
                    o, w);
    }
}
void launch_p_setup(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    double *s, double *const cs[3], double *rhs, hipStream_t st, int part, double *rho_out) {
    const int words = (part & kPCoef ? 2 + dim + (rho_out ? 1 : 0) : 0) + (part & kPRhs ? 1 + dim : 0);
    DISPATCH(K_P_SETUP, words, dim, k_p_setup, g.N, st, g, k, phi_new, mk_u3(ustar), s, mk_w3(cs), rhs, part, rho_out);
}
void launch_p_coef_from_rho(int dim, const Geo &g, double ih2, const double *rho, double *s, double *const cs[3],
                            hipStream_t st) {
    DISPATCH(K_P_SETUP, 2 + dim, dim, k_p_coef_rho, g.N, st, g, ih2, rho, s, mk_w3(cs));
}
void launch_project(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    const double *p, double *phi, double *const u[3], hipStream_t st) {
    DISPATCH(K_PROJECT, 3 + 2 * dim, dim, k_project, g.N, st, g, k, phi_new, mk_u3(ustar), p, phi, mk_w3(u));
}
// Extrapolation in time from x^n = a and the older solutions b, c as far as
// they are finite (no history yet: NaN): 3a - 3b + c, 2a - b or a.
__device__ inline double time_extrap(double a, double b, double c) {
    return isfinite(c) ? 3.0 * a - 3.0 * b + c : (isfinite(b) ? 2.0 * a - b : a);
}

// S8 initial guess, cell by cell only where the incoming p^n is the handle's
// previous solution (a state edited or swapped by the caller keeps its own p
// there, and its history restarts); the history moves one step.
__global__ void __launch_bounds__(kBlock) k_pressure_guess(int N, double *__restrict__ p, const double *__restrict__ h0,
                                                           double *__restrict__ h1, double *__restrict__ h2) {
    for (int c = xcd_block() * kBlock + (int)threadIdx.x; c < N; c += (int)gridDim.x * kBlock) {
        const double pc = p[c], b = h1[c];
        const bool cont = pc == h0[c];
        if (cont) p[c] = time_extrap(pc, b, h2[c]);
        h2[c] = cont ? b : __longlong_as_double(-1LL);   // all-ones bytes: NaN, no history
        h1[c] = pc;
    }
}

void launch_pressure_guess(const Geo &g, double *p, double *const h[3], hipStream_t st) {
    TLAUNCH(K_P_SETUP, 48.0 * g.N, k_pressure_guess, dim3(grid_for(g.N)), dim3(kBlock), st, (int)g.N, p,
            (const double *)h[0], h[1], h[2]);
}

// The same for a velocity component of S7 from its last three solutions
// (the incoming pressure stands for the state: where it is the handle's
// previous solution, the velocity is too), else u^n (un); every cell of u is
// written (the set-up leaves it to this kernel)
__global__ void __launch_bounds__(kBlock) k_velocity_guess(int N, double *__restrict__ u, double *__restrict__ h0,
                                                           double *__restrict__ h1, const double *__restrict__ h2,
                                                           const double *__restrict__ un,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ plast) {
    for (int c = xcd_block() * kBlock + (int)threadIdx.x; c < N; c += (int)gridDim.x * kBlock) {
        if (p[c] == plast[c]) {
            u[c] = time_extrap(h0[c], h1[c], h2[c]);
        } else {
            // another trajectory: its history restarts with this step's solution
            u[c] = un[c];
            h0[c] = __longlong_as_double(-1LL);
            h1[c] = __longlong_as_double(-1LL);
        }
    }
}

void launch_velocity_guess(const Geo &g, double *u, double *const h[3], const double *un, const double *p,
                           const double *plast, hipStream_t st) {
    TLAUNCH(K_MOM_SETUP, 48.0 * g.N, k_velocity_guess, dim3(grid_for(g.N)), dim3(kBlock), st, (int)g.N, u, h[0], h[1],
            (const double *)h[2], un, p, plast);
}

void launch_fill_ch(int dim, const Geo &g, double csval, double *s, double *const cs[3], hipStream_t st) {
    DISPATCH(K_MG_SETUP, 1 + dim, dim, k_fill_ch, g.N, st, g, csval, s, mk_w3(cs));
}
void launch_diagnostics(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                        double *part, unsigned int *counter, double *out, hipStream_t st) {
    DISPATCH(K_DIAG, 1 + dim, dim, k_diag, g.N, st, g, k, phi, mk_u3(u), part, counter, out);
}

}  // namespace chns
