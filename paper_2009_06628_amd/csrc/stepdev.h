// Device helpers shared by the step and adjoint kernels.
#pragma once
#include "step.h"

namespace chns {

struct U3 {
    const double *a[3];
};
struct W3 {
    double *a[3];
};

inline U3 mk_u3(const double *const u[3]) { return U3{{u[0], u[1], u[2]}}; }
inline W3 mk_w3(double *const u[3]) { return W3{{u[0], u[1], u[2]}}; }

__device__ inline double dpsi(double p) { return p * p * p - p; }
__device__ inline double pullback(double p) { return fabs(p) <= 1.0 ? p : copysign(1.0, p); }
// derivative of the pull-back (1 inside (-1, 1), 0 outside)
__device__ inline double dpullback(double p) { return fabs(p) < 1.0 ? 1.0 : 0.0; }

// Store marked non-temporal (streamed past the L2): a pass that writes
// many arrays which no kernel reads back while they would still be in the
// L2 keeps the L2 for the input planes its stencils read again (the
// momentum set-up writes 15 arrays per cell: 198 -> 163 us at 128^3).
template <typename T>
__device__ inline void st_nt(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

#define CELL_LOOP(N) \
    for (int c = xcd_block() * (int)blockDim.x + (int)threadIdx.x; c < (int)(N); c += (int)(gridDim.x * blockDim.x))

template <int DIM>
__device__ inline void cc(const Geo &g, int c, int &i, int &j, int &k) {
    if (DIM == 2)
        cell_coords2(g, c, i, j, k);
    else
        cell_coords(g, c, i, j, k);
}

// Mass flux m_b = A_b(alpha phi + beta) u_b + J_b / Pe on the face f of axis
// b (index ib of f along b), zero on wall faces.
template <int DIM>
__device__ inline double mflux(const Geo &g, const StepConst &k, const double *__restrict__ phi,
                               const double *__restrict__ mu, const double *__restrict__ ub, int b, int f, int ib) {
    if (f < 0) return 0.0;                       // unstored upper wall face
    if (!g.per[b] && ib == 0) return 0.0;        // stored wall face
    const int lo = nb_lo(g, f, ib, b);
    const double rl = k.alpha * phi[f] + k.beta, rlo = k.alpha * phi[lo] + k.beta;
    return (0.5 * (rl + rlo)) * ub[f] - (k.alpha / (k.Cn * k.Pe)) * ((mu[f] - mu[lo]) * k.ih);
}

// Mixture policy of the two-phase model: the density / viscosity maps with
// the pull-back, the mass flux m = A(alpha phi^n + beta) u + J / Pe and the
// potential-form capillary force (1/(We Cn)) A(phi^n) G mu^{n+1} on a face.
// The set-up bodies below take a policy, so that the three-phase model
// (ternary.hip) runs the same momentum / pressure / projection arithmetic.
struct Mix2 {
    static constexpr bool kStoredFlux = false;          // mass flux evaluated per face (mflux_face)
    double alpha, beta, gamma, xi, jcoef, stcoef, ih;   // jcoef = alpha/(Cn Pe), stcoef = 1/(We Cn)
    const double *phi, *phin, *mu;                     // phi^n, phi^{n+1}, mu^{n+1}
    __device__ double rho_new(int e) const { return alpha * pullback(phin[e]) + beta; }
    __device__ double rho_old(int e) const { return alpha * pullback(phi[e]) + beta; }
    __device__ double eta_new(int e) const { return gamma * pullback(phin[e]) + xi; }
    // m_b on the face f between lo = f - e_b and f (not a wall face)
    __device__ double mflux_face(double ub, int f, int lo) const {
        const double rl = alpha * phi[f] + beta, rlo = alpha * phi[lo] + beta;
        return (0.5 * (rl + rlo)) * ub - jcoef * ((mu[f] - mu[lo]) * ih);
    }
    // capillary term subtracted from the momentum right-hand side on the face
    // between cam = c - e_a and c
    __device__ double capillary(int c, int cam) const {
        return stcoef * (0.5 * (phi[c] + phi[cam])) * ((mu[c] - mu[cam]) * ih);
    }
};

__host__ __device__ inline Mix2 mk_mix2(const StepConst &k, const double *phi, const double *phin, const double *mu) {
    return Mix2{k.alpha, k.beta, k.gamma, k.xi, k.alpha / (k.Cn * k.Pe), k.inv_We / k.Cn, k.ih, phi, phin, mu};
}

// Mass flux of a mixture policy on the face f of axis b (index ib of f
// along b), zero on wall faces.
template <int DIM, typename Mix>
__device__ inline double mflux_mix(const Geo &g, const Mix &mx, const double *__restrict__ ub, int b, int f, int ib) {
    if (f < 0) return 0.0;                       // unstored upper wall face
    if constexpr (Mix::kStoredFlux) {
        return mx.m[b][f];                       // the step's face fluxes (0 on stored wall faces)
    } else {
        if (!g.per[b] && ib == 0) return 0.0;    // stored wall face
        return mx.mflux_face(ub[f], f, nb_lo(g, f, ib, b));
    }
}

__device__ inline int wrap_next(int ib, int n) { return ib + 1 < n ? ib + 1 : 0; }
__device__ inline int wrap_prev(int ib, int n) { return ib > 0 ? ib - 1 : n - 1; }

// ---------------------------------------------------------------------------
// per-cell bodies of the step (shared by the grid-wide kernels and the
// workgroup-per-problem batched kernel)
// ---------------------------------------------------------------------------

// S1: r = phi - dt D(u A phi) + dt kM L(psi'(phi) - S phi); phihat = phi
template <int DIM>
__device__ inline void ch_rhs_cell(const Geo &g, const StepConst &k, const double *__restrict__ phi, const U3 &u,
                                   double *__restrict__ r, double *__restrict__ phihat, int c) {
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double pc = phi[c];
    const double gc = dpsi(pc) - k.S * pc;
    double div = 0.0, lap = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lo = nb_lo(g, c, ia[a], a);
        const int hi = nb_hi(g, c, ia[a], a);
        double flo = 0.0, fhi = 0.0;
        if (lo >= 0) {
            const double pl = phi[lo];
            flo = u.a[a][c] * (0.5 * (pl + pc));
            lap += (dpsi(pl) - k.S * pl) - gc;
        }
        if (hi >= 0) {
            const double ph = phi[hi];
            fhi = u.a[a][hi] * (0.5 * (pc + ph));
            lap += (dpsi(ph) - k.S * ph) - gc;
        }
        div += fhi - flo;
    }
    r[c] = pc - k.dt * (div * k.ih) + k.dt * k.kM * (lap * k.ih2);
    if (phihat) phihat[c] = pc;   // the guess of an iterative S2 solve (null: direct solve)
}

// S3: mu = psi'(phi) + S (phihat - phi) - Cn^2 L phihat
template <int DIM>
__device__ inline void mu_cell(const Geo &g, const StepConst &k, const double *__restrict__ phi,
                               const double *__restrict__ ph, double *__restrict__ mu, int c) {
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double xc = ph[c];
    double lap = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lo = nb_lo(g, c, ia[a], a);
        const int hi = nb_hi(g, c, ia[a], a);
        if (lo >= 0) lap += ph[lo] - xc;
        if (hi >= 0) lap += ph[hi] - xc;
    }
    const double pc = phi[c];
    mu[c] = dpsi(pc) + k.S * (xc - pc) - k.Cn * k.Cn * (lap * k.ih2);
}

// S4: flux-form update; both cells of a face evaluate its flux with the same
// operands in the same order, so sum(phi) telescopes to round-off.
__device__ inline double phi_face_flux(const StepConst &k, double uf, double pl, double pu, double ml, double mu_) {
    return uf * (0.5 * (pl + pu)) - k.kM * ((mu_ - ml) * k.ih);
}

template <int DIM>
__device__ inline void phi_update_cell(const Geo &g, const StepConst &k, const double *__restrict__ phi, const U3 &u,
                                       const double *__restrict__ mu, double *__restrict__ phin, int c) {
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double pc = phi[c], mc = mu[c];
    double div = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lo = nb_lo(g, c, ia[a], a);
        const int hi = nb_hi(g, c, ia[a], a);
        const double flo = lo >= 0 ? phi_face_flux(k, u.a[a][c], phi[lo], pc, mu[lo], mc) : 0.0;
        const double fhi = hi >= 0 ? phi_face_flux(k, u.a[a][hi], pc, phi[hi], mc, mu[hi]) : 0.0;
        div += fhi - flo;
    }
    phin[c] = pc - k.dt * (div * k.ih);
}

// S5-S7 set-up for component a: level-0 coefficients of the momentum operator,
// right-hand side, initial guess ustar_a = u_a
// WALLS: some walls move (wv their tangential velocities): the no-slip ghost
// value next to such a wall is 2 U - u instead of -u, which adds 2 k U to
// the right-hand side of the row (k the wall edge's coefficient).
// CN: the midpoint momentum equation of the Crank-Nicolson variant, for the
// unknown v~ with k.dt = dt/2: the operator (2 rho~_f/dt) - (1/Re) div(eta~ grad),
// the right-hand side (2 rho~_f/dt) v^k (vk) - (m~ . grad) v~m - capillary
// - (1/We) G p~m (pm) + gravity, where u holds v~m and mx the midpoint
// mixture; the advection is the advective form (the advective half of the
// skew-symmetric operator) instead of the skew-symmetric one.
// NT: the stores are non-temporal (the grid-wide set-up of every component,
// whose outputs are read only by later kernels).
template <int DIM, typename Mix, bool WALLS = false, bool CN = false, bool NT = false>
__device__ inline void mom_setup_body(const Geo &g, const StepConst &k, int a, const Mix &mx, const U3 &u,
                                      double *__restrict__ s, const W3 &cs, double *__restrict__ rhs,
                                      double *__restrict__ ustar, int coef_only, int c,
                                      const WallVel *wv = nullptr, const double *__restrict__ vk = nullptr,
                                      const double *__restrict__ pm = nullptr) {
    const double rvis = k.inv_Re * k.ih2;
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double *ua = u.a[a];
    auto put = [](double *q, double v) {
        if (NT)
            st_nt(q, v);
        else
            *q = v;
    };
    if (!g.per[a] && ia[a] == 0) {
        // wall face of a walled axis: decoupled identity row, u = 0
        put(&s[c], 1.0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) put(&cs.a[b][c], 0.0);
        if (!coef_only) {
            put(&rhs[c], 0.0);
            if (ustar) put(&ustar[c], 0.0);
        }
        return;
    }
    const int cam = nb_lo(g, c, ia[a], a);   // cell c - e_a
    auto eta_of = [&](int e) { return mx.eta_new(e); };
    const double rf_new = 0.5 * (mx.rho_new(c) + mx.rho_new(cam));
    const double rf_old = 0.5 * (mx.rho_old(c) + mx.rho_old(cam));
    const double e_c = eta_of(c), e_am = eta_of(cam);
    double fwall = 0.0;
    double sd = rf_new / k.dt;
    double nadv = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b);
        const int hi = nb_hi(g, c, ia[b], b);
        if (b == a) {
            // viscous coupling through the cell centres c - e_a (lower) and c (upper)
            double w = e_am * rvis;
            if (!g.per[a] && ia[a] == 1) {
                sd += w;        // neighbour is the wall face (u = 0)
                w = 0.0;
            }
            if (!g.per[a] && ia[a] == g.n[a] - 1) sd += e_c * rvis;   // upper wall face
            put(&cs.a[b][c], w);
            // skew advection, b == a
            const double m_c = mflux_mix<DIM>(g, mx, u.a[a], a, c, ia[a]);
            const double m_hi = hi >= 0 ? mflux_mix<DIM>(g, mx, u.a[a], a, hi, wrap_next(ia[a], g.n[a])) : 0.0;
            const double m_lo = mflux_mix<DIM>(g, mx, u.a[a], a, lo, wrap_prev(ia[a], g.n[a]));
            const double mp = 0.5 * (m_c + m_hi), mm = 0.5 * (m_lo + m_c);
            const double up = hi >= 0 ? ua[hi] : 0.0;
            const double um = (!g.per[a] && ia[a] == 1) ? 0.0 : ua[lo];   // wall face
            nadv += CN ? mp * (up - ua[c]) + mm * (ua[c] - um) : mp * up - mm * um;
        } else {
            // viscous coupling through the edge between faces c - e_b and c
            if (lo >= 0) {
                const int lam = nb_lo(g, lo, ia[a], a);   // c - e_b - e_a
                const double ee = 0.25 * (((e_c + e_am) + eta_of(lo)) + eta_of(lam));
                put(&cs.a[b][c], (!g.per[b] && ia[b] == 0) ? 0.0 : ee * rvis);
            } else {
                put(&cs.a[b][c], 0.0);
            }
            if (!g.per[b] && ia[b] == 0) {
                sd += 2.0 * (0.5 * (e_c + e_am)) * rvis;
                if (WALLS && wv->v[b][0][a]) fwall += (2.0 * (0.5 * (e_c + e_am)) * rvis) * wv->v[b][0][a][c];
            }
            if (!g.per[b] && ia[b] == g.n[b] - 1) {
                sd += 2.0 * (0.5 * (e_c + e_am)) * rvis;
                if (WALLS && wv->v[b][1][a]) fwall += (2.0 * (0.5 * (e_c + e_am)) * rvis) * wv->v[b][1][a][c];
            }
            // skew advection, b != a
            const int ibn = wrap_next(ia[b], g.n[b]);
            const double mph = hi >= 0 ? mflux_mix<DIM>(g, mx, u.a[b], b, hi, ibn) : 0.0;
            const int hiam = hi >= 0 ? nb_lo(g, hi, ia[a], a) : -1;   // c + e_b - e_a
            const double mpha = hi >= 0 ? mflux_mix<DIM>(g, mx, u.a[b], b, hiam, ibn) : 0.0;
            const double mp = 0.5 * (mph + mpha);
            const double mm = 0.5 * (mflux_mix<DIM>(g, mx, u.a[b], b, c, ia[b]) +
                                     mflux_mix<DIM>(g, mx, u.a[b], b, cam, ia[b]));
            const double uc = ua[c];
            const double up = hi >= 0 ? ua[hi] : -uc;
            const double um = lo >= 0 ? ua[lo] : -uc;
            nadv += CN ? mp * (up - uc) + mm * (uc - um) : mp * up - mm * um;
        }
    }
    nadv *= 0.5 * k.ih;
    const double st = mx.capillary(c, cam);
    double f = CN ? rf_new / k.dt * vk[c] - nadv - st - k.inv_We * ((pm[c] - pm[cam]) * k.ih)
                  : (0.5 * (rf_new + rf_old)) / k.dt * ua[c] - nadv - st;
    if (a == 1 && k.inv_Fr != 0.0) f -= rf_new * k.inv_Fr;     // g_hat = (0, -1, 0)
    if (WALLS) f += fwall;
    put(&s[c], sd);
    if (!coef_only) {
        put(&rhs[c], f);
        if (ustar) put(&ustar[c], ua[c]);   // null: the guess is written by k_velocity_guess
    }
}

// Set-up of every component at cell index c (the face of axis a at c for
// component a), one component after the other with the body above.
template <int DIM, typename Mix, bool WALLS = false>
__device__ inline void mom_setup_all_body(const Geo &g, const StepConst &k, const Mix &mx, const U3 &u,
                                          const MomOut &o, int c, const WallVel *wv = nullptr) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const W3 cs{{o.cs[a][0], o.cs[a][1], o.cs[a][2]}};
        mom_setup_body<DIM, Mix, WALLS, false, true>(g, k, a, mx, u, o.s[a], cs, o.rhs[a], o.ustar[a], 0, c, wv);
    }
}

template <int DIM>
__device__ inline void mom_setup_cell(const Geo &g, const StepConst &k, int a, const double *__restrict__ phi,
                                      const double *__restrict__ phin, const double *__restrict__ mu, const U3 &u,
                                      double *__restrict__ s, const W3 &cs, double *__restrict__ rhs,
                                      double *__restrict__ ustar, int coef_only, int c) {
    mom_setup_body<DIM>(g, k, a, mk_mix2(k, phi, phin, mu), u, s, cs, rhs, ustar, coef_only, c);
}

// S8 set-up: pressure coefficients 1/(rho_f h^2) from clamp(phi_new)
// (part & kPCoef; rho_out, when given, receives the cell density the
// coefficients are formed from), rhs = -(We/dt) D ustar (part & kPRhs).
template <int DIM, typename Mix>
__device__ inline void p_setup_body(const Geo &g, const StepConst &k, const Mix &mx, const U3 &us,
                                    double *__restrict__ s, const W3 &cs, double *__restrict__ rhs, int part, int c,
                                    double *__restrict__ rho_out = nullptr) {
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double rc = (part & kPCoef) ? mx.rho_new(c) : 0.0;
    double div = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b);
        const int hi = nb_hi(g, c, ia[b], b);
        if (part & kPCoef) {
            if (lo >= 0) {
                const double rl = mx.rho_new(lo);
                cs.a[b][c] = 1.0 / (0.5 * (rc + rl)) * k.ih2;
            } else {
                cs.a[b][c] = 0.0;
            }
        }
        const double flo = lo >= 0 ? us.a[b][c] : 0.0;
        const double fhi = hi >= 0 ? us.a[b][hi] : 0.0;
        div += fhi - flo;
    }
    if (part & kPCoef) {
        s[c] = 0.0;
        if (rho_out) rho_out[c] = rc;
    }
    if (part & kPRhs) rhs[c] = -(k.We / k.dt) * (div * k.ih);
}

template <int DIM>
__device__ inline void p_setup_cell(const Geo &g, const StepConst &k, const double *__restrict__ phin, const U3 &us,
                                    double *__restrict__ s, const W3 &cs, double *__restrict__ rhs, int part, int c) {
    p_setup_body<DIM>(g, k, mk_mix2(k, phin, phin, phin), us, s, cs, rhs, part, c);
}

// S9: u = ustar - (dt/We) G p / rho_f; phi = phi_new
template <int DIM, typename Mix>
__device__ inline void project_body(const Geo &g, const StepConst &k, const Mix &mx, const U3 &us,
                                    const double *__restrict__ p, const W3 &u, int c) {
    int i, j, kk;
    if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
    const int ia[3] = {i, j, kk};
    const double rc = mx.rho_new(c);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lo = nb_lo(g, c, ia[a], a);
        double v = 0.0;
        if (lo >= 0) {
            const double rf = 0.5 * (rc + mx.rho_new(lo));
            v = us.a[a][c] - (k.dt * k.inv_We) * ((p[c] - p[lo]) * k.ih) / rf;
        }
        u.a[a][c] = v;
    }
}

template <int DIM>
__device__ inline void project_cell(const Geo &g, const StepConst &k, const double *__restrict__ phin, const U3 &us,
                                    const double *__restrict__ p, double *__restrict__ phi, const W3 &u, int c) {
    project_body<DIM>(g, k, mk_mix2(k, phin, phin, phin), us, p, u, c);
    phi[c] = phin[c];
}

}  // namespace chns
