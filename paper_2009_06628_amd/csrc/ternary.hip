// Kernels of the three-phase step (nphases = 3, gfx950).  The paper's model
// is two-phase; the three-phase extension reads its binary free-energy
// density into the Boyer-Lapuerta construction:
//   phases i = 1, 2, 3 with c_i = (1 + phi_i)/2 and sum_i c_i = 1; the state
//   holds phi_1, phi_2 and phi_3 = -1 - phi_1 - phi_2 is implied;
//   E_free = (1/Cn) sum_i (Sigma_i/2) int psi(phi_i) + Cn^2/2 |grad phi_i|^2,
//   Sigma_i = sigma_ij + sigma_ik - sigma_jk;
//   mu~_i = psi'(phi_i) - Cn^2 lap phi_i - w_i Lambda, Lambda = sum_j psi'(phi_j),
//   w_i = Sigma_T / (3 Sigma_i), 3 / Sigma_T = sum_j 1 / Sigma_j (sum_i mu~_i = 0);
//   d phi_i/dt + div(u phi_i) = kM lap mu~_i (the paper's CH equation per phase);
//   rho = sum_i rho_i clamp(c_i, 0, 1), eta likewise (pull-back per phase);
//   J = -(kM/2) sum_i rho_i grad mu~_i, m = rho_lin u + J;
//   capillary force -(1/(2 Cn)) sum_i Sigma_i phi_i grad mu~_i.
// For a pair i|j with the third phase absent all of this is the paper's
// binary model with 1/We = sigma_ij.  The step (T1..T9) is the binary step
// S1..S9 per phase with Lambda taken at t^n; the momentum, pressure and
// projection kernels are the binary per-cell bodies with this mixture.
#include "stepdev.h"

namespace chns {

// Five cell arrays written by one kernel.
struct W5 {
    double *a[5];
};

// Mixture policy of the three-phase model (see stepdev.h for the interface).
struct Mix3 {
    static constexpr bool kStoredFlux = false;
    double rho[3], eta[3];
    double jc[2];     // (kM/2)(rho_i - rho_3), i = 1, 2
    double cap[3];    // Sigma_i / (2 Cn)
    double ih;
    const double *phi1, *phi2;     // phi^n
    const double *phin1, *phin2;   // phi^{n+1}
    const double *mu1, *mu2;       // mu~^{n+1}
    __device__ static double c01(double p) { return fmin(fmax(0.5 * (1.0 + p), 0.0), 1.0); }
    __device__ static double mixc(const double q[3], double p1, double p2) {
        const double p3 = -1.0 - p1 - p2;
        double out = q[0] * c01(p1);
        out = out + q[1] * c01(p2);
        return out + q[2] * c01(p3);
    }
    __device__ double rho_lin(int e) const {
        const double p1 = phi1[e], p2 = phi2[e], p3 = -1.0 - p1 - p2;
        double out = rho[0] * (0.5 * (1.0 + p1));
        out = out + rho[1] * (0.5 * (1.0 + p2));
        return out + rho[2] * (0.5 * (1.0 + p3));
    }
    __device__ double rho_new(int e) const { return mixc(rho, phin1[e], phin2[e]); }
    __device__ double rho_old(int e) const { return mixc(rho, phi1[e], phi2[e]); }
    __device__ double eta_new(int e) const { return mixc(eta, phin1[e], phin2[e]); }
    __device__ double mflux_face(double ub, int f, int lo) const {
        const double J = jc[0] * ((mu1[f] - mu1[lo]) * ih) + jc[1] * ((mu2[f] - mu2[lo]) * ih);
        return (0.5 * (rho_lin(f) + rho_lin(lo))) * ub - J;
    }
    __device__ double capillary(int c, int cam) const {
        const double a1 = 0.5 * (phi1[c] + phi1[cam]), a2 = 0.5 * (phi2[c] + phi2[cam]);
        const double a3 = 0.5 * ((-1.0 - phi1[c] - phi2[c]) + (-1.0 - phi1[cam] - phi2[cam]));
        const double g1 = (mu1[c] - mu1[cam]) * ih, g2 = (mu2[c] - mu2[cam]) * ih;
        const double g3 = ((-mu1[c] - mu2[c]) - (-mu1[cam] - mu2[cam])) * ih;
        return cap[0] * a1 * g1 + cap[1] * a2 * g2 + cap[2] * a3 * g3;
    }
};

// The same mixture read from cell fields computed once per step by
// k_phi_update3 (rho^{n+1}, rho^n with the pull-back, eta^{n+1}, rho_lin^n and
// chi = (kM/2) sum_{i=1,2} (rho_i - rho_3) mu~_i, so that J = -G chi): the
// momentum set-up evaluates the mass flux on up to 11 faces per cell and
// component, and the three-phase maps are the costly part of it.
struct MixPre {
    static constexpr bool kStoredFlux = false;
    const double *rn, *ro, *en, *rl, *chi;
    double ih;
    double cap[3];
    const double *phi1, *phi2, *mu1, *mu2;
    __device__ double rho_new(int e) const { return rn[e]; }
    __device__ double rho_old(int e) const { return ro[e]; }
    __device__ double eta_new(int e) const { return en[e]; }
    __device__ double mflux_face(double ub, int f, int lo) const {
        return (0.5 * (rl[f] + rl[lo])) * ub - (chi[f] - chi[lo]) * ih;
    }
    __device__ double capillary(int c, int cam) const {
        const double a1 = 0.5 * (phi1[c] + phi1[cam]), a2 = 0.5 * (phi2[c] + phi2[cam]);
        const double a3 = 0.5 * ((-1.0 - phi1[c] - phi2[c]) + (-1.0 - phi1[cam] - phi2[cam]));
        const double g1 = (mu1[c] - mu1[cam]) * ih, g2 = (mu2[c] - mu2[cam]) * ih;
        const double g3 = ((-mu1[c] - mu2[c]) - (-mu1[cam] - mu2[cam])) * ih;
        return cap[0] * a1 * g1 + cap[1] * a2 * g2 + cap[2] * a3 * g3;
    }
};

// The same with the step's face mass fluxes read from m[b] (written once per
// step by k_mflux3 with MixPre's expression): the momentum set-up evaluates
// the flux on 11 faces per face and component in 3D, five loads each.
struct MixPreFlux : MixPre {
    static constexpr bool kStoredFlux = true;
    const double *m[3];
};

static Mix3 mk_mix3(const StepConst &k, const TernConst &t, const double *phi1, const double *phi2,
                    const double *phin1, const double *phin2, const double *mu1, const double *mu2) {
    Mix3 m;
    for (int i = 0; i < 3; ++i) {
        m.rho[i] = t.rho[i];
        m.eta[i] = t.eta[i];
        m.cap[i] = (0.5 / k.Cn) * t.Sg[i];
    }
    for (int i = 0; i < 2; ++i) m.jc[i] = (0.5 * k.kM) * (t.rho[i] - t.rho[2]);
    m.ih = k.ih;
    m.phi1 = phi1;
    m.phi2 = phi2;
    m.phin1 = phin1;
    m.phin2 = phin2;
    m.mu1 = mu1;
    m.mu2 = mu2;
    return m;
}

__device__ inline double lambda3(double p1, double p2) {
    const double p3 = -1.0 - p1 - p2;
    return (dpsi(p1) + dpsi(p2)) + dpsi(p3);
}

// T1: r_i = phi_i - dt D(u A phi_i) + dt kM L(psi'(phi_i) - S phi_i - w_i Lambda),
// i = 1, 2; phihat_i = phi_i (initial guess of an iterative S2 solve)
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_ch_rhs3(Geo g, StepConst k, TernConst t, const double *__restrict__ phi1,
                                                    const double *__restrict__ phi2, U3 u, double *__restrict__ r1,
                                                    double *__restrict__ r2, double *__restrict__ ph1,
                                                    double *__restrict__ ph2) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double p1 = phi1[c], p2 = phi2[c];
        const double lc = lambda3(p1, p2);
        const double g1c = (dpsi(p1) - k.S * p1) - t.w[0] * lc, g2c = (dpsi(p2) - k.S * p2) - t.w[1] * lc;
        double div1 = 0.0, div2 = 0.0, lap1 = 0.0, lap2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            double f1lo = 0.0, f1hi = 0.0, f2lo = 0.0, f2hi = 0.0;
            if (lo >= 0) {
                const double q1 = phi1[lo], q2 = phi2[lo], l = lambda3(q1, q2);
                const double ua = u.a[a][c];
                f1lo = ua * (0.5 * (q1 + p1));
                f2lo = ua * (0.5 * (q2 + p2));
                lap1 += ((dpsi(q1) - k.S * q1) - t.w[0] * l) - g1c;
                lap2 += ((dpsi(q2) - k.S * q2) - t.w[1] * l) - g2c;
            }
            if (hi >= 0) {
                const double q1 = phi1[hi], q2 = phi2[hi], l = lambda3(q1, q2);
                const double ua = u.a[a][hi];
                f1hi = ua * (0.5 * (p1 + q1));
                f2hi = ua * (0.5 * (p2 + q2));
                lap1 += ((dpsi(q1) - k.S * q1) - t.w[0] * l) - g1c;
                lap2 += ((dpsi(q2) - k.S * q2) - t.w[1] * l) - g2c;
            }
            div1 += f1hi - f1lo;
            div2 += f2hi - f2lo;
        }
        r1[c] = p1 - k.dt * (div1 * k.ih) + k.dt * k.kM * (lap1 * k.ih2);
        r2[c] = p2 - k.dt * (div2 * k.ih) + k.dt * k.kM * (lap2 * k.ih2);
        if (ph1) {   // the guesses of iterative T2 solves (null: direct solve)
            ph1[c] = p1;
            ph2[c] = p2;
        }
    }
}

// T3: mu~_i = psi'(phi_i) + S (phihat_i - phi_i) - Cn^2 L phihat_i - w_i Lambda
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mu3(Geo g, StepConst k, TernConst t, const double *__restrict__ phi1,
                                                const double *__restrict__ phi2, const double *__restrict__ ph1,
                                                const double *__restrict__ ph2, double *__restrict__ mu1,
                                                double *__restrict__ mu2) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double x1 = ph1[c], x2 = ph2[c];
        double lap1 = 0.0, lap2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            if (lo >= 0) {
                lap1 += ph1[lo] - x1;
                lap2 += ph2[lo] - x2;
            }
            if (hi >= 0) {
                lap1 += ph1[hi] - x1;
                lap2 += ph2[hi] - x2;
            }
        }
        const double p1 = phi1[c], p2 = phi2[c];
        const double lc = lambda3(p1, p2);
        mu1[c] = dpsi(p1) + k.S * (x1 - p1) - k.Cn * k.Cn * (lap1 * k.ih2) - t.w[0] * lc;
        mu2[c] = dpsi(p2) + k.S * (x2 - p2) - k.Cn * k.Cn * (lap2 * k.ih2) - t.w[1] * lc;
    }
}

// T4: phi_i^{n+1} = phi_i - dt D(u A phi_i - kM G mu~_i): each face flux is
// evaluated identically by both of its cells, so every phase mass (the
// implied third one too) telescopes to round-off
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_phi_update3(Geo g, StepConst k, const double *__restrict__ phi1,
                                                        const double *__restrict__ phi2, U3 u,
                                                        const double *__restrict__ mu1,
                                                        const double *__restrict__ mu2, double *__restrict__ pn1,
                                                        double *__restrict__ pn2, Mix3 mx, W5 fields) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double p1 = phi1[c], p2 = phi2[c], m1 = mu1[c], m2 = mu2[c];
        double div1 = 0.0, div2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            if (lo >= 0) {
                const double ua = u.a[a][c];
                div1 -= phi_face_flux(k, ua, phi1[lo], p1, mu1[lo], m1);
                div2 -= phi_face_flux(k, ua, phi2[lo], p2, mu2[lo], m2);
            }
            if (hi >= 0) {
                const double ua = u.a[a][hi];
                div1 += phi_face_flux(k, ua, p1, phi1[hi], m1, mu1[hi]);
                div2 += phi_face_flux(k, ua, p2, phi2[hi], m2, mu2[hi]);
            }
        }
        const double q1 = p1 - k.dt * (div1 * k.ih), q2 = p2 - k.dt * (div2 * k.ih);
        // seven arrays written past the L2 (128^3: 71 -> 55 us)
        st_nt(&pn1[c], q1);
        st_nt(&pn2[c], q2);
        // the cell fields of MixPre: rho^{n+1}, rho^n (pull-back), eta^{n+1},
        // rho_lin^n and chi = (kM/2) sum_{i=1,2} (rho_i - rho_3) mu~_i
        st_nt(&fields.a[0][c], Mix3::mixc(mx.rho, q1, q2));
        st_nt(&fields.a[1][c], Mix3::mixc(mx.rho, p1, p2));
        st_nt(&fields.a[2][c], Mix3::mixc(mx.eta, q1, q2));
        st_nt(&fields.a[3][c], mx.rho_lin(c));
        st_nt(&fields.a[4][c], mx.jc[0] * m1 + mx.jc[1] * m2);
    }
}

// T5-T7 set-up of every component (the binary body with the three-phase mixture)
template <int DIM, bool WALLS>
__global__ void __launch_bounds__(kBlock) k_mom_setup3_all(Geo g, StepConst k, MixPreFlux mx, U3 u, MomOut o,
                                                           WallVel wv) {
    CELL_LOOP(g.N) mom_setup_all_body<DIM, MixPreFlux, WALLS>(g, k, mx, u, o, c, &wv);
}

// The face mass fluxes m_b = A_b(rho_lin) u_b - G_b chi of the step on every
// face (0 on the stored wall faces).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mflux3(Geo g, MixPre mx, U3 u, W3 m) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
#pragma unroll
        for (int b = 0; b < DIM; ++b) m.a[b][c] = mflux_mix<DIM>(g, mx, u.a[b], b, c, ia[b]);
    }
}

// T8 set-up
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_p_setup3(Geo g, StepConst k, MixPre mx, U3 us, double *__restrict__ s,
                                                     W3 cs, double *__restrict__ rhs, int part,
                                                     double *__restrict__ rho_out) {
    CELL_LOOP(g.N) p_setup_body<DIM>(g, k, mx, us, s, cs, rhs, part, c, rho_out);
}

// T9: projection; phi_i = phi_i^{n+1}
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_project3(Geo g, StepConst k, MixPre mx, U3 us, const double *__restrict__ p,
                                                     W3 u, const double *__restrict__ pn1, const double *__restrict__ pn2,
                                                     double *__restrict__ phi1, double *__restrict__ phi2) {
    CELL_LOOP(g.N) {
        project_body<DIM>(g, k, mx, us, p, u, c);
        phi1[c] = pn1[c];
        phi2[c] = pn2[c];
    }
}

// Diagnostics: sums of c_1, c_2, c_3, kinetic, sum_i (Sigma_i/2) psi(phi_i),
// sum_i (Sigma_i/2) sum_a (G_a phi_i)^2, gravity potential; max|u|, max|D u|
constexpr int kNDiag3 = 9;

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_diag3(Geo g, StepConst k, TernConst t, const double *__restrict__ phi1,
                                                  const double *__restrict__ phi2, U3 u, double *part,
                                                  unsigned int *counter, double *out) {
    __shared__ double lds[kBlock / kWave];
    double acc[kNDiag3] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double hs[3] = {0.5 * t.Sg[0], 0.5 * t.Sg[1], 0.5 * t.Sg[2]};
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double p[3] = {phi1[c], phi2[c], -1.0 - phi1[c] - phi2[c]};
        const double rc = Mix3::mixc(t.rho, p[0], p[1]);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            acc[q] += 0.5 * (1.0 + p[q]);
            acc[4] += hs[q] * (0.25 * (p[q] * p[q] - 1.0) * (p[q] * p[q] - 1.0));
        }
        if (k.inv_Fr != 0.0) acc[6] += rc * ((j + 0.5) * k.h);
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            const double uc = u.a[a][c];
            if (lo >= 0) {
                const double q1 = phi1[lo], q2 = phi2[lo];
                const double rf = 0.5 * (rc + Mix3::mixc(t.rho, q1, q2));
                acc[3] += 0.5 * rf * uc * uc;
                const double d1 = (p[0] - q1) * k.ih, d2 = (p[1] - q2) * k.ih;
                const double d3 = (p[2] - (-1.0 - q1 - q2)) * k.ih;
                acc[5] += hs[0] * (d1 * d1) + hs[1] * (d2 * d2) + hs[2] * (d3 * d3);
                acc[7] = fmax(acc[7], fabs(uc));
            }
            div += (hi >= 0 ? u.a[a][hi] : 0.0) - (lo >= 0 ? uc : 0.0);
        }
        acc[8] = fmax(acc[8], fabs(div * k.ih));
    }
#pragma unroll
    for (int q = 0; q < kNDiag3; ++q) {
        double v = (q >= 7) ? block_max(acc[q], lds) : block_sum(acc[q], lds);
        if (threadIdx.x == 0) part[q * kMaxBlocks + blockIdx.x] = v;
    }
    if (last_block(counter)) {
        for (int q = 0; q < kNDiag3; ++q) {
            double v = 0.0;
            for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
                const double x = ((volatile double *)part)[q * kMaxBlocks + b];
                v = (q >= 7) ? fmax(v, x) : v + x;
            }
            v = (q >= 7) ? block_max(v, lds) : block_sum(v, lds);
            if (threadIdx.x == 0) out[q] = v;
        }
        if (threadIdx.x == 0) *counter = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)
#define DISPATCH(cls, arrays, dim, kern, n, st, ...)                            \
    do {                                                                        \
        const double bytes_ = 8.0 * (double)(arrays) * (double)(n);              \
        if ((dim) == 2)                                                         \
            LAUNCH(cls, bytes_, (kern<2>), n, st, __VA_ARGS__);                 \
        else                                                                    \
            LAUNCH(cls, bytes_, (kern<3>), n, st, __VA_ARGS__);                 \
    } while (0)

TernConst tern_const_of(const chns_props &p) {
    TernConst t;
    const double s12 = p.sigma3[0], s13 = p.sigma3[1], s23 = p.sigma3[2];
    t.Sg[0] = s12 + s13 - s23;
    t.Sg[1] = s12 + s23 - s13;
    t.Sg[2] = s13 + s23 - s12;
    const double inv_sum = 1.0 / t.Sg[0] + 1.0 / t.Sg[1] + 1.0 / t.Sg[2];
    for (int i = 0; i < 3; ++i) {
        t.rho[i] = p.rho3[i];
        t.eta[i] = p.eta3[i];
        t.w[i] = (1.0 / t.Sg[i]) / inv_sum;
    }
    return t;
}

void launch_ch_rhs3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                    const double *const u[3], double *r1, double *r2, double *hat1, double *hat2, hipStream_t st) {
    DISPATCH(K_CH_RHS, (hat1 ? 6 : 4) + dim, dim, k_ch_rhs3, g.N, st, g, k, t, ph.phi[0], ph.phi[1], mk_u3(u), r1, r2,
             hat1, hat2);
}

void launch_mu3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph, const double *hat1,
                const double *hat2, hipStream_t st) {
    DISPATCH(K_MU, 6, dim, k_mu3, g.N, st, g, k, t, ph.phi[0], ph.phi[1], hat1, hat2, ph.mu[0], ph.mu[1]);
}

static Mix3 mix_of(const StepConst &k, const TernConst &t, const Phases3 &ph) {
    return mk_mix3(k, t, ph.phi[0], ph.phi[1], ph.phin[0], ph.phin[1], ph.mu[0], ph.mu[1]);
}

void launch_phi_update3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                        const double *const u[3], hipStream_t st) {
    const W5 f{{ph.mix[0], ph.mix[1], ph.mix[2], ph.mix[3], ph.mix[4]}};
    // phi_i, mu_i, u[d] read; phi_i^{n+1} and the five mixture fields written
    DISPATCH(K_PHI_UPDATE, 4 + dim + 7, dim, k_phi_update3, g.N, st, g, k, ph.phi[0], ph.phi[1], mk_u3(u), ph.mu[0],
             ph.mu[1], ph.phin[0], ph.phin[1], mix_of(k, t, ph), f);
}

static MixPre pre_of(const StepConst &k, const TernConst &t, const Phases3 &ph) {
    MixPre m;
    m.rn = ph.mix[0];
    m.ro = ph.mix[1];
    m.en = ph.mix[2];
    m.rl = ph.mix[3];
    m.chi = ph.mix[4];
    m.ih = k.ih;
    for (int i = 0; i < 3; ++i) m.cap[i] = (0.5 / k.Cn) * t.Sg[i];
    m.phi1 = ph.phi[0];
    m.phi2 = ph.phi[1];
    m.mu1 = ph.mu[0];
    m.mu2 = ph.mu[1];
    return m;
}

void launch_mom_setup3_all(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                           const double *const u[3], const MomOut &o, double *const m[3], hipStream_t st,
                           const WallVel *wv) {
    WallVel w{};
    if (wv) w = *wv;
    const MixPre pre = pre_of(k, t, ph);
    const dim3 grid(grid_for(g.N)), block(kBlock);
    // face fluxes: rho_lin, chi and u[d] read, m[d] written
    if (dim == 2)
        TLAUNCH(K_MOM_SETUP, 8.0 * (2 + 2 * dim) * g.N, (k_mflux3<2>), grid, block, st, g, pre, mk_u3(u), mk_w3(m));
    else
        TLAUNCH(K_MOM_SETUP, 8.0 * (2 + 2 * dim) * g.N, (k_mflux3<3>), grid, block, st, g, pre, mk_u3(u), mk_w3(m));
    MixPreFlux mx;
    static_cast<MixPre &>(mx) = pre;
    for (int b = 0; b < 3; ++b) mx.m[b] = m[b];
    // rho^{n+1}, rho^n, eta^{n+1}, phi_1, phi_2, mu_1, mu_2, m[d] and u[d] read; s, cs[d], rhs, ustar written
    // per component
    const double bytes = 8.0 * (7 + 2 * dim + dim * (3 + dim) - (o.ustar[0] ? 0 : dim)) * g.N;
    if (dim == 2) {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup3_all<2, true>), grid, block, st, g, k, mx, mk_u3(u), o, w);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup3_all<2, false>), grid, block, st, g, k, mx, mk_u3(u), o, w);
    } else {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup3_all<3, true>), grid, block, st, g, k, mx, mk_u3(u), o, w);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_mom_setup3_all<3, false>), grid, block, st, g, k, mx, mk_u3(u), o, w);
    }
}

void launch_p_setup3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                     const double *const ustar[3], double *s, double *const cs[3], double *rhs, hipStream_t st,
                     int part, double *rho_out) {
    const int words = (part & kPCoef ? 2 + dim + (rho_out ? 1 : 0) : 0) + (part & kPRhs ? 1 + dim : 0);
    DISPATCH(K_P_SETUP, words, dim, k_p_setup3, g.N, st, g, k, pre_of(k, t, ph), mk_u3(ustar), s, mk_w3(cs), rhs,
             part, rho_out);
}

void launch_project3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const Phases3 &ph,
                     const double *const ustar[3], const double *p, double *phi1, double *phi2, double *const u[3],
                     hipStream_t st) {
    DISPATCH(K_PROJECT, 6 + 2 * dim, dim, k_project3, g.N, st, g, k, pre_of(k, t, ph), mk_u3(ustar), p, mk_w3(u),
             ph.phin[0], ph.phin[1], phi1, phi2);
}

void launch_diagnostics3(int dim, const Geo &g, const StepConst &k, const TernConst &t, const double *phi1,
                         const double *phi2, const double *const u[3], double *part, unsigned int *counter,
                         double *out, hipStream_t st) {
    DISPATCH(K_DIAG, 2 + dim, dim, k_diag3, g.N, st, g, k, t, phi1, phi2, mk_u3(u), part, counter, out);
}

}  // namespace chns
