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
    CELL_LOOP(g.N) {
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
        phihat[c] = pc;
    }
}

// ---------------------------------------------------------------------------
// S3
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mu(Geo g, StepConst k, const double *__restrict__ phi,
                                               const double *__restrict__ ph, double *__restrict__ mu) {
    CELL_LOOP(g.N) {
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
}

// ---------------------------------------------------------------------------
// S4: flux-form update; both cells of a face evaluate its flux with the same
// operands in the same order, so sum(phi) telescopes to round-off.
// ---------------------------------------------------------------------------
__device__ inline double phi_face_flux(const StepConst &k, double uf, double pl, double pu, double ml, double mu_) {
    return uf * (0.5 * (pl + pu)) - k.kM * ((mu_ - ml) * k.ih);
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_phi_update(Geo g, StepConst k, const double *__restrict__ phi, U3 u,
                                                       const double *__restrict__ mu, double *__restrict__ phin) {
    CELL_LOOP(g.N) {
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
}

// ---------------------------------------------------------------------------
// S5-S7 set-up for component a
// ---------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_mom_setup(Geo g, StepConst k, int a, const double *__restrict__ phi,
                                                      const double *__restrict__ phin, const double *__restrict__ mu,
                                                      U3 u, double *__restrict__ s, W3 cs, double *__restrict__ rhs,
                                                      double *__restrict__ ustar, int coef_only) {
    const double rvis = k.inv_Re * k.ih2;
    CELL_LOOP(g.N) {
        int i, j, kk;
        if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double *ua = u.a[a];
        if (!g.per[a] && ia[a] == 0) {
            // wall face of a walled axis: decoupled identity row, u = 0
            s[c] = 1.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) cs.a[b][c] = 0.0;
            if (!coef_only) {
                rhs[c] = 0.0;
                ustar[c] = 0.0;
            }
            continue;
        }
        const int cam = nb_lo(g, c, ia[a], a);   // cell c - e_a
        auto eta_of = [&](int e) { return k.gamma * pullback(phin[e]) + k.xi; };
        const double rf_new = 0.5 * ((k.alpha * pullback(phin[c]) + k.beta) + (k.alpha * pullback(phin[cam]) + k.beta));
        const double rf_old = 0.5 * ((k.alpha * pullback(phi[c]) + k.beta) + (k.alpha * pullback(phi[cam]) + k.beta));
        const double e_c = eta_of(c), e_am = eta_of(cam);
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
                cs.a[b][c] = w;
                // skew advection, b == a
                const double m_c = mflux<DIM>(g, k, phi, mu, u.a[a], a, c, ia[a]);
                const double m_hi = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[a], a, hi, wrap_next(ia[a], g.n[a])) : 0.0;
                const double m_lo = mflux<DIM>(g, k, phi, mu, u.a[a], a, lo, wrap_prev(ia[a], g.n[a]));
                const double mp = 0.5 * (m_c + m_hi), mm = 0.5 * (m_lo + m_c);
                const double up = hi >= 0 ? ua[hi] : 0.0;
                const double um = (!g.per[a] && ia[a] == 1) ? 0.0 : ua[lo];   // wall face
                nadv += mp * up - mm * um;
            } else {
                // viscous coupling through the edge between faces c - e_b and c
                if (lo >= 0) {
                    const int lam = nb_lo(g, lo, ia[a], a);   // c - e_b - e_a
                    const double ee = 0.25 * (((e_c + e_am) + eta_of(lo)) + eta_of(lam));
                    cs.a[b][c] = (!g.per[b] && ia[b] == 0) ? 0.0 : ee * rvis;
                } else {
                    cs.a[b][c] = 0.0;
                }
                if (!g.per[b] && ia[b] == 0) sd += 2.0 * (0.5 * (e_c + e_am)) * rvis;
                if (!g.per[b] && ia[b] == g.n[b] - 1) sd += 2.0 * (0.5 * (e_c + e_am)) * rvis;
                // skew advection, b != a
                const int ibn = wrap_next(ia[b], g.n[b]);
                const double mph = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[b], b, hi, ibn) : 0.0;
                const int hiam = hi >= 0 ? nb_lo(g, hi, ia[a], a) : -1;   // c + e_b - e_a
                const double mpha = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[b], b, hiam, ibn) : 0.0;
                const double mp = 0.5 * (mph + mpha);
                const double mm = 0.5 * (mflux<DIM>(g, k, phi, mu, u.a[b], b, c, ia[b]) +
                                         mflux<DIM>(g, k, phi, mu, u.a[b], b, cam, ia[b]));
                const double uc = ua[c];
                const double up = hi >= 0 ? ua[hi] : -uc;
                const double um = lo >= 0 ? ua[lo] : -uc;
                nadv += mp * up - mm * um;
            }
        }
        nadv *= 0.5 * k.ih;
        const double st = (k.inv_We / k.Cn) * (0.5 * (phi[c] + phi[cam])) * ((mu[c] - mu[cam]) * k.ih);
        double f = (0.5 * (rf_new + rf_old)) / k.dt * ua[c] - nadv - st;
        if (a == 1 && k.inv_Fr != 0.0) f -= rf_new * k.inv_Fr;     // g_hat = (0, -1, 0)
        s[c] = sd;
        if (!coef_only) {
            rhs[c] = f;
            ustar[c] = ua[c];
        }
    }
}

// ---------------------------------------------------------------------------
// S8 set-up
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_p_setup(Geo g, StepConst k, const double *__restrict__ phin, U3 us,
                                                    double *__restrict__ s, W3 cs, double *__restrict__ rhs) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double rc = k.alpha * pullback(phin[c]) + k.beta;
        double div = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int lo = nb_lo(g, c, ia[b], b);
            const int hi = nb_hi(g, c, ia[b], b);
            if (lo >= 0) {
                const double rl = k.alpha * pullback(phin[lo]) + k.beta;
                cs.a[b][c] = 1.0 / (0.5 * (rc + rl)) * k.ih2;
            } else {
                cs.a[b][c] = 0.0;
            }
            const double flo = lo >= 0 ? us.a[b][c] : 0.0;
            const double fhi = hi >= 0 ? us.a[b][hi] : 0.0;
            div += fhi - flo;
        }
        s[c] = 0.0;
        rhs[c] = -(k.We / k.dt) * (div * k.ih);
    }
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
    CELL_LOOP(g.N) {
        int i, j, kk;
        if (DIM == 2) cell_coords2(g, c, i, j, kk); else cell_coords(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double pn = phin[c];
        const double rc = k.alpha * pullback(pn) + k.beta;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            double v = 0.0;
            if (lo >= 0) {
                const double rf = 0.5 * (rc + (k.alpha * pullback(phin[lo]) + k.beta));
                v = us.a[a][c] - (k.dt * k.inv_We) * ((p[c] - p[lo]) * k.ih) / rf;
            }
            u.a[a][c] = v;
        }
        phi[c] = pn;
    }
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
    DISPATCH(K_CH_RHS, 3 + dim, dim, k_ch_rhs, g.N, st, g, k, phi, mk_u3(u), r, phihat);
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
                      double *ustar, hipStream_t st, int coef_only) {
    DISPATCH(K_MOM_SETUP, 6 + 2 * dim, dim, k_mom_setup, g.N, st, g, k, a, phi, phi_new, mu, mk_u3(u), s, mk_w3(cs), rhs,
             ustar, coef_only);
}
void launch_p_setup(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    double *s, double *const cs[3], double *rhs, hipStream_t st) {
    DISPATCH(K_P_SETUP, 3 + 2 * dim, dim, k_p_setup, g.N, st, g, k, phi_new, mk_u3(ustar), s, mk_w3(cs), rhs);
}
void launch_p_coef_from_rho(int dim, const Geo &g, double ih2, const double *rho, double *s, double *const cs[3],
                            hipStream_t st) {
    DISPATCH(K_P_SETUP, 2 + dim, dim, k_p_coef_rho, g.N, st, g, ih2, rho, s, mk_w3(cs));
}
void launch_project(int dim, const Geo &g, const StepConst &k, const double *phi_new, const double *const ustar[3],
                    const double *p, double *phi, double *const u[3], hipStream_t st) {
    DISPATCH(K_PROJECT, 3 + 2 * dim, dim, k_project, g.N, st, g, k, phi_new, mk_u3(ustar), p, phi, mk_w3(u));
}
void launch_fill_ch(int dim, const Geo &g, double csval, double *s, double *const cs[3], hipStream_t st) {
    DISPATCH(K_MG_SETUP, 1 + dim, dim, k_fill_ch, g.N, st, g, csval, s, mk_w3(cs));
}
void launch_diagnostics(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                        double *part, unsigned int *counter, double *out, hipStream_t st) {
    DISPATCH(K_DIAG, 1 + dim, dim, k_diag, g.N, st, g, k, phi, mk_u3(u), part, counter, out);
}

}  // namespace chns
