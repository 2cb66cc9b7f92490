// Discrete adjoint of one split CHNS step (gfx950), FP64.
//
// Reverse-mode transposition of S9 .. S1 with the forward intermediates of
// the same step (recomputed by the caller).  Notation: phi = phi^n,
// u = u^n, phin = phi^{n+1}, p = pressure, mu = mu^{n+1}, u* = predictor;
// adjoints carry a "bar".  Parameters: k = 1/(Pe Cn) (CH mobility and the
// consistent flux J / Pe = -alpha k G mu) and s_t = 1/(We Cn) (potential-form
// surface tension).  We does not reach u^{n+1} through the projection (the
// pressure scales with We and cancels), so the loss sees sigma only through
// k and s_t.
//
// Every face-to-cell scatter of the transpose is written as a gather over
// the faces that reference a cell, so no kernel has write races; parameter
// derivatives are deterministic block partials summed in a fixed order.
// The elliptic adjoints reuse the forward operators (all symmetric): the
// pressure pseudo-inverse with mean-zero projection, the momentum operator
// per component, and the CH operator.
//
// Stages of the reverse sweep (labels used below):
//   A1  pbar = (dt/We) D(ubar'/rho_f')                    (reverse of S9)
//   A2  P zeta = pbar (mean zero)                         (reverse of S8, host)
//   A3  ustar_bar, rho_f' bar; zero the accumulators
//   A4  K_a nu_a = ustar_bar_a per component               (host)
//   A5  momentum operator / right-hand side adjoints on the faces of a
//   A6  gathers of A5 onto eta (cells) and the mass flux m (faces)
//   A7  density / viscosity maps and the pull-back -> phi' and phi
//   A8  flux of S4 and the mass flux -> G mu, u, A(phi)
//   A9  mu_bar = G^T (G mu)_bar; S3's psi'' term
//   A10 right-hand side of the CH adjoint solve
//   A11 M omega = chr                                      (host)
//   A12 S2 / S1 parameter terms; phi_bar += omega + ...
//   A14 advective flux of S1 and S4 -> u, A(phi)
//   A15 A(phi)_bar -> phi
// Parameter partials are block sums (regions 0..2: k, 3..5: s_t per axis).
#include "adjoint.h"
#include "stepdev.h"

namespace chns {

__device__ inline double rho_of(const StepConst &k, double p) { return k.alpha * pullback(p) + k.beta; }
__device__ inline double eta_of(const StepConst &k, double p) { return k.gamma * pullback(p) + k.xi; }

// (L q)(c) with walls Neumann, q given by a functor
template <int DIM, typename F>
__device__ inline double lap_c(const Geo &g, int c, const int ia[3], double ih2, F q) {
    const double qc = q(c);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lo = nb_lo(g, c, ia[a], a), hi = nb_hi(g, c, ia[a], a);
        if (lo >= 0) acc += q(lo) - qc;
        if (hi >= 0) acc += q(hi) - qc;
    }
    return acc * ih2;
}

__device__ inline double block_partial(double v, double *lds) { return block_sum(v, lds); }

// ---------------------------------------------------------------------------
// A1: pbar = (dt/We) D(ubar' / rho_f')
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_p_rhs(Geo g, StepConst k, const double *__restrict__ phin, U3 ub,
                                                      double *__restrict__ pbar, double *__restrict__ zeta) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        const double rc = rho_of(k, phin[c]);
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a), hi = nb_hi(g, c, ia[a], a);
            const double wlo = lo >= 0 ? ub.a[a][c] / (0.5 * (rc + rho_of(k, phin[lo]))) : 0.0;
            const double whi = hi >= 0 ? ub.a[a][hi] / (0.5 * (rho_of(k, phin[hi]) + rc)) : 0.0;
            div += whi - wlo;
        }
        pbar[c] = (k.dt * k.inv_We) * (div * k.ih);
        zeta[c] = 0.0;   // zero initial guess of the adjoint pressure solve
    }
}

// ---------------------------------------------------------------------------
// A3: ustar_bar = ubar' + (We/dt) G zeta;
//     rho_f'_bar = [ubar' (dt/We) G p + G zeta G p] / rho_f'^2;
//     all other accumulators set to zero.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_proj_faces(Geo g, StepConst k, const double *__restrict__ phin,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ zeta, U3 ub, W3 usb, W3 rfnb,
                                                           W3 rfob, W3 aphib, W3 gmub, W3 mb, W3 nu, W3 uout,
                                                           double *__restrict__ etab) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        const double rc = rho_of(k, phin[c]);
        etab[c] = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            double us = 0.0, rb = 0.0;
            if (lo >= 0) {
                const double rf = 0.5 * (rc + rho_of(k, phin[lo]));
                const double Gp = (p[c] - p[lo]) * k.ih;
                const double Gz = (zeta[c] - zeta[lo]) * k.ih;
                us = ub.a[a][c] + (k.We / k.dt) * Gz;
                rb = (ub.a[a][c] * (k.dt * k.inv_We) * Gp + Gz * Gp) / (rf * rf);
            }
            usb.a[a][c] = us;
            rfnb.a[a][c] = rb;
            rfob.a[a][c] = 0.0;
            aphib.a[a][c] = 0.0;
            gmub.a[a][c] = 0.0;
            mb.a[a][c] = 0.0;
            nu.a[a][c] = 0.0;
            uout.a[a][c] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// A5: momentum adjoint, face part (component a), after K_a nu_a = ustar_bar_a
// ---------------------------------------------------------------------------

// N_a(m, w)(c) = (1/(2h)) sum_b [mbar+ w(c+e_b) - mbar- w(c-e_b)] with the
// forward's wall rules (normal component zero on the walls, tangential ghost
// -w); m from the forward state.
template <int DIM>
__device__ inline double nadv_at(const Geo &g, const StepConst &k, int a, int c, const int ia[3],
                                 const double *__restrict__ phi, const double *__restrict__ mu, const U3 &u,
                                 const double *__restrict__ w) {
    const int cam = nb_lo(g, c, ia[a], a);
    double n = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b), hi = nb_hi(g, c, ia[b], b);
        if (b == a) {
            const double m_c = mflux<DIM>(g, k, phi, mu, u.a[a], a, c, ia[a]);
            const double m_hi = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[a], a, hi, wrap_next(ia[a], g.n[a])) : 0.0;
            const double m_lo = mflux<DIM>(g, k, phi, mu, u.a[a], a, lo, wrap_prev(ia[a], g.n[a]));
            const double wp = hi >= 0 ? w[hi] : 0.0;
            const double wm = (!g.per[a] && ia[a] == 1) ? 0.0 : w[lo];
            n += 0.5 * (m_c + m_hi) * wp - 0.5 * (m_lo + m_c) * wm;
        } else {
            const int ibn = wrap_next(ia[b], g.n[b]);
            const double mph = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[b], b, hi, ibn) : 0.0;
            const int hiam = hi >= 0 ? nb_lo(g, hi, ia[a], a) : -1;
            const double mpha = hi >= 0 ? mflux<DIM>(g, k, phi, mu, u.a[b], b, hiam, ibn) : 0.0;
            const double mm = 0.5 * (mflux<DIM>(g, k, phi, mu, u.a[b], b, c, ia[b]) +
                                     mflux<DIM>(g, k, phi, mu, u.a[b], b, cam, ia[b]));
            const double wc = w[c];
            const double wp = hi >= 0 ? w[hi] : -wc;
            const double wm = lo >= 0 ? w[lo] : -wc;
            n += 0.5 * (mph + mpha) * wp - mm * wm;
        }
    }
    return n * 0.5 * k.ih;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_mom_faces(Geo g, StepConst k, int a, const double *__restrict__ phi,
                                                          const double *__restrict__ phin,
                                                          const double *__restrict__ mu, U3 u, U3 ustar,
                                                          const double *__restrict__ nu, double *__restrict__ sbar,
                                                          W3 csb, W3 rfnb, W3 rfob, W3 aphib, W3 gmub, W3 uout,
                                                          double *__restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    const double st = k.inv_We / k.Cn;
    double acc = 0.0;
    const double *us = ustar.a[a];
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        if (!g.per[a] && ia[a] == 0) {
            sbar[c] = 0.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) csb.a[b][c] = 0.0;
            continue;
        }
        const int cam = nb_lo(g, c, ia[a], a);
        const double nuc = nu[c], usc = us[c];
        const double sb = -nuc * usc;
        sbar[c] = sb;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int lo = nb_lo(g, c, ia[b], b);
            const bool coupled = (b == a) ? !(!g.per[a] && ia[a] <= 1) : (lo >= 0);
            csb.a[b][c] = coupled ? -(nuc - nu[lo]) * (usc - us[lo]) : 0.0;
        }
        const double rf_new = 0.5 * (rho_of(k, phin[c]) + rho_of(k, phin[cam]));
        const double rf_old = 0.5 * (rho_of(k, phi[c]) + rho_of(k, phi[cam]));
        const double uac = u.a[a][c];
        double rb = sb / k.dt + nuc * uac / (2.0 * k.dt);
        if (a == 1 && k.inv_Fr != 0.0) rb -= k.inv_Fr * nuc;
        rfnb.a[a][c] += rb;
        rfob.a[a][c] += nuc * uac / (2.0 * k.dt);
        // -(dN/du)^T nu = +N(m, nu) (skew-symmetry of the advection)
        uout.a[a][c] += nuc * (0.5 * (rf_new + rf_old)) / k.dt + nadv_at<DIM>(g, k, a, c, ia, phi, mu, u, nu);
        const double aphi = 0.5 * (phi[c] + phi[cam]);
        const double gmu = (mu[c] - mu[cam]) * k.ih;
        aphib.a[a][c] += -st * nuc * gmu;
        gmub.a[a][c] += -st * nuc * aphi;
        acc += -nuc * aphi * gmu;
    }
    const double s = block_partial(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// A6: gathers of the momentum adjoint onto cells (eta_bar) and onto the mass
// flux faces of every axis (m_bar) for component a.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_mom_gather(Geo g, StepConst k, int a, U3 u,
                                                           const double *__restrict__ nu,
                                                           const double *__restrict__ sbar, U3 csb,
                                                           double *__restrict__ etab, W3 mb) {
    const double rvis = k.inv_Re * k.ih2;
    const double *ua = u.a[a];
    CELL_LOOP(g.N) {
        int ie[3];
        cc<DIM>(g, c, ie[0], ie[1], ie[2]);
        const int e = c;
        const int ea = nb_hi(g, e, ie[a], a);   // e + e_a
        double acc = 0.0;
        // viscous coefficient through the cell centre e of row e + e_a
        if (ea >= 0) acc += csb.a[a][ea];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            // edge coefficients of rows e, e+e_a, e+e_b, e+e_a+e_b
            const int eb = nb_hi(g, e, ie[b], b);
            const int eab = ea >= 0 ? nb_hi(g, ea, ie[b], b) : -1;
            acc += 0.25 * csb.a[b][e];
            if (ea >= 0) acc += 0.25 * csb.a[b][ea];
            if (eb >= 0) acc += 0.25 * csb.a[b][eb];
            if (eab >= 0) acc += 0.25 * csb.a[b][eab];
            // no-slip folds of rows e and e+e_a on each walled b boundary
            if (!g.per[b]) {
                const int nf = (ie[b] == 0 ? 1 : 0) + (ie[b] == g.n[b] - 1 ? 1 : 0);
                if (nf) acc += nf * (sbar[e] + (ea >= 0 ? sbar[ea] : 0.0));
            }
        }
        if (!g.per[a]) {
            if (ie[a] == 0 && ea >= 0) acc += sbar[ea];   // row with i_a = 1: eta(c - e_a)
            if (ie[a] == g.n[a] - 1) acc += sbar[e];       // row with i_a = N - 1: eta(c)
        }
        etab[e] += acc * rvis;

        // m_bar on the face e of every axis b
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (!g.per[b] && ie[b] == 0) continue;   // wall face: m = 0
            double gs = 0.0;
            if (b == a) {
                const int elo = nb_lo(g, e, ie[a], a);
                // row e: both halves
                {
                    const double wp = ea >= 0 ? ua[ea] : 0.0;
                    const double wm = (!g.per[a] && ie[a] == 1) ? 0.0 : ua[elo];
                    gs += nu[e] * wp - nu[e] * wm;
                }
                // row e - e_a: upper half (if that row is not the wall row)
                if (g.per[a] || ie[a] >= 2) gs += nu[elo] * ua[e];
                // row e + e_a: lower half
                if (ea >= 0) {
                    const int iea = ie[a] + 1 < g.n[a] ? ie[a] + 1 : 0;
                    const double wm = (!g.per[a] && iea == 1) ? 0.0 : ua[e];
                    gs -= nu[ea] * wm;
                }
            } else {
                const int elb = nb_lo(g, e, ie[b], b);      // e - e_b (exists: face e valid)
                const int r2 = nb_hi(g, elb, ie[a], a);     // e - e_b + e_a
                const bool rows_lo_ok = g.per[a] || ie[a] >= 1;   // rows e, e - e_b are not wall rows
                auto wplus = [&](int r, int ib) {            // u_a(r + e_b) or ghost
                    const int rh = nb_hi(g, r, ib, b);
                    return rh >= 0 ? ua[rh] : -ua[r];
                };
                auto wminus = [&](int r, int ib) {           // u_a(r - e_b) or ghost
                    const int rl = nb_lo(g, r, ib, b);
                    return rl >= 0 ? ua[rl] : -ua[r];
                };
                const int iblo = wrap_prev(ie[b], g.n[b]);
                if (rows_lo_ok) gs += nu[elb] * wplus(elb, iblo);
                if (r2 >= 0) gs += nu[r2] * wplus(r2, iblo);
                if (rows_lo_ok) gs -= nu[e] * wminus(e, ie[b]);
                if (ea >= 0) gs -= nu[ea] * wminus(ea, ie[b]);
            }
            mb.a[b][e] += -0.25 * k.ih * gs;
        }
    }
}

// ---------------------------------------------------------------------------
// A7: rho_f'_bar, rho_f_bar -> cells; eta_bar; pull-back; phi' total adjoint
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_rho(Geo g, StepConst k, const double *__restrict__ phi,
                                                    const double *__restrict__ phin, const double *__restrict__ mu,
                                                    const double *phibar_in, U3 rfnb, U3 rfob,
                                                    const double *__restrict__ etab, double *__restrict__ pbt,
                                                    double *phibar_out, double *__restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double acc = 0.0;
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        double rbn = 0.0, rbo = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a), hi = nb_hi(g, c, ia[a], a);
            if (lo >= 0) {
                rbn += 0.5 * rfnb.a[a][c];
                rbo += 0.5 * rfob.a[a][c];
            }
            if (hi >= 0) {
                rbn += 0.5 * rfnb.a[a][hi];
                rbo += 0.5 * rfob.a[a][hi];
            }
        }
        const double pt = phibar_in[c] + (k.alpha * rbn + k.gamma * etab[c]) * dpullback(phin[c]);
        pbt[c] = pt;
        phibar_out[c] = k.alpha * rbo * dpullback(phi[c]) + pt;
        auto muv = [&](int e) { return mu[e]; };
        acc += k.dt * pt * lap_c<DIM>(g, c, ia, k.ih2, muv);
    }
    const double s = block_partial(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// A8: phi-update and mass-flux adjoints on faces
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_flux(Geo g, StepConst k, const double *__restrict__ phi,
                                                     const double *__restrict__ mu, U3 u,
                                                     const double *__restrict__ pbt, W3 Fb, W3 gmub, W3 aphib,
                                                     U3 mb, W3 uout, double *__restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    const double ak = k.alpha / (k.Cn * k.Pe);   // alpha k
    double acc = 0.0;
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            if (lo < 0) {
                Fb.a[a][c] = 0.0;
                continue;
            }
            const double Gpb = (pbt[c] - pbt[lo]) * k.ih;
            Fb.a[a][c] = k.dt * Gpb;
            const double mbc = mb.a[a][c];
            const double gmu = (mu[c] - mu[lo]) * k.ih;
            gmub.a[a][c] += -ak * mbc - k.dt * k.kM * Gpb;
            uout.a[a][c] += mbc * (0.5 * ((k.alpha * phi[c] + k.beta) + (k.alpha * phi[lo] + k.beta)));
            aphib.a[a][c] += k.alpha * mbc * u.a[a][c];
            acc += -k.alpha * mbc * gmu;   // d m / d k = -alpha G mu
        }
    }
    const double s = block_partial(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// A9: mu_bar = -D(G mu_bar); phi_bar += (psi'' - S) mu_bar
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_mu(Geo g, StepConst k, const double *__restrict__ phi, U3 gmub,
                                                   double *__restrict__ mub, double *__restrict__ phibar_out) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a), hi = nb_hi(g, c, ia[a], a);
            div += (hi >= 0 ? gmub.a[a][hi] : 0.0) - (lo >= 0 ? gmub.a[a][c] : 0.0);
        }
        const double m = -div * k.ih;
        mub[c] = m;
        const double pc = phi[c];
        phibar_out[c] += (3.0 * pc * pc - 1.0 - k.S) * m;
    }
}

// A10: right-hand side of the CH adjoint, S mu_bar - Cn^2 L mu_bar; L phihat
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_chrhs(Geo g, StepConst k, const double *__restrict__ phihat,
                                                      const double *__restrict__ mub, double *__restrict__ chr,
                                                      double *__restrict__ lphi, double *__restrict__ omega) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        auto mv = [&](int e) { return mub[e]; };
        auto hv = [&](int e) { return phihat[e]; };
        chr[c] = k.S * mub[c] - k.Cn * k.Cn * lap_c<DIM>(g, c, ia, k.ih2, mv);
        lphi[c] = lap_c<DIM>(g, c, ia, k.ih2, hv);
        omega[c] = 0.0;   // zero initial guess of the adjoint CH solve
    }
}

// A12: after M omega = chr: dL/dk from the CH operator and the explicit
// stage; phi_bar += omega + (psi'' - S) dt k L omega
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_ch_post(Geo g, StepConst k, const double *__restrict__ phi,
                                                        const double *__restrict__ omega,
                                                        const double *__restrict__ lphi,
                                                        double *__restrict__ phibar_out, double *__restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double acc = 0.0;
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        auto lv = [&](int e) { return lphi[e]; };
        auto ov = [&](int e) { return omega[e]; };
        auto gv = [&](int e) { return dpsi(phi[e]) - k.S * phi[e]; };
        const double om = omega[c];
        acc += k.dt * om * (k.S * lphi[c] - k.Cn * k.Cn * lap_c<DIM>(g, c, ia, k.ih2, lv)) +
               k.dt * om * lap_c<DIM>(g, c, ia, k.ih2, gv);
        const double pc = phi[c];
        phibar_out[c] += om + (3.0 * pc * pc - 1.0 - k.S) * k.dt * k.kM * lap_c<DIM>(g, c, ia, k.ih2, ov);
    }
    const double s = block_partial(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// A14: advective flux adjoint F_bar = Fb + dt G omega -> u_bar, A(phi)_bar
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_adv(Geo g, StepConst k, const double *__restrict__ phi, U3 u,
                                                    const double *__restrict__ omega, U3 Fb, W3 aphib, W3 uout) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            if (lo < 0) continue;
            const double fb = Fb.a[a][c] + k.dt * (omega[c] - omega[lo]) * k.ih;
            uout.a[a][c] += fb * (0.5 * (phi[lo] + phi[c]));
            aphib.a[a][c] += fb * u.a[a][c];
        }
    }
}

// A15: phi_bar += sum_a A_a^T (A(phi)_bar)
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_aphi(Geo g, U3 aphib, double *__restrict__ phibar_out) {
    CELL_LOOP(g.N) {
        int ia[3];
        cc<DIM>(g, c, ia[0], ia[1], ia[2]);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a), hi = nb_hi(g, c, ia[a], a);
            if (lo >= 0) s += 0.5 * aphib.a[a][c];
            if (hi >= 0) s += 0.5 * aphib.a[a][hi];
        }
        phibar_out[c] += s;
    }
}

// Parameter derivatives of this step: fixed-order sums of the regions give
// dL/dk and dL/ds_t; with sigma = 1/We and M = We/Pe, k = M sigma / Cn and
// s_t = sigma / Cn, so dL/dsigma = (M dL/dk + dL/ds_t) / Cn and
// dL/dM = sigma dL/dk / Cn.
__global__ void __launch_bounds__(kBlock) k_adj_params(const double *__restrict__ gpart, int nparts, int dim,
                                                       double sigma, double mob, double Cn,
                                                       double *__restrict__ out) {
    __shared__ double lds[kBlock / kWave];
    double vk = 0.0, vs = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) vk += gpart[r * kRedBlocks + i];
    for (int r = 0; r < dim; ++r)
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) vs += gpart[(3 + r) * kRedBlocks + i];
    const double tk = block_sum(vk, lds);
    const double ts = block_sum(vs, lds);
    if (threadIdx.x == 0) {
        out[0] = (mob * tk + ts) / Cn;
        out[1] = sigma * tk / Cn;
        out[2] = tk;
        out[3] = ts;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)
#define LAUNCHR(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_red(n)), dim3(kBlock), st, __VA_ARGS__)
#define ADISPATCH(R, arrays, dim, kern, n, st, ...)                                   \
    do {                                                                              \
        const double bytes_ = 8.0 * (double)(arrays) * (double)(n);                   \
        if ((dim) == 2)                                                               \
            R(K_ADJOINT, bytes_, (kern<2>), n, st, __VA_ARGS__);                         \
        else                                                                          \
            R(K_ADJOINT, bytes_, (kern<3>), n, st, __VA_ARGS__);                         \
    } while (0)

static U3 cu3(double *const v[3]) { return U3{{v[0], v[1], v[2]}}; }

void adj_p_rhs(int dim, const Geo &g, const StepConst &k, const double *phin, const double *const ubar[3],
               double *pbar, double *zeta, hipStream_t st) {
    ADISPATCH(LAUNCH, 3 + dim, dim, k_adj_p_rhs, (int)g.N, st, g, k, phin, mk_u3(ubar), pbar, zeta);
}

void adj_proj_faces(int dim, const Geo &g, const StepConst &k, const double *phin, const double *p, const double *zeta,
                    const double *const ubar[3], AdjBufs &A, double *const uout[3], hipStream_t st) {
    ADISPATCH(LAUNCH, 4 + 9 * dim, dim, k_adj_proj_faces, (int)g.N, st, g, k, phin, p, zeta, mk_u3(ubar),
              mk_w3(A.usb), mk_w3(A.rfnb), mk_w3(A.rfob), mk_w3(A.aphib), mk_w3(A.gmub), mk_w3(A.mb), mk_w3(A.nu),
              mk_w3(uout), A.etab);
}

void adj_mom(int dim, const Geo &g, const StepConst &k, int a, const double *phi, const double *phin,
             const double *mu, const double *const u[3], const double *const ustar[3], AdjBufs &A,
             double *const uout[3], hipStream_t st) {
    ADISPATCH(LAUNCHR, 12 + dim, dim, k_adj_mom_faces, (int)g.N, st, g, k, a, phi, phin, mu, mk_u3(u), mk_u3(ustar),
              (const double *)A.nu[a], A.sbar, mk_w3(A.csb), mk_w3(A.rfnb), mk_w3(A.rfob), mk_w3(A.aphib),
              mk_w3(A.gmub), mk_w3(uout), A.gpart + (3 + a) * kRedBlocks);
    ADISPATCH(LAUNCH, 4 + 2 * dim, dim, k_adj_mom_gather, (int)g.N, st, g, k, a, mk_u3(u), (const double *)A.nu[a],
              (const double *)A.sbar, cu3(A.csb), A.etab, mk_w3(A.mb));
}

void adj_rho_flux_mu(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phin,
                     const double *mu, const double *const u[3], const double *phibar_in, AdjBufs &A,
                     double *const uout[3], double *phibar_out, hipStream_t st) {
    ADISPATCH(LAUNCHR, 7 + 2 * dim, dim, k_adj_rho, (int)g.N, st, g, k, phi, phin, mu, phibar_in, cu3(A.rfnb),
              cu3(A.rfob), (const double *)A.etab, A.pbt, phibar_out, A.gpart + 0 * kRedBlocks);
    ADISPATCH(LAUNCHR, 3 + 9 * dim, dim, k_adj_flux, (int)g.N, st, g, k, phi, mu, mk_u3(u), (const double *)A.pbt,
              mk_w3(A.Fb), mk_w3(A.gmub), mk_w3(A.aphib), cu3(A.mb), mk_w3(uout), A.gpart + 1 * kRedBlocks);
    ADISPATCH(LAUNCH, 3 + dim, dim, k_adj_mu, (int)g.N, st, g, k, phi, cu3(A.gmub), A.mub, phibar_out);
}

void adj_ch_rhs(int dim, const Geo &g, const StepConst &k, const double *phihat, AdjBufs &A, hipStream_t st) {
    ADISPATCH(LAUNCH, 5, dim, k_adj_chrhs, (int)g.N, st, g, k, phihat, (const double *)A.mub, A.chr, A.lphi, A.omega);
}

void adj_ch_post(int dim, const Geo &g, const StepConst &k, const double *phi, const double *const u[3],
                 AdjBufs &A, double *const uout[3], double *phibar_out, hipStream_t st) {
    ADISPATCH(LAUNCHR, 5, dim, k_adj_ch_post, (int)g.N, st, g, k, phi, (const double *)A.omega,
              (const double *)A.lphi, phibar_out, A.gpart + 2 * kRedBlocks);
    ADISPATCH(LAUNCH, 2 + 6 * dim, dim, k_adj_adv, (int)g.N, st, g, k, phi, mk_u3(u), (const double *)A.omega,
              cu3(A.Fb), mk_w3(A.aphib), mk_w3(uout));
    ADISPATCH(LAUNCH, 2 + dim, dim, k_adj_aphi, (int)g.N, st, g, cu3(A.aphib), phibar_out);
}

void adj_params(int dim, const Geo &g, const StepConst &k, const AdjBufs &A, double *out, hipStream_t st) {
    const int nb = grid_red(g.N);
    const double sigma = k.inv_We, mob = k.We / k.Pe;
    TLAUNCH(K_ADJOINT, 8.0 * kAdjRegions * nb, (k_adj_params), dim3(1), dim3(kBlock), st, (const double *)A.gpart, nb,
            dim, sigma, mob, k.Cn, out);
}

}  // namespace chns
