// Kernels of the Crank-Nicolson variant of the step (gfx950).  The paper's
// time scheme evaluates every term at the midpoint (v~, phi~, mu~, p~ and
// rho(phi~), eta(phi~)); the library solves that system by Picard iterations
// whose sub-steps are the split step's linear solves (C1..C9, see the
// header).  Per iteration m, with phi~m, v~m, p~m:
//   C1  r = phi^k - dt/2 D(v~m A phi~m) + dt/2 kM L(psi'(phi~m) - S phi~m)
//   C2  (I - dt/2 kM S L + dt/2 kM Cn^2 L L) phi~ = r        (CH solve)
//   C3  mu~ = psi'(phi~m) + S (phi~ - phi~m) - Cn^2 L phi~    (k_mu)
//   C4  phi^{k+1} = phi^k - dt D(v~m A phi~m - kM G mu~), phi~{m+1} = (phi^k + phi^{k+1})/2
//   C5-C7  midpoint momentum set-up (mom_setup_body with CN) and solves
//   C8  -D(rho~_f^{-1} G dp) = -(2 We/dt) D v~*                (pressure solve)
//   C9  v~{m+1} = v~* - (dt/(2 We)) rho~_f^{-1} G dp, p~ += dp
// and at the end v^{k+1} = 2 v~ - v^k, phi = phi^{k+1}.
#include "stepdev.h"

namespace chns {

// C1 (kh: the step constants with dt/2)
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cn_ch_rhs(Geo g, StepConst kh, const double *__restrict__ phik,
                                                      const double *__restrict__ phim, U3 vm, double *__restrict__ r,
                                                      double *__restrict__ phihat) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double pc = phim[c];
        const double gc = dpsi(pc) - kh.S * pc;
        double div = 0.0, lap = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            double flo = 0.0, fhi = 0.0;
            if (lo >= 0) {
                const double pl = phim[lo];
                flo = vm.a[a][c] * (0.5 * (pl + pc));
                lap += (dpsi(pl) - kh.S * pl) - gc;
            }
            if (hi >= 0) {
                const double ph = phim[hi];
                fhi = vm.a[a][hi] * (0.5 * (pc + ph));
                lap += (dpsi(ph) - kh.S * ph) - gc;
            }
            div += fhi - flo;
        }
        r[c] = phik[c] - kh.dt * (div * kh.ih) + kh.dt * kh.kM * (lap * kh.ih2);
        phihat[c] = pc;
    }
}

// C4: flux form (each face flux evaluated identically by both of its cells)
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cn_phi_update(Geo g, StepConst k, const double *__restrict__ phik,
                                                          const double *__restrict__ phim, U3 vm,
                                                          const double *__restrict__ mu, double *__restrict__ phin,
                                                          double *__restrict__ phimid) {
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double pc = phim[c], mc = mu[c];
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            const int hi = nb_hi(g, c, ia[a], a);
            const double flo = lo >= 0 ? phi_face_flux(k, vm.a[a][c], phim[lo], pc, mu[lo], mc) : 0.0;
            const double fhi = hi >= 0 ? phi_face_flux(k, vm.a[a][hi], pc, phim[hi], mc, mu[hi]) : 0.0;
            div += fhi - flo;
        }
        const double pn = phik[c] - k.dt * (div * k.ih);
        phin[c] = pn;
        phimid[c] = 0.5 * (phik[c] + pn);
    }
}

// C5-C7 set-up of component a (kh: dt/2, so rho~_f / kh.dt = 2 rho~_f / dt)
template <int DIM, bool WALLS>
__global__ void __launch_bounds__(kBlock) k_cn_mom_setup(Geo g, StepConst kh, int a, Mix2 mx, U3 vm,
                                                         double *__restrict__ s, W3 cs, double *__restrict__ rhs,
                                                         double *__restrict__ ustar, WallVel wv,
                                                         const double *__restrict__ vk, const double *__restrict__ pm) {
    CELL_LOOP(g.N)
    mom_setup_body<DIM, Mix2, WALLS, true>(g, kh, a, mx, vm, s, cs, rhs, ustar, 0, c, &wv, vk, pm);
}

// C9: v~ = v~* - (dt/(2 We)) G dp / rho~_f (mx.phin: phi~{m+1}); p~ += dp
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cn_project(Geo g, StepConst kh, Mix2 mx, U3 us,
                                                       const double *__restrict__ dp, W3 vt, double *__restrict__ p) {
    CELL_LOOP(g.N) {
        project_body<DIM>(g, kh, mx, us, dp, vt, c);
        p[c] = p[c] + dp[c];
    }
}

// End of the step: v^{k+1} = 2 v~ - v^k (0 on wall faces), phi = phi^{k+1}
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cn_finish(Geo g, U3 vt, W3 u, double *__restrict__ phi,
                                                      const double *__restrict__ phin) {
    CELL_LOOP(g.N) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) u.a[a][c] = 2.0 * vt.a[a][c] - u.a[a][c];
        phi[c] = phin[c];
    }
}

__global__ void __launch_bounds__(kBlock) k_cn_zero(long long N, double *__restrict__ x) {
    CELL_LOOP(N) x[c] = 0.0;
}

#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)
#define DISPATCH(cls, arrays, dim, kern, n, st, ...)                            \
    do {                                                                        \
        const double bytes_ = 8.0 * (double)(arrays) * (double)(n);              \
        if ((dim) == 2)                                                         \
            LAUNCH(cls, bytes_, (kern<2>), n, st, __VA_ARGS__);                 \
        else                                                                    \
            LAUNCH(cls, bytes_, (kern<3>), n, st, __VA_ARGS__);                 \
    } while (0)

void launch_cn_ch_rhs(int dim, const Geo &g, const StepConst &kh, const double *phik, const double *phim,
                      const double *const vm[3], double *r, double *phihat, hipStream_t st) {
    DISPATCH(K_CH_RHS, 4 + dim, dim, k_cn_ch_rhs, g.N, st, g, kh, phik, phim, mk_u3(vm), r, phihat);
}

void launch_cn_phi_update(int dim, const Geo &g, const StepConst &k, const double *phik, const double *phim,
                          const double *const vm[3], const double *mu, double *phin, double *phimid, hipStream_t st) {
    DISPATCH(K_PHI_UPDATE, 5 + dim, dim, k_cn_phi_update, g.N, st, g, k, phik, phim, mk_u3(vm), mu, phin, phimid);
}

void launch_cn_mom_setup(int dim, const Geo &g, const StepConst &kh, int a, const double *phim,
                         const double *phimid, const double *mu, const double *const vm[3], double *s,
                         double *const cs[3], double *rhs, double *ustar, const double *vk, const double *pm,
                         const WallVel *wv, hipStream_t st) {
    const Mix2 mx = mk_mix2(kh, phim, phimid, mu);
    WallVel w;
    if (wv) w = *wv;
    const double bytes = 8.0 * (9 + 2 * dim) * g.N;
    const dim3 grid(grid_for(g.N)), block(kBlock);
    if (dim == 2) {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_cn_mom_setup<2, true>), grid, block, st, g, kh, a, mx, mk_u3(vm), s,
                    mk_w3(cs), rhs, ustar, w, vk, pm);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_cn_mom_setup<2, false>), grid, block, st, g, kh, a, mx, mk_u3(vm), s,
                    mk_w3(cs), rhs, ustar, w, vk, pm);
    } else {
        if (wv)
            TLAUNCH(K_MOM_SETUP, bytes, (k_cn_mom_setup<3, true>), grid, block, st, g, kh, a, mx, mk_u3(vm), s,
                    mk_w3(cs), rhs, ustar, w, vk, pm);
        else
            TLAUNCH(K_MOM_SETUP, bytes, (k_cn_mom_setup<3, false>), grid, block, st, g, kh, a, mx, mk_u3(vm), s,
                    mk_w3(cs), rhs, ustar, w, vk, pm);
    }
}

void launch_cn_project(int dim, const Geo &g, const StepConst &kh, const double *phimid,
                       const double *const ustar[3], const double *dp, double *const vt[3], double *p, hipStream_t st) {
    const Mix2 mx = mk_mix2(kh, phimid, phimid, phimid);
    DISPATCH(K_PROJECT, 4 + 2 * dim, dim, k_cn_project, g.N, st, g, kh, mx, mk_u3(ustar), dp, mk_w3(vt), p);
}

void launch_cn_finish(int dim, const Geo &g, const double *const vt[3], double *const u[3], double *phi,
                      const double *phin, hipStream_t st) {
    DISPATCH(K_PROJECT, 2 + 3 * dim, dim, k_cn_finish, g.N, st, g, mk_u3(vt), mk_w3(u), phi, phin);
}

void launch_cn_zero(const Geo &g, double *x, hipStream_t st) {
    LAUNCH(K_PCG_INIT, 8.0 * g.N, k_cn_zero, g.N, st, g.N, x);
}

}  // namespace chns
