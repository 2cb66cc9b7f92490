// Energy-law step monitor (gfx950): the four terms of the time-step
// condition of the paper's energy-stability theorem, evaluated for one step
// of the split scheme with that step's fields (u^{n+1}, mu^{n+1},
// eta^{n+1}) in place of the theorem's Crank-Nicolson averages:
//   visc  = sum_a u_a^T K_a u_a h^d, K_a the viscous part of the momentum
//           operator of component a (the step's own level-0 coefficients,
//           minus the rho_f/dt shift): (1/Re) ||sqrt(eta) grad u||^2
//   chem  = (1/(Pe Cn^2 We)) sum_faces (G mu)^2 h^d
//   cubic = (1/(24 We Cn)) sum 6 max(|phi^n|, |phi^{n+1}|) |phi^{n+1} - phi^n|^3 h^d
//   inert = (1/8) sum_a sum_faces |A_a(rho^{n+1} - rho^n)| (u_a^{n+1} - u_a^n)^2 h^d
// (the last two bound the magnitudes of the sign-indeterminate terms, with
// psi''' = 6 phi).  One kernel after the pressure solve, before the
// projection overwrites u^n: u^{n+1} is formed from u* and p on the fly.
#include "stepdev.h"

namespace chns {

struct MonSlots {
    const double *s[3];
    const double *cs[3][3];   // cs[a][b]: component a, direction b
};

constexpr int kNMon = 4;   // visc, chem, cubic, inert

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_energy_mon(Geo g, StepConst k, const double *__restrict__ phi,
                                                       const double *__restrict__ phin, const double *__restrict__ mu,
                                                       U3 u, U3 us, const double *__restrict__ p, MonSlots ms,
                                                       double *part, unsigned int *counter, double *out) {
    __shared__ double lds[kBlock / kWave];
    double acc[kNMon] = {0, 0, 0, 0};
    auto rho_new = [&](int e) { return k.alpha * pullback(phin[e]) + k.beta; };
    auto rho_old = [&](int e) { return k.alpha * pullback(phi[e]) + k.beta; };
    CELL_LOOP(g.N) {
        int i, j, kk;
        cc<DIM>(g, c, i, j, kk);
        const int ia[3] = {i, j, kk};
        const double p0 = phi[c], p1 = phin[c], dp = fabs(p1 - p0);
        acc[2] += 6.0 * fmax(fabs(p0), fabs(p1)) * (dp * dp * dp);
        const double drc = rho_new(c) - rho_old(c);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int lo = nb_lo(g, c, ia[a], a);
            if (lo < 0 || (!g.per[a] && ia[a] == 0)) continue;   // wall face: G mu = 0, u = 0
            const double gm = (mu[c] - mu[lo]) * k.ih;
            acc[1] += gm * gm;
            // u^{n+1}_a on face f (between f - e_a and f), as the projection forms it
            auto unew = [&](int f, int fa) -> double {
                const int fl = nb_lo(g, f, fa, a);
                if (fl < 0 || (!g.per[a] && fa == 0)) return 0.0;
                const double rf = 0.5 * (rho_new(f) + rho_new(fl));
                return us.a[a][f] - (k.dt * k.inv_We) * ((p[f] - p[fl]) * k.ih) / rf;
            };
            const double uc = unew(c, ia[a]);
            const double rfn = 0.5 * (rho_new(c) + rho_new(lo));
            double v = (ms.s[a][c] - rfn / k.dt) * (uc * uc);
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                const double w = ms.cs[a][b][c];
                if (w == 0.0) continue;
                const int nb = nb_lo(g, c, ia[b], b);     // face c - e_b of component a
                const int nba = b == a ? wrap_prev(ia[a], g.n[a]) : ia[a];
                const double d = uc - unew(nb, nba);
                v += w * (d * d);
            }
            acc[0] += v;
            const double du = uc - u.a[a][c];
            acc[3] += fabs(0.5 * (drc + (rho_new(lo) - rho_old(lo)))) * (du * du);
        }
    }
#pragma unroll
    for (int q = 0; q < kNMon; ++q) {
        const double v = block_sum(acc[q], lds);
        if (threadIdx.x == 0) part[q * kMaxBlocks + blockIdx.x] = v;
    }
    if (last_block(counter)) {
        for (int q = 0; q < kNMon; ++q) {
            double v = 0.0;
            for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) v += ((volatile double *)part)[q * kMaxBlocks + b];
            v = block_sum(v, lds);
            if (threadIdx.x == 0) out[q] = v;
        }
        if (threadIdx.x == 0) *counter = 0;
    }
}

// Sums visc / chem / cubic / inert (unscaled) into out[0..3].
void launch_energy_monitor(int dim, const Geo &g, const StepConst &k, const double *phi, const double *phi_new,
                           const double *mu, const double *const u[3], const double *const ustar[3], const double *p,
                           const double *const s[3], const double *const cs[3][3], double *part,
                           unsigned int *counter, double *out, hipStream_t st) {
    MonSlots ms;
    for (int a = 0; a < 3; ++a) {
        ms.s[a] = s[a];
        for (int b = 0; b < 3; ++b) ms.cs[a][b] = cs[a][b];
    }
    const double bytes = 8.0 * (4 + 2 * dim + dim * (1 + dim)) * g.N;
    if (dim == 2)
        TLAUNCH(K_DIAG, bytes, (k_energy_mon<2>), dim3(grid_for(g.N)), dim3(kBlock), st, g, k, phi, phi_new, mu,
                mk_u3(u), mk_u3(ustar), p, ms, part, counter, out);
    else
        TLAUNCH(K_DIAG, bytes, (k_energy_mon<3>), dim3(grid_for(g.N)), dim3(kBlock), st, g, k, phi, phi_new, mu,
                mk_u3(u), mk_u3(ustar), p, ms, part, counter, out);
}

}  // namespace chns
