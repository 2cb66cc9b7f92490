"""Second-order Crank-Nicolson variant of the split step (oracle, test
infrastructure): Algorithm C.

The paper's time scheme (section "Numerical method and its properties",
eqns. averaging1, psi_ave_def and the time-discrete variational problem)
evaluates every term at the midpoint: v~ = (v^k + v^{k+1})/2,
phi~ = (phi^k + phi^{k+1})/2, mu~, p~, with rho~ = rho(phi~), eta~ = eta(phi~),
psi'(phi~), the flux J~ from grad mu~ and the momentum advection
(rho~ v~ + J~/Pe) . grad v~.  The paper solves that nonlinear system fully
coupled with Newton's method; here it is solved by Picard iterations whose
every sub-step is a linear system of the split step's kind (a reading, see
the design notes), iterate m -> m+1 with phi~m, v~m, p~m:

  C1  r = phi^k - dt/2 D(v~m A phi~m) + dt/2 kM L(psi'(phi~m) - S phi~m)
  C2  (I - dt/2 kM S L + dt/2 kM Cn^2 L L) phi~ = r
  C3  mu~ = psi'(phi~m) + S (phi~ - phi~m) - Cn^2 L phi~
  C4  phi^{k+1} = phi^k - dt D(v~m A phi~m - kM G mu~)       (flux form)
      phi~{m+1} = (phi^k + phi^{k+1}) / 2
  C5  m~ = A(alpha phi~m + beta) v~m - (alpha kM) G mu~     (= rho_lin v + J/Pe)
  C6  rho~, eta~ from the pulled-back phi~{m+1}
  C7  per component: (2 rho~_f/dt) v~* - (1/Re) div(eta~ grad v~*)
        = (2 rho~_f/dt) v^k - Adv(m~, v~m) - (1/We) G p~m
          - (1/(We Cn)) A(phi~m) G mu~ + rho~_f g_hat / Fr,
      Adv the advective form m . grad v (the advective half of the split
      step's skew-symmetric operator)
  C8  -D(rho~_f^{-1} G dp) = -(2 We/dt) D v~*,  mean(dp) = 0
  C9  v~{m+1} = v~* - (dt/(2 We)) rho~_f^{-1} G dp,  p~{m+1} = p~m + dp,
      v^{k+1} = 2 v~{m+1} - v^k

starting from phi~0 = phi^k, v~0 = v^k, p~0 = the stored pressure (the
previous step's midpoint pressure).  At a fixed point the stabiliser terms
S(phi~ - phi~m) and the pressure increment vanish, so the iteration solves
the midpoint system itself: C3 is the paper's chemical-potential equation
at phi~, C2 / C4 its CH equation, C7 its momentum equation and C9 its
solenoidality.  `picard` sets the number of iterations (a fixed count, so
that the GPU path can follow the same sequence).
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from .chns import (Params, ch_solve_spectral, coefficients, dpsi, mbar, momentum_solve, neighbours_u,
                   pressure_solve, pullback, wall_velocity_rhs)
from .grid import MACGrid


def advective_form(g: MACGrid, m, u: np.ndarray, a: int) -> np.ndarray:
    """m . grad u_a on the faces of axis a: the upwind-free advective
    difference (mp (u_+ - u) + mm (u - u_-)) / (2h) per direction, with m
    interpolated to the u_a control-volume faces (as in the split step's
    skew-symmetric operator, of which it is the advective half)."""
    out = np.zeros(g.shape)
    for b in range(g.dim):
        mp, mm = mbar(g, m, a, b)
        up, um = neighbours_u(g, u, a, b)
        out += 0.5 * (mp * (up - u) + mm * (u - um)) / g.h
    return out


def step_cn(g: MACGrid, st: Dict, prm: Params, picard: int = 3, forcing: Optional[Dict] = None,
            wall_u: Optional[Dict] = None, ch_only: bool = False) -> Dict:
    """One step k -> k+1 of Algorithm C.  st = {'phi', 'u', 'p'} with p the
    previous midpoint pressure.  forcing (manufactured solutions): 'phi',
    'mu' (cells) and 'u' (faces) at the midpoint time t^{k+1/2}.  ch_only:
    the Cahn-Hilliard part alone (u stays as given).  Returns 'phi', 'u',
    'p' (the new midpoint pressure), 'mu' (mu~), and 'phit', 'ut' (the
    midpoints)."""
    d = g.dim
    phik, vk = st["phi"], st["u"]
    alpha, beta, gamma, xi = coefficients(prm)
    dt, Cn, S = prm.dt, prm.Cn, prm.S
    kM = 1.0 / (prm.Pe * Cn)
    f = forcing or {}
    phim = phik.copy()
    vm = [x.copy() for x in vk]
    pm = st["p"].copy()
    a_ch, b_ch = 0.5 * dt * kM * S, 0.5 * dt * kM * Cn * Cn
    for _ in range(picard):
        # C1 - C4
        F = [vm[a] * g.avg(phim, a) for a in range(d)]
        r = phik - 0.5 * dt * g.div(F) + 0.5 * dt * kM * g.lap(dpsi(phim) - S * phim)
        if "phi" in f:
            r = r + 0.5 * dt * f["phi"]
        if "mu" in f:
            r = r + 0.5 * dt * kM * g.lap(f["mu"])
        phit = ch_solve_spectral(g, r, a_ch, b_ch)
        mu = dpsi(phim) + S * (phit - phim) - Cn * Cn * g.lap(phit)
        if "mu" in f:
            mu = mu + f["mu"]
        Gmu = [g.grad(mu, a) for a in range(d)]
        phin = phik - dt * g.div([F[a] - kM * Gmu[a] for a in range(d)])
        if "phi" in f:
            phin = phin + dt * f["phi"]
        phit_new = 0.5 * (phik + phin)
        if ch_only:
            phim = phit_new
            continue
        # C5, C6
        m = [np.where(g.wall_face_mask(a), 0.0, g.avg(alpha * phim + beta, a) * vm[a] - alpha * kM * Gmu[a])
             for a in range(d)]
        rho_t = alpha * pullback(phit_new) + beta
        eta_t = gamma * pullback(phit_new) + xi
        rhof = [g.avg(rho_t, a) for a in range(d)]
        # C7
        vstar = []
        half = Params(**{**prm.__dict__, "dt": 0.5 * dt})     # the operator 2 rho/dt - (1/Re) div(eta grad)
        for a in range(d):
            rhs = 2.0 * rhof[a] / dt * vk[a]
            rhs = rhs - advective_form(g, m, vm[a], a)
            rhs = rhs - g.grad(pm, a) / prm.We
            rhs = rhs - (1.0 / (prm.We * Cn)) * g.avg(phim, a) * Gmu[a]
            if a == 1 and prm.inv_Fr != 0.0:
                rhs = rhs - rhof[a] * prm.inv_Fr
            if "u" in f:
                rhs = rhs + f["u"][a]
            if wall_u:
                rhs = rhs + wall_velocity_rhs(g, a, eta_t, prm, wall_u)
            vstar.append(momentum_solve(g, a, rhof[a], eta_t, half, rhs))
        # C8, C9
        dp = pressure_solve(g, rhof, -(2.0 * prm.We / dt) * g.div(vstar))
        vm = []
        for a in range(d):
            va = vstar[a] - (0.5 * dt / prm.We) * g.grad(dp, a) / rhof[a]
            vm.append(np.where(g.wall_face_mask(a), 0.0, va))
        pm = pm + dp
        phim = phit_new
    vnew = [np.where(g.wall_face_mask(a), 0.0, 2.0 * vm[a] - vk[a]) for a in range(d)]
    if ch_only:
        vnew = [x.copy() for x in vk]
    out = {"phi": phin, "u": vnew, "p": pm - pm.mean(), "mu": mu, "phit": phim, "ut": vm}
    if not ch_only:
        out["m"] = m
    return out
