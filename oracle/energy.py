"""Energy-law step monitor (oracle, test infrastructure).

The paper's energy-stability theorem bounds the change of the total energy
over one step by two dissipation terms and two sign-indeterminate terms, and
gives a time-step restriction under which the dissipation dominates:

  dt/Re ||sqrt(eta) grad v||^2 + dt/(Pe Cn^2 We) ||grad mu||^2
      >= 1/(24 We Cn) (psi'''(lambda), (phi^{n+1} - phi^n)^3)
       + 1/8 int (rho^{n+1} - rho^n) |v^{n+1} - v^n|^2 .

This module evaluates the discrete counterparts of these four terms for one
step of Algorithm S (oracle.chns.step), with the step's own fields in place
of the paper's Crank-Nicolson averages (v -> u^{n+1}, mu -> mu^{n+1},
eta -> eta^{n+1}):

  visc   = sum_a u_a^T K_a u_a h^d, K_a the viscous part -(1/Re) div(eta grad)
           of the momentum operator of component a (the oracle's momentum
           matrix with zero shift): the discrete (1/Re)||sqrt(eta) grad u||^2
  chem   = (1/(Pe Cn^2 We)) sum_a sum_faces (G_a mu)^2 h^d
  cubic  = (1/(24 We Cn)) sum 6 max(|phi^n|, |phi^{n+1}|) |phi^{n+1} - phi^n|^3 h^d
           (psi''' = 6 phi, lambda between phi^n and phi^{n+1}: a bound of the
           magnitude of the first indeterminate term)
  inert  = (1/8) sum_a sum_faces |A_a(rho^{n+1} - rho^n)| (u_a^{n+1} - u_a^n)^2 h^d
           (a bound of the second)

and the step condition dt (visc + chem) >= cubic + inert.  The two bounds
grow like dt^3 and the dissipation like dt, so the largest step that keeps
the condition is estimated as dt_max = dt sqrt(dt (visc + chem) / (cubic + inert)).
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

from .chns import Params, coefficients, diagnostics, momentum_matrix, pullback, step
from .grid import MACGrid


def viscous_dissipation(g: MACGrid, u, eta: np.ndarray, Re: float) -> float:
    """sum_a u_a^T K_a u_a h^d with K_a = -(1/Re) div_h(eta grad_h) on the
    faces of axis a (no-slip walls as in the momentum solve)."""
    hd = g.h ** g.dim
    total = 0.0
    for a in range(g.dim):
        K, unk = momentum_matrix(g, a, np.zeros(g.shape), eta, Re)
        x = u[a][unk]
        total += float(x @ (K @ x)) * hd
    return total


def chemical_dissipation(g: MACGrid, mu: np.ndarray, prm: Params) -> float:
    hd = g.h ** g.dim
    s = sum(float(np.sum(g.grad(mu, a) ** 2)) for a in range(g.dim))
    return s * hd / (prm.Pe * prm.Cn ** 2 * prm.We)


def cubic_bound(g: MACGrid, phi0: np.ndarray, phi1: np.ndarray, prm: Params) -> float:
    hd = g.h ** g.dim
    lam = np.maximum(np.abs(phi0), np.abs(phi1))
    return float(np.sum(6.0 * lam * np.abs(phi1 - phi0) ** 3)) * hd / (24.0 * prm.We * prm.Cn)


def inertia_bound(g: MACGrid, rho0: np.ndarray, rho1: np.ndarray, u0, u1) -> float:
    hd = g.h ** g.dim
    s = 0.0
    for a in range(g.dim):
        s += float(np.sum(np.abs(g.avg(rho1 - rho0, a)) * (u1[a] - u0[a]) ** 2))
    return s * hd / 8.0


def step_monitor(g: MACGrid, st: Dict, prm: Params):
    """One step of Algorithm S and its energy-law terms.  Returns the new
    state and a dict with visc, chem, cubic, inert, dt_max (inf when both
    bounds vanish), holds (the step condition), energy_before, energy_after."""
    new = step(g, st, prm)
    alpha, beta, _, _ = coefficients(prm)
    visc = viscous_dissipation(g, new["u"], new["eta"], prm.Re)
    chem = chemical_dissipation(g, new["mu"], prm)
    cubic = cubic_bound(g, st["phi"], new["phi"], prm)
    rho0 = alpha * pullback(st["phi"]) + beta
    inert = inertia_bound(g, rho0, new["rho"], st["u"], new["u"])
    diss = prm.dt * (visc + chem)
    ind = cubic + inert
    dt_max = math.inf if ind == 0.0 else prm.dt * math.sqrt(diss / ind)
    out = {"visc": visc, "chem": chem, "cubic": cubic, "inert": inert, "dt_max": dt_max,
           "holds": diss >= ind, "energy_before": diagnostics(g, st, prm)["energy"],
           "energy_after": diagnostics(g, new, prm)["energy"]}
    return new, out
