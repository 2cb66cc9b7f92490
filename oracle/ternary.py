"""Three-phase (N = 3) split step (oracle, test infrastructure).

The paper's model is two-phase; its three-phase extension here is a reading
(documented with the other readings of the paper in the design notes):

* Phases i = 1, 2, 3 with volume fractions c_i = (1 + phi_i)/2 and
  sum_i c_i = 1, i.e. sum_i phi_i = -1.  The state holds phi_1 and phi_2; the
  third field is phi_3 = -1 - phi_1 - phi_2, so the constraint holds by
  construction.
* Free energy (Boyer-Lapuerta construction on the paper's binary density of
  the free-energy equation, written in each phi_i):
      E_free = (1/Cn) sum_i (Sigma_i / 2) int [psi(phi_i) + Cn^2/2 |grad phi_i|^2],
  Sigma_i = sigma_ij + sigma_ik - sigma_jk (spreading coefficients, all
  > 0).  For a pair i|j with the third phase absent (phi_k = -1,
  phi_j = -phi_i) this is sigma_ij times the paper's binary free energy with
  sigma = 1/We.
* Dynamics: with mu_i = psi'(phi_i) - Cn^2 lap phi_i (the paper's binary
  chemical potential of phi_i), the constrained potentials
      mu~_i = mu_i - w_i Lambda,  Lambda = sum_j mu_j,  w_i = Sigma_T / (3 Sigma_i),
  3 / Sigma_T = sum_i 1 / Sigma_i,
  satisfy sum_i mu~_i = 0 (sum_i w_i = 1), and each phase moves as the
  paper's CH equation with the same mobility:
      d phi_i/dt + div(u phi_i) = kM lap mu~_i,  kM = 1/(Pe Cn).
  (Mobility M0/Sigma_i in the Boyer-Lapuerta potentials (Sigma_i/Cn) mu~_i.)
  Because sum_j lap phi_j = 0, Lambda = sum_j psi'(phi_j).
* Mixture: rho = sum_i rho_i c_i*, eta = sum_i eta_i c_i*, c_i* = clamp(c_i, 0, 1)
  (the pull-back of the density remark applied per phase);
  consistent flux J = -(kM/2) sum_i rho_i grad mu~_i (from
  d rho/dt = sum_i rho_i d c_i/dt), so m = rho_lin u + J.
* Surface tension (potential form, as the binary step):
      f = -(1/(2 Cn)) sum_i Sigma_i phi_i grad mu~_i,
  which for a pair i|j reduces exactly to -(sigma_ij/Cn) phi grad mu.

Discrete step (Algorithm T; the binary Algorithm S for each phase, coupled
through Lambda taken at t^n):
  T1  Lambda = sum_{i=1..3} psi'(phi_i^n);  for i = 1, 2:
      r_i = phi_i - dt D(u A phi_i) + dt kM L(psi'(phi_i) - S phi_i - w_i Lambda)
  T2  (I - dt kM S L + dt kM Cn^2 L L) phihat_i = r_i
  T3  mu~_i = psi'(phi_i) + S (phihat_i - phi_i) - Cn^2 L phihat_i - w_i Lambda,
      mu~_3 = -mu~_1 - mu~_2
  T4  phi_i^{n+1} = phi_i - dt D(u A phi_i - kM G mu~_i)      (i = 1, 2)
  T5  m = A(rho_lin(phi^n)) u^n - (kM/2) sum_{i=1,2} (rho_i - rho_3) G mu~_i
  T6  rho^{n+1}, eta^{n+1} from the pulled-back c_i^{n+1}
  T7  momentum as S7 of the binary step with the force above
  T8, T9 pressure and projection as S8, S9 (We is the pressure scale).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence

import numpy as np

from .grid import MACGrid
from .chns import ch_solve_spectral, dpsi, momentum_solve, pressure_solve, psi, skew_advection


@dataclasses.dataclass
class Params3:
    """rho[i], eta[i]: density and viscosity of phase i (i = 0, 1, 2 for phases
    1, 2, 3); sigma = (sigma_12, sigma_13, sigma_23).  We scales the pressure
    only (the binary step's 1/We grad p); the capillary forces come from
    sigma."""
    rho: Sequence[float]
    eta: Sequence[float]
    sigma: Sequence[float]
    Re: float
    We: float
    Cn: float
    Pe: float
    inv_Fr: float
    dt: float
    S: float = 2.0

    @staticmethod
    def from_props(pr) -> "Params3":
        return Params3(tuple(pr.rho3), tuple(pr.eta3), tuple(pr.sigma3), pr.Re, pr.We, pr.Cn, pr.Pe, pr.inv_Fr,
                       pr.dt, pr.S)


def spreading(sigma: Sequence[float]):
    """Sigma_i = sigma_ij + sigma_ik - sigma_jk for sigma = (s12, s13, s23)."""
    s12, s13, s23 = sigma
    return (s12 + s13 - s23, s12 + s23 - s13, s13 + s23 - s12)


def weights(sigma: Sequence[float]):
    """w_i = Sigma_T / (3 Sigma_i) with 3 / Sigma_T = sum_i 1 / Sigma_i."""
    Sg = spreading(sigma)
    if min(Sg) <= 0.0:
        raise ValueError("spreading coefficients must be positive")
    inv_sum = sum(1.0 / s for s in Sg)
    return tuple((1.0 / s) / inv_sum for s in Sg)


def third(phi1: np.ndarray, phi2: np.ndarray) -> np.ndarray:
    return -1.0 - phi1 - phi2


def clamp01(c):
    return np.clip(c, 0.0, 1.0)


def mixture(prm: Params3, phis: List[np.ndarray], key: str, pull: bool = True) -> np.ndarray:
    """sum_i q_i c_i (c_i pulled back into [0, 1] if pull) for q = rho or eta."""
    q = prm.rho if key == "rho" else prm.eta
    out = np.zeros_like(phis[0])
    for i in range(3):
        c = 0.5 * (1.0 + phis[i])
        out = out + q[i] * (clamp01(c) if pull else c)
    return out


def step3(g: MACGrid, st: Dict, prm: Params3, ch_only: bool = False) -> Dict:
    """One step of Algorithm T.  st = {'phi': [phi_1, phi_2], 'u': [..], 'p'}.
    Returns {'phi': [phi_1, phi_2], 'u', 'p', 'mu': [mu~_1, mu~_2]} and the
    intermediates 'phihat', 'ustar', 'rho', 'eta', 'm'."""
    d = g.dim
    p1, p2 = st["phi"]
    p3 = third(p1, p2)
    phis = [p1, p2, p3]
    u = st["u"]
    dt, Cn, S = prm.dt, prm.Cn, prm.S
    kM = 1.0 / (prm.Pe * Cn)
    w = weights(prm.sigma)
    Sg = spreading(prm.sigma)

    # T1, T2
    Lam = dpsi(p1) + dpsi(p2) + dpsi(p3)
    a_ch, b_ch = dt * kM * S, dt * kM * Cn * Cn
    Fa, phihat, mus, phin = [], [], [], []
    for i in range(2):
        F = [u[a] * g.avg(phis[i], a) for a in range(d)]
        r = phis[i] - dt * g.div(F) + dt * kM * g.lap(dpsi(phis[i]) - S * phis[i] - w[i] * Lam)
        ph = ch_solve_spectral(g, r, a_ch, b_ch)
        # T3
        mu = dpsi(phis[i]) + S * (ph - phis[i]) - Cn * Cn * g.lap(ph) - w[i] * Lam
        Fa.append(F)
        phihat.append(ph)
        mus.append(mu)
    mus.append(-mus[0] - mus[1])
    Gmu = [[g.grad(mus[i], a) for a in range(d)] for i in range(3)]
    # T4
    for i in range(2):
        phin.append(phis[i] - dt * g.div([Fa[i][a] - kM * Gmu[i][a] for a in range(d)]))
    phis_new = [phin[0], phin[1], third(phin[0], phin[1])]
    if ch_only:
        return {"phi": phin, "u": [x.copy() for x in u], "p": st["p"].copy(), "mu": mus[:2], "phihat": phihat}

    # T5  consistent mass flux
    rho_lin_old = mixture(prm, phis, "rho", pull=False)
    m = []
    for a in range(d):
        J = -(0.5 * kM) * sum((prm.rho[i] - prm.rho[2]) * Gmu[i][a] for i in range(2))
        ma = g.avg(rho_lin_old, a) * u[a] + J
        m.append(np.where(g.wall_face_mask(a), 0.0, ma))

    # T6
    rho_old = mixture(prm, phis, "rho")
    rho_new = mixture(prm, phis_new, "rho")
    eta_new = mixture(prm, phis_new, "eta")
    rhof_old = [g.avg(rho_old, a) for a in range(d)]
    rhof_new = [g.avg(rho_new, a) for a in range(d)]

    # T7
    ustar = []
    for a in range(d):
        rhs = 0.5 * (rhof_new[a] + rhof_old[a]) / dt * u[a]
        rhs = rhs - skew_advection(g, m, u[a], a)
        force = -(0.5 / Cn) * sum(Sg[i] * g.avg(phis[i], a) * Gmu[i][a] for i in range(3))
        rhs = rhs + force
        if a == 1 and prm.inv_Fr != 0.0:
            rhs = rhs - rhof_new[a] * prm.inv_Fr
        ustar.append(momentum_solve(g, a, rhof_new[a], eta_new, prm, rhs))

    # T8, T9
    p = pressure_solve(g, rhof_new, -(prm.We / dt) * g.div(ustar))
    u_new = []
    for a in range(d):
        ua = ustar[a] - (dt / prm.We) * g.grad(p, a) / rhof_new[a]
        u_new.append(np.where(g.wall_face_mask(a), 0.0, ua))
    return {"phi": phin, "u": u_new, "p": p, "mu": mus[:2], "phihat": phihat, "ustar": ustar,
            "rho": rho_new, "eta": eta_new, "m": m}


def run3(g: MACGrid, st: Dict, prm: Params3, steps: int, **kw) -> Dict:
    for _ in range(steps):
        st = step3(g, st, prm, **kw)
    return st


def diagnostics3(g: MACGrid, st: Dict, prm: Params3) -> Dict[str, float]:
    """Masses sum c_i h^d of the three phases, the discrete energy
    1/2 sum rho_f u^2 h^d + E_free + inv_Fr sum rho y h^d (E_free as in the
    module docstring, gradients on faces), max|u|, max|D u|."""
    d = g.dim
    hd = g.h ** d
    p1, p2 = st["phi"]
    phis = [p1, p2, third(p1, p2)]
    u = st["u"]
    Sg = spreading(prm.sigma)
    rho = mixture(prm, phis, "rho")
    kin = sum(0.5 * float(np.sum(g.avg(rho, a) * u[a] * u[a])) for a in range(d)) * hd
    free = 0.0
    for i in range(3):
        grad2 = sum(float(np.sum(g.grad(phis[i], a) ** 2)) for a in range(d))
        free += 0.5 * Sg[i] * (float(np.sum(psi(phis[i]))) + 0.5 * prm.Cn ** 2 * grad2) * hd / prm.Cn
    grav = prm.inv_Fr * float(np.sum(rho * g.coords()[1])) * hd if prm.inv_Fr != 0.0 else 0.0
    out = {"mass%d" % (i + 1): float(np.sum(0.5 * (1.0 + phis[i]))) * hd for i in range(3)}
    out.update({"energy": kin + free + grav, "kinetic": kin, "free": free,
                "umax": max(float(np.abs(x).max()) for x in u), "divmax": float(np.abs(g.div(u)).max())})
    return out
