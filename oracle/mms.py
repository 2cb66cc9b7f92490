"""Manufactured-solution forcing (oracle, test infrastructure).

Fields of the paper's manufactured-solution experiment (2D, unit square with
walls):  v = (pi sin^2(pi x) sin(2 pi y) sin t, -pi sin(2 pi x) sin^2(pi y) sin t),
p = cos(pi x) sin(pi y) sin t,  phi = mu = cos(pi x) cos(pi y) sin t,
with Re = 10, We = 1, Cn = 1, Pe = 3, Fr = 1 and density ratio 1 (viscosity
ratio 1 assumed).  With unit density ratio alpha = 0, so rho = eta = 1 and
J = 0.  The forcing is the residual of the continuous equations as the split
step discretises them (surface tension in the potential form
(1/(We Cn)) phi grad mu, so p is the modified pressure):

  f_phi = phi_t + div(v phi) - (1/(Pe Cn)) lap mu
  f_mu  = mu - psi'(phi) + Cn^2 lap phi
  f_v   = v_t + (v.grad) v + (1/We) grad p - (1/Re) lap v
          + (1/(We Cn)) phi grad mu + inv_Fr e_y
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sy

X, Y, T = sy.symbols("x y t", real=True)
PI = sy.pi


def exact_fields():
    vx = PI * sy.sin(PI * X) ** 2 * sy.sin(2 * PI * Y) * sy.sin(T)
    vy = -PI * sy.sin(2 * PI * X) * sy.sin(PI * Y) ** 2 * sy.sin(T)
    p = sy.cos(PI * X) * sy.sin(PI * Y) * sy.sin(T)
    phi = sy.cos(PI * X) * sy.cos(PI * Y) * sy.sin(T)
    mu = phi
    return vx, vy, p, phi, mu


@functools.lru_cache(maxsize=None)
def forcing_functions(Re, We, Cn, Pe, inv_Fr):
    vx, vy, p, phi, mu = exact_fields()
    lap = lambda q: sy.diff(q, X, 2) + sy.diff(q, Y, 2)
    f_phi = sy.diff(phi, T) + sy.diff(vx * phi, X) + sy.diff(vy * phi, Y) - lap(mu) / (Pe * Cn)
    f_mu = mu - (phi ** 3 - phi) + Cn ** 2 * lap(phi)
    f_vx = (sy.diff(vx, T) + vx * sy.diff(vx, X) + vy * sy.diff(vx, Y) + sy.diff(p, X) / We
            - lap(vx) / Re + phi * sy.diff(mu, X) / (We * Cn))
    f_vy = (sy.diff(vy, T) + vx * sy.diff(vy, X) + vy * sy.diff(vy, Y) + sy.diff(p, Y) / We
            - lap(vy) / Re + phi * sy.diff(mu, Y) / (We * Cn) + inv_Fr)
    mk = lambda e: sy.lambdify((X, Y, T), e, "numpy")
    return {k: mk(e) for k, e in dict(phi=f_phi, mu=f_mu, vx=f_vx, vy=f_vy,
                                        ex_phi=phi, ex_vx=vx, ex_vy=vy, ex_p=p).items()}


def _b(v, shape):
    return np.broadcast_to(np.asarray(v, dtype=np.float64), shape).copy()


def forcing(g, prm, t):
    """Forcing dict for oracle.chns.step at time t (cells / staggered faces)."""
    F = forcing_functions(prm.Re, prm.We, prm.Cn, prm.Pe, prm.inv_Fr)
    xc, yc = g.coords()
    xf = g.index(0) * g.h  # x-face location
    yf = g.index(1) * g.h
    return {"phi": _b(F["phi"](xc, yc, t), g.shape), "mu": _b(F["mu"](xc, yc, t), g.shape),
            "u": [_b(F["vx"](xf, yc, t), g.shape), _b(F["vy"](xc, yf, t), g.shape)]}


def exact_state(g, prm, t):
    F = forcing_functions(prm.Re, prm.We, prm.Cn, prm.Pe, prm.inv_Fr)
    xc, yc = g.coords()
    xf = g.index(0) * g.h
    yf = g.index(1) * g.h
    ux = _b(F["ex_vx"](xf, yc, t), g.shape)
    uy = _b(F["ex_vy"](xc, yf, t), g.shape)
    ux[g.wall_face_mask(0)] = 0.0
    uy[g.wall_face_mask(1)] = 0.0
    return {"phi": _b(F["ex_phi"](xc, yc, t), g.shape), "u": [ux, uy],
            "p": _b(F["ex_p"](xc, yc, t), g.shape)}
