"""Algorithm S: one split time step of the two-phase CHNS model (oracle).

Test infrastructure only (see the package docstring).  Every linear system is
solved exactly: the constant-coefficient Cahn-Hilliard operator by FFT / DCT
diagonalisation (sparse LU as a cross-check), the momentum and pressure
systems by sparse LU (SuperLU) -- 2D -- or by conjugate gradients to a
relative residual of 1e-14 -- 3D.

Paper anchors (section / equation of arXiv 2009.06628):
  * mixture maps rho = alpha phi + beta, eta = gamma phi + xi: governing
    equations, eqn. alpha_beta_defn;
  * momentum / thermo-consistency / solenoidality / continuity / chemical
    potential / CH equations: eqns. nav_stokes ... phi_eqn;
  * psi = (phi^2 - 1)^2 / 4, psi' = phi^3 - phi: eqn. free_energy;
  * total energy: eqn. energy_functional;
  * pull-back phi* = clamp(phi, -1, 1) used only for rho and eta: remark
    phi_pullback (eqn. phi_for_density);
  * mass conservation under no-flux / no-slip walls: proposition
    mass_conservation;
  * surface tension as (1/(We Cn)) phi grad mu: lemma forcing_equivalent and
    the strong-equivalence corollary in the appendix;
  * skew-symmetric advection B1 + B2 = m_j d_j v_i + v_i d_j m_j / 2: appendix
    remark skew-symmetry.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import MACGrid


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    rho_minus: float
    eta_minus: float
    Re: float
    We: float
    Cn: float
    Pe: float
    inv_Fr: float
    dt: float
    S: float = 2.0

    @staticmethod
    def from_props(pr) -> "Params":
        return Params(pr.rho_minus, pr.eta_minus, pr.Re, pr.We, pr.Cn, pr.Pe, pr.inv_Fr, pr.dt, pr.S)


def coefficients(prm: Params):
    """alpha, beta, gamma, xi of eqn. alpha_beta_defn with rho_+ = eta_+ = 1."""
    rp, rm = 1.0, prm.rho_minus
    ep, em = 1.0, prm.eta_minus
    return (rp - rm) / (2 * rp), (rp + rm) / (2 * rp), (ep - em) / (2 * ep), (ep + em) / (2 * ep)


def psi(phi):
    """Double-well free-energy density, eqn. free_energy."""
    return 0.25 * (phi * phi - 1.0) ** 2


def dpsi(phi):
    """psi'(phi) = phi^3 - phi, eqn. free_energy."""
    return phi ** 3 - phi


def pullback(phi):
    """phi* of eqn. phi_for_density: phi where |phi| <= 1, sign(phi) otherwise."""
    return np.where(np.abs(phi) <= 1.0, phi, np.sign(phi))


# ---------------------------------------------------------------------------
# Cahn-Hilliard solve  (I - a L + b L L) x = r
# ---------------------------------------------------------------------------

def ch_operator_symbol(g: MACGrid):
    """Eigenvalues of L per axis: periodic -> Fourier modes, walled (cell-centred
    Neumann) -> DCT-II modes.  Returned broadcastable to the cell shape."""
    lam = np.zeros(g.shape)
    for a in range(g.dim):
        n = g.n[a]
        k = np.arange(n)
        if g.periodic[a]:
            la = (2.0 * np.cos(2.0 * np.pi * k / n) - 2.0) / g.h ** 2
        else:
            la = (2.0 * np.cos(np.pi * k / n) - 2.0) / g.h ** 2
        sh = [1] * g.dim
        sh[g.ax(a)] = n
        lam = lam + la.reshape(sh)
    return lam


def _fwd(X, g):
    for a in range(g.dim):
        ax = g.ax(a)
        if g.periodic[a]:
            X = sfft.fft(X, axis=ax)
        else:
            X = sfft.dct(X.real, type=2, axis=ax, norm="ortho") + 1j * sfft.dct(X.imag, type=2, axis=ax, norm="ortho")
    return X


def _inv(X, g):
    for a in reversed(range(g.dim)):
        ax = g.ax(a)
        if g.periodic[a]:
            X = sfft.ifft(X, axis=ax)
        else:
            X = sfft.idct(X.real, type=2, axis=ax, norm="ortho") + 1j * sfft.idct(X.imag, type=2, axis=ax, norm="ortho")
    return X


def ch_solve_spectral(g: MACGrid, r: np.ndarray, a: float, b: float) -> np.ndarray:
    lam = ch_operator_symbol(g)
    X = _fwd(r.astype(np.complex128), g)
    X = X / (1.0 - a * lam + b * lam * lam)
    return _inv(X, g).real


def ch_matrix(g: MACGrid, a: float, b: float):
    L = g.lap_matrix()
    N = L.shape[0]
    return (sp.identity(N, format="csr") - a * L + b * (L @ L)).tocsc()


def ch_solve_sparse(g: MACGrid, r: np.ndarray, a: float, b: float) -> np.ndarray:
    return spla.spsolve(ch_matrix(g, a, b), r.ravel()).reshape(g.shape)


# ---------------------------------------------------------------------------
# momentum: skew advection, viscous operator
# ---------------------------------------------------------------------------

def _at(g: MACGrid, q: np.ndarray, shifts: Dict[int, int], fill=0.0):
    """q[c + sum_b s_b e_b] (fill outside walled axes)."""
    r = q
    for b, s in shifts.items():
        if s:
            r = g.shift(r, b, s, fill=fill)
    return r


def _top(g: MACGrid, b: int) -> np.ndarray:
    """Mask of cells in the last layer of a walled axis b."""
    if g.periodic[b]:
        return np.zeros(g.shape, dtype=bool)
    return g.index(b) == g.n[b] - 1


def _bot(g: MACGrid, b: int) -> np.ndarray:
    if g.periodic[b]:
        return np.zeros(g.shape, dtype=bool)
    return g.index(b) == 0


def mbar(g: MACGrid, m: List[np.ndarray], a: int, b: int):
    """Mass flux m_b interpolated to the two b-faces of the u_a control volume.

    The u_a control volume around face c spans cells c - e_a and c.
      b == a: its faces are the centres of cells c (+) and c - e_a (-);
              m_a averaged from the two faces of that cell.
      b != a: its faces are the edges shared with faces c +- e_b; m_b averaged
              from the b-faces of cells c and c - e_a on that side.
    Walls carry zero flux (stored wall faces of m are zero, the upper wall face
    is zero by definition)."""
    if b == a:
        mp = 0.5 * (m[a] + _at(g, m[a], {a: +1}))
        mm = 0.5 * (_at(g, m[a], {a: -1}) + m[a])
    else:
        mp = 0.5 * (_at(g, m[b], {b: +1}) + _at(g, m[b], {b: +1, a: -1}))
        mm = 0.5 * (m[b] + _at(g, m[b], {a: -1}))
    return mp, mm


def neighbours_u(g: MACGrid, u: np.ndarray, a: int, b: int):
    """u_a at faces c +- e_b with the wall rules: normal velocity is zero on
    the walls, tangential velocity has the no-slip ghost -u."""
    up = _at(g, u, {b: +1})
    um = _at(g, u, {b: -1})
    if not g.periodic[b]:
        if b == a:
            up = np.where(_top(g, b), 0.0, up)
            um = np.where(_bot(g, b), 0.0, um)  # only reached by wall rows
        else:
            up = np.where(_top(g, b), -u, up)
            um = np.where(_bot(g, b), -u, um)
    return up, um


def skew_advection(g: MACGrid, m: List[np.ndarray], u: np.ndarray, a: int) -> np.ndarray:
    """N_a = (advective form + divergence form) / 2 of the momentum flux
    (appendix remark skew-symmetry: B1 + B2 = m_j d_j v_i + v_i d_j m_j / 2,
    which is half the sum of m.grad v and div(m v))."""
    h = g.h
    adv = np.zeros(g.shape)
    dv = np.zeros(g.shape)
    for b in range(g.dim):
        mp, mm = mbar(g, m, a, b)
        up, um = neighbours_u(g, u, a, b)
        adv += 0.5 * (mp * (up - u) + mm * (u - um)) / h
        dv += (mp * 0.5 * (u + up) - mm * 0.5 * (u + um)) / h
    return 0.5 * (adv + dv)


def momentum_matrix(g: MACGrid, a: int, shift_diag: np.ndarray, eta: np.ndarray, Re: float):
    """Sparse matrix of  shift_diag * u - (1/Re) div_h(eta grad_h u)  on the
    faces of axis a (viscous term of eqn. nav_stokes in the paper's
    div(eta grad v_i) form).  Returns (A, unknown_mask): wall faces of a
    walled axis a are not unknowns (u = 0 there).

    Coefficient locations for the u_a control volume of face c:
      b == a: cell centres c (+) and c - e_a (-);
      b != a: edges, eta averaged over the four surrounding cells; on a wall
              edge over the two interior cells, with ghost value -u (no slip).
    """
    h2 = g.h * g.h
    idx = g.cell_index()
    unk = ~g.wall_face_mask(a)
    N = idx.size
    diag = shift_diag.copy()
    rows, cols, vals = [], [], []
    for b in range(g.dim):
        for s in (+1, -1):
            if b == a:
                k = (eta if s > 0 else _at(g, eta, {a: -1}, fill=0.0)) / (Re * h2)
                nb = _at(g, idx, {b: s}, fill=-1)
                # neighbour is a wall face (Dirichlet 0) when outside or stored wall
                if not g.periodic[b]:
                    if s > 0:
                        nb = np.where(_top(g, b), -1, nb)
                    else:
                        nb = np.where(g.index(b) == 1, -1, nb)
                ghost = np.zeros(g.shape, dtype=bool)
            else:
                e1 = eta
                e2 = _at(g, eta, {a: -1}, fill=0.0)
                e3 = _at(g, eta, {b: s}, fill=0.0)
                e4 = _at(g, eta, {b: s, a: -1}, fill=0.0)
                k = 0.25 * (e1 + e2 + e3 + e4)
                ghost = (_top(g, b) if s > 0 else _bot(g, b))
                k = np.where(ghost, 0.5 * (e1 + e2), k) / (Re * h2)
                nb = _at(g, idx, {b: s}, fill=-1)
                nb = np.where(ghost, -1, nb)
            diag = diag + np.where(ghost, 2.0 * k, k)
            ok = unk & (nb >= 0)
            ok = ok & unk.ravel()[np.where(nb >= 0, nb, 0)].reshape(g.shape)
            rows.append(idx[ok]); cols.append(nb[ok]); vals.append(-k[ok])
    rows.append(idx[unk]); cols.append(idx[unk]); vals.append(diag[unk])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    sel = idx[unk]
    return A[sel][:, sel].tocsc(), unk


def _solve_spd(A, b, dim):
    if dim <= 2:
        return spla.spsolve(A, b)
    d = A.diagonal()
    M = sp.diags(1.0 / d)
    x, info = spla.cg(A, b, rtol=1e-14, atol=0.0, maxiter=20000, M=M)
    if info != 0:
        raise RuntimeError("oracle CG did not converge")
    return x


def momentum_solve(g, a, rhof_new, eta, prm, rhs):
    A, unk = momentum_matrix(g, a, rhof_new / prm.dt, eta, prm.Re)
    x = np.zeros(g.shape)
    x[unk] = _solve_spd(A, rhs[unk], g.dim)
    return x


# ---------------------------------------------------------------------------
# pressure
# ---------------------------------------------------------------------------

def pressure_matrix(g: MACGrid, rhof: List[np.ndarray]):
    """-D (rho_f^{-1} G) as a sparse matrix (singular: constants in its kernel)."""
    A = None
    for a in range(g.dim):
        t = -(g.div_matrix(a) @ sp.diags((1.0 / rhof[a]).ravel()) @ g.grad_matrix(a))
        A = t if A is None else A + t
    return A.tocsr()


def pressure_solve(g: MACGrid, rhof: List[np.ndarray], rhs: np.ndarray) -> np.ndarray:
    """Solve -D(rho_f^{-1} G p) = rhs with mean(p) = 0 (rhs projected to mean 0).

    2D: bordered system [[A, 1], [1^T, 0]] by sparse LU.  3D: CG on the
    consistent singular system to 1e-14, then the mean is removed."""
    A = pressure_matrix(g, rhof)
    b = rhs.ravel() - rhs.mean()
    N = b.size
    if g.dim <= 2:
        one = sp.csr_matrix(np.ones((N, 1)))
        K = sp.bmat([[A, one], [one.T, None]], format="csc")
        x = spla.spsolve(K, np.concatenate([b, [0.0]]))[:N]
    else:
        d = A.diagonal()
        x, info = spla.cg(A, b, rtol=1e-14, atol=0.0, maxiter=50000, M=sp.diags(1.0 / d))
        if info != 0:
            raise RuntimeError("oracle pressure CG did not converge")
    x = x - x.mean()
    return x.reshape(g.shape)


# ---------------------------------------------------------------------------
# the step
# ---------------------------------------------------------------------------

def wall_velocity_rhs(g: MACGrid, a: int, eta_new: np.ndarray, prm, wall_u: Optional[Dict]) -> np.ndarray:
    """Right-hand-side term of the momentum rows of component a next to a wall
    that moves tangentially (inhomogeneous Dirichlet data, as the lid of the
    paper's lid-driven cavity): with the no-slip ghost value 2 U - u in place
    of -u, the wall edge adds 2 k U, k = (eta_c + eta_{c-e_a}) / (2 Re h^2)
    the coefficient of that edge in the momentum matrix.  wall_u maps
    (b, side, a) -> face array of component a whose layer next to the wall
    (index 0 along b for side 0, n_b - 1 for side 1) holds U."""
    out = np.zeros(g.shape)
    if not wall_u:
        return out
    e2 = _at(g, eta_new, {a: -1}, fill=0.0)
    kw = 0.5 * (eta_new + e2) / (prm.Re * g.h * g.h)
    for (b, side, comp), U in wall_u.items():
        if comp != a or b == a or g.periodic[b]:
            continue
        mask = _top(g, b) if side else _bot(g, b)
        out = out + np.where(mask, 2.0 * kw * U, 0.0)
    return out


def step(g: MACGrid, st: Dict, prm: Params, forcing: Optional[Dict] = None, ch_solver: str = "spectral",
         ch_only: bool = False, wall_u: Optional[Dict] = None) -> Dict:
    """One step n -> n+1 of Algorithm S.  st = {'phi', 'u': [..], 'p'}.

    Returns a new state dict with 'phi', 'u', 'p', 'mu' and the intermediates
    'phihat', 'ustar', 'rho', 'eta', 'm'.  `forcing` (manufactured-solution
    tests only) may hold 'phi' (cells), 'mu' (cells) and 'u' (faces), all
    evaluated at t^{n+1}.  ch_only=True stops after S4 (velocity and pressure
    are carried over unchanged): the Cahn-Hilliard sub-step alone.  wall_u:
    tangential velocities of moving walls (see wall_velocity_rhs); the
    normal velocity and the mass flux through every wall stay 0, so only
    the viscous wall term of S7 changes."""
    d = g.dim
    phi = st["phi"]
    u = st["u"]
    alpha, beta, gamma, xi = coefficients(prm)
    dt, Cn, S = prm.dt, prm.Cn, prm.S
    kM = 1.0 / (prm.Pe * Cn)           # 1/(Pe Cn) with mobility m(phi) = 1
    f = forcing or {}

    # S1  explicit CH stage: advective flux and the explicit part of mu
    Fa = [u[a] * g.avg(phi, a) for a in range(d)]
    r = phi - dt * g.div(Fa) + dt * kM * g.lap(dpsi(phi) - S * phi)
    if "phi" in f:
        r = r + dt * f["phi"]
    if "mu" in f:
        r = r + dt * kM * g.lap(f["mu"])

    # S2  (I - dt kM S L + dt kM Cn^2 L L) phihat = r
    a_ch, b_ch = dt * kM * S, dt * kM * Cn * Cn
    if ch_solver == "spectral":
        phihat = ch_solve_spectral(g, r, a_ch, b_ch)
    else:
        phihat = ch_solve_sparse(g, r, a_ch, b_ch)

    # S3  chemical potential at n+1 (eqn. mu_eqn, linearised with stabiliser S)
    mu = dpsi(phi) + S * (phihat - phi) - Cn * Cn * g.lap(phihat)
    if "mu" in f:
        mu = mu + f["mu"]

    # S4  flux-form phi update (mass conserved to round-off, proposition
    #     mass_conservation)
    Gmu = [g.grad(mu, a) for a in range(d)]
    phi_new = phi - dt * g.div([Fa[a] - kM * Gmu[a] for a in range(d)])
    if "phi" in f:
        phi_new = phi_new + dt * f["phi"]

    if ch_only:
        return {"phi": phi_new, "u": [x.copy() for x in u], "p": st["p"].copy(), "mu": mu,
                "phihat": phihat, "r_ch": r}

    # S5  thermodynamically consistent flux J and mass flux m
    J = [-(alpha / Cn) * Gmu[a] for a in range(d)]
    rho_lin_old = alpha * phi + beta
    m = [g.avg(rho_lin_old, a) * u[a] + J[a] / prm.Pe for a in range(d)]
    for a in range(d):
        m[a] = np.where(g.wall_face_mask(a), 0.0, m[a])

    # S6  properties with the pull-back
    rho_old = alpha * pullback(phi) + beta
    rho_new = alpha * pullback(phi_new) + beta
    eta_new = gamma * pullback(phi_new) + xi
    rhof_old = [g.avg(rho_old, a) for a in range(d)]
    rhof_new = [g.avg(rho_new, a) for a in range(d)]

    # S7  momentum predictor, component by component
    ustar = []
    for a in range(d):
        rhs = 0.5 * (rhof_new[a] + rhof_old[a]) / dt * u[a]
        rhs = rhs - skew_advection(g, m, u[a], a)
        rhs = rhs - (1.0 / (prm.We * Cn)) * g.avg(phi, a) * Gmu[a]
        if a == 1 and prm.inv_Fr != 0.0:        # g_hat = (0, -1, 0)
            rhs = rhs - rhof_new[a] * prm.inv_Fr
        if "u" in f:
            rhs = rhs + f["u"][a]
        if wall_u:
            rhs = rhs + wall_velocity_rhs(g, a, eta_new, prm, wall_u)
        ustar.append(momentum_solve(g, a, rhof_new[a], eta_new, prm, rhs))

    # S8  pressure:  -D(rho_f^{-1} G p) = -(We/dt) D u*
    p = pressure_solve(g, rhof_new, -(prm.We / dt) * g.div(ustar))

    # S9  projection
    u_new = []
    for a in range(d):
        ua = ustar[a] - (dt / prm.We) * g.grad(p, a) / rhof_new[a]
        ua = np.where(g.wall_face_mask(a), 0.0, ua)
        u_new.append(ua)

    return {"phi": phi_new, "u": u_new, "p": p, "mu": mu,
            "phihat": phihat, "ustar": ustar, "rho": rho_new, "eta": eta_new, "m": m, "r_ch": r}


def run(g: MACGrid, st: Dict, prm: Params, steps: int, **kw) -> Dict:
    for _ in range(steps):
        st = step(g, st, prm, **kw)
    return st


# ---------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------

def diagnostics(g: MACGrid, st: Dict, prm: Params) -> Dict[str, float]:
    """Phase masses, discrete total energy (eqn. energy_functional), max|u|,
    max|D u|.

    Energy E_h = 1/2 sum_a sum_faces rho_f u_a^2 h^d
               + 1/(Cn We) sum [psi(phi) + Cn^2/2 sum_a (G_a phi)^2] h^d
               + inv_Fr sum rho(phi*) y h^d.
    The gravity potential is taken outside the 1/(Cn We) bracket (the work of
    the body force rho g_hat / Fr in the momentum equation)."""
    d = g.dim
    hd = g.h ** d
    phi = st["phi"]
    u = st["u"]
    alpha, beta, gamma, xi = coefficients(prm)
    rho = alpha * pullback(phi) + beta
    kin = 0.0
    for a in range(d):
        kin += 0.5 * float(np.sum(g.avg(rho, a) * u[a] * u[a])) * hd
    grad2 = sum(float(np.sum(g.grad(phi, a) ** 2)) for a in range(d))
    free = (float(np.sum(psi(phi))) * hd + 0.5 * prm.Cn ** 2 * grad2 * hd) / (prm.Cn * prm.We)
    grav = 0.0
    if prm.inv_Fr != 0.0:
        y = g.coords()[1]
        grav = prm.inv_Fr * float(np.sum(rho * y)) * hd
    return {
        "mass_plus": float(np.sum(0.5 * (1.0 + phi))) * hd,
        "mass_minus": float(np.sum(0.5 * (1.0 - phi))) * hd,
        "energy": kin + free + grav,
        "kinetic": kin,
        "free": free,
        "umax": max(float(np.abs(x).max()) for x in u),
        "divmax": float(np.abs(g.div(u)).max()),
    }
