"""Seeded synthetic workloads for the two-phase Cahn-Hilliard Navier-Stokes step.

This module is shared by the CPU oracle, the GPU tests and the benchmark.  It
holds only problem *definitions* (grid, physical parameters, step count) and
initial-condition generators; none of the time-step arithmetic lives here.

Conventions
-----------
* Non-dimensionalisation follows the paper's governing-equations section: the
  "+" fluid is the reference, so rho_plus = eta_plus = 1 and the mixture maps
  are rho(phi) = alpha*phi + beta, eta(phi) = gamma*phi + xi.
* phi = +1 is the carrier fluid, phi = -1 the drop / bubble.
* Arrays are numpy float64, C order, x fastest: shape (ny, nx) in 2D and
  (nz, ny, nx) in 3D.  Face arrays of axis a have the same shape as the cell
  arrays; entry c holds the face between cell c - e_a and cell c.  On a walled
  axis the entry with index 0 along that axis is the wall face (always zero for
  the normal velocity) and the opposite wall face is not stored.
* Interface profiles use the flat equilibrium of the double-well energy,
  phi = tanh(d / (sqrt(2) Cn)), with d the signed distance (positive in the
  carrier).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

PERIODIC = "periodic"
WALL = "wall"


@dataclasses.dataclass
class Props:
    """Physical and numerical parameters of one problem (non-dimensional).

    rho_minus / eta_minus are the density / viscosity of the phi=-1 fluid
    relative to the phi=+1 fluid.  inv_Fr = 0 switches gravity off.
    Pe is the Peclet number; the mobility m(phi) is 1.
    """

    rho_minus: float = 1.0
    eta_minus: float = 1.0
    Re: float = 10.0
    We: float = 1.0
    Cn: float = 0.05
    Pe: float = 1000.0
    inv_Fr: float = 0.0
    dt: float = 1e-4
    S: float = 2.0
    # linear-solver controls (relative residual, iteration cap)
    rtol_ch: float = 1e-15
    rtol_mom: float = 1e-13
    rtol_p: float = 1e-12
    max_iter: int = 300
    # three-phase problems (nphases = 3): density and viscosity of phases
    # 1, 2, 3 and the pairwise surface tensions (sigma_12, sigma_13,
    # sigma_23); rho_minus / eta_minus are then unused and We only scales the
    # pressure
    nphases: int = 2
    rho3: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    eta3: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    sigma3: Tuple[float, float, float] = (1.0, 1.0, 1.0)

    def copy(self, **kw) -> "Props":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Problem:
    name: str
    n: Tuple[int, ...]          # cells per axis (nx, ny[, nz])
    h: float
    bc: Tuple[str, ...]         # per axis: PERIODIC or WALL
    props: Props
    steps: int
    init: str                   # initial-condition recipe name
    init_args: Dict = dataclasses.field(default_factory=dict)

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.n))

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def periodic(self) -> Tuple[bool, ...]:
        return tuple(b == PERIODIC for b in self.bc)

    @property
    def wall_velocity(self) -> Dict:
        """Tangential velocities of moving walls (see wall_velocity())."""
        return wall_velocity(self)


# ---------------------------------------------------------------------------
# coordinates
# ---------------------------------------------------------------------------

def cell_centres(n: Tuple[int, ...], h: float) -> List[np.ndarray]:
    """Cell-centre coordinates x_a = (i_a + 1/2) h broadcast to the cell shape."""
    dim = len(n)
    shape = tuple(reversed(n))
    out = []
    for a in range(dim):
        c = (np.arange(n[a], dtype=np.float64) + 0.5) * h
        sh = [1] * dim
        sh[dim - 1 - a] = n[a]
        out.append(np.broadcast_to(c.reshape(sh), shape).copy())
    return out


def _min_image(d: np.ndarray, L: float, periodic: bool) -> np.ndarray:
    if not periodic:
        return d
    return d - L * np.round(d / L)


def interface(d: np.ndarray, Cn: float) -> np.ndarray:
    """Equilibrium profile phi = tanh(d / (sqrt 2 Cn)); d > 0 in the carrier."""
    return np.tanh(d / (math.sqrt(2.0) * Cn))


# ---------------------------------------------------------------------------
# initial conditions
# ---------------------------------------------------------------------------

def phi_drop(p: Problem, centre, radius) -> np.ndarray:
    X = cell_centres(p.n, p.h)
    r2 = np.zeros(p.shape)
    for a in range(p.dim):
        d = _min_image(X[a] - centre[a], p.n[a] * p.h, p.periodic[a])
        r2 += d * d
    return interface(np.sqrt(r2) - radius, p.props.Cn)


def phi_ellipse(p: Problem, centre, semi_axes) -> np.ndarray:
    """Axis-aligned ellipse; d = F/|grad F| with F = sqrt(sum (x_a/s_a)^2) - 1."""
    X = cell_centres(p.n, p.h)
    q = np.zeros(p.shape)
    g = np.zeros(p.shape)
    for a in range(p.dim):
        d = _min_image(X[a] - centre[a], p.n[a] * p.h, p.periodic[a])
        q += (d / semi_axes[a]) ** 2
        g += (d / semi_axes[a] ** 2) ** 2
    rad = np.sqrt(q)
    grad = np.sqrt(g) / np.maximum(rad, 1e-300)
    dist = np.where(rad > 0, (rad - 1.0) / np.maximum(grad, 1e-300), -min(semi_axes))
    return interface(dist, p.props.Cn)


def drop_set(p: Problem, seed: int, count: int, rmin: float, rmax: float, gap: float):
    """Seeded drop centres / radii by rejection sampling in the periodic box:
    surfaces at least `gap` apart (minimum-image distances)."""
    rng = np.random.default_rng(seed)
    L = [p.n[a] * p.h for a in range(p.dim)]
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place the drops")
        r = rng.uniform(rmin, rmax)
        c = [rng.uniform(0, L[a]) for a in range(p.dim)]
        ok = True
        for c2, r2 in zip(centres, radii):
            d2 = 0.0
            for a in range(p.dim):
                d = _min_image(c[a] - c2[a], L[a], p.periodic[a])
                d2 += d * d
            if math.sqrt(d2) < r + r2 + gap:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    return centres, radii


def phi_drops(p: Problem, centres, radii) -> np.ndarray:
    """Union of spherical drops: d = min_i (|x - c_i| - R_i)."""
    X = cell_centres(p.n, p.h)
    dmin = np.full(p.shape, np.inf)
    for c, r in zip(centres, radii):
        r2 = np.zeros(p.shape)
        for a in range(p.dim):
            d = _min_image(X[a] - c[a], p.n[a] * p.h, p.periodic[a])
            r2 += d * d
        dmin = np.minimum(dmin, np.sqrt(r2) - r)
    return interface(dmin, p.props.Cn)


def phi_slab(p: Problem, height: float) -> np.ndarray:
    """Flat interface at y = height, carrier (phi=+1) below."""
    X = cell_centres(p.n, p.h)
    return interface(height - X[1], p.props.Cn)


def phi_spinodal(p: Problem, seed: int, amp: float = 0.05) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1.0, 1.0, size=p.shape)


def velocity_streamfunction(p: Problem, seed: int, amp: float, kmax: int = 2) -> List[np.ndarray]:
    """Discretely divergence-free MAC velocity from a seeded 2D streamfunction.

    psi lives on cell corners (i h, j h); u_x(face i,j) = (psi(i,j+1) - psi(i,j))/h,
    u_y(face i,j) = -(psi(i+1,j) - psi(i,j))/h.  On walled axes psi is
    multiplied by a profile that vanishes (with zero slope) on the walls, so
    the normal velocity is zero there.  Scaled so that max|u| = amp.
    """
    assert p.dim == 2
    rng = np.random.default_rng(seed)
    nx, ny = p.n
    Lx, Ly = nx * p.h, ny * p.h
    xs = np.arange(nx + 1) * p.h
    ys = np.arange(ny + 1) * p.h
    Xc, Yc = np.meshgrid(xs, ys)  # (ny+1, nx+1)
    psi = np.zeros_like(Xc)
    for kx in range(0, kmax + 1):
        for ky in range(0, kmax + 1):
            if kx == 0 and ky == 0:
                continue
            ph = rng.uniform(0, 2 * np.pi, size=2)
            amp_k = rng.normal()
            fx = np.cos(2 * np.pi * kx * Xc / Lx + ph[0]) if p.periodic[0] else np.cos(np.pi * kx * Xc / Lx)
            fy = np.cos(2 * np.pi * ky * Yc / Ly + ph[1]) if p.periodic[1] else np.cos(np.pi * ky * Yc / Ly)
            psi += amp_k * fx * fy
    if not p.periodic[0]:
        psi *= np.sin(np.pi * Xc / Lx) ** 2
    if not p.periodic[1]:
        psi *= np.sin(np.pi * Yc / Ly) ** 2
    ux = (psi[1:, :nx] - psi[:ny, :nx]) / p.h
    uy = -(psi[:ny, 1:] - psi[:ny, :nx]) / p.h
    if not p.periodic[0]:
        ux[:, 0] = 0.0
    if not p.periodic[1]:
        uy[0, :] = 0.0
    m = max(np.abs(ux).max(), np.abs(uy).max())
    return [ux * (amp / m), uy * (amp / m)]


def velocity_potential3d(p: Problem, seed: int, amp: float, kmax2: int = 4) -> List[np.ndarray]:
    """Discretely divergence-free 3D MAC velocity u = curl_h A (all-periodic grid).

    A_x, A_y, A_z live on cell edges; Fourier modes 1 <= |k|^2 <= kmax2 with
    seeded phases and amplitudes.  Scaled so that max|u| = amp.
    """
    assert p.dim == 3 and all(p.periodic)
    rng = np.random.default_rng(seed)
    nx, ny, nz = p.n
    h = p.h
    L = [nx * h, ny * h, nz * h]
    idx = [np.arange(n_) for n_ in (nx, ny, nz)]
    # coordinates: index i -> i*h (lower corner) or (i+1/2)h (centre)
    def coord(a, centred):
        return (idx[a] + (0.5 if centred else 0.0)) * h
    # A_x at (x centred, y corner, z corner) etc.
    comps = []
    for a in range(3):
        cen = [b == a for b in range(3)]
        Xs = np.meshgrid(coord(2, cen[2]), coord(1, cen[1]), coord(0, cen[0]), indexing="ij")
        Z, Y, X = Xs
        A = np.zeros((nz, ny, nx))
        for kx in range(-2, 3):
            for ky in range(-2, 3):
                for kz in range(-2, 3):
                    k2 = kx * kx + ky * ky + kz * kz
                    if k2 < 1 or k2 > kmax2:
                        continue
                    ph = rng.uniform(0, 2 * np.pi)
                    c = rng.normal()
                    A += c * np.cos(2 * np.pi * (kx * X / L[0] + ky * Y / L[1] + kz * Z / L[2]) + ph)
        comps.append(A)
    Ax, Ay, Az = comps

    def dplus(q, a):  # forward difference along axis a (numpy axis 2-a), periodic
        return (np.roll(q, -1, axis=2 - a) - q) / h

    # u_x at x-face (corner in x, centred in y,z) = dAz/dy - dAy/dz
    ux = dplus(Az, 1) - dplus(Ay, 2)
    uy = dplus(Ax, 2) - dplus(Az, 0)
    uz = dplus(Ay, 0) - dplus(Ax, 1)
    m = max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max())
    return [ux * (amp / m), uy * (amp / m), uz * (amp / m)]


def _drop_distance(p: Problem, centres, radii) -> np.ndarray:
    """Signed distance to the nearest of the given spheres / discs (negative
    inside), minimum-image on periodic axes."""
    X = cell_centres(p.n, p.h)
    dmin = np.full(p.shape, np.inf)
    for c, r in zip(centres, radii):
        r2 = np.zeros(p.shape)
        for a in range(p.dim):
            d = _min_image(X[a] - c[a], p.n[a] * p.h, p.periodic[a])
            r2 += d * d
        dmin = np.minimum(dmin, np.sqrt(r2) - r)
    return dmin


def ternary_fields(p: Problem) -> List[np.ndarray]:
    """phi_1, phi_2 of a three-phase initial condition (phi_i = 2 c_i - 1;
    phase 3 fills the rest)."""
    a = p.init_args
    Cn = p.props.Cn
    if p.init == "ternary_drops":
        cs_, rs_ = drop_set(p, a["seed"], 2 * a["count"], a["rmin"], a["rmax"], a["gap"])
        # drops alternate between the two phases in placement order
        d1 = _drop_distance(p, cs_[0::2], rs_[0::2])
        d2 = _drop_distance(p, cs_[1::2], rs_[1::2])
        return [-interface(d1, Cn), -interface(d2, Cn)]
    if p.init == "ternary_layers":
        # phase 1 below y1, phase 2 between y1 and y2, phase 3 above y2
        X = cell_centres(p.n, p.h)
        y = X[1]
        y1, y2 = a["y1"], a["y2"]
        c1 = 0.5 * (1.0 - interface(y - y1, Cn))
        c12 = 0.5 * (1.0 - interface(y - y2, Cn))
        return [2.0 * c1 - 1.0, 2.0 * (c12 - c1) - 1.0]
    if p.init == "ternary_pair":
        # two-phase drop of phase a["inside"] in phase a["outside"]; the third is absent
        d = _drop_distance(p, [a["centre"]], [a["radius"]])
        phi_in = -interface(d, Cn)
        out = [None, None, None]
        out[a["inside"]] = phi_in
        out[a["outside"]] = -phi_in
        k = 3 - a["inside"] - a["outside"]
        out[k] = np.full(p.shape, -1.0)
        return out[:2]
    if p.init == "ternary_mix":
        rng = np.random.default_rng(a.get("seed", 0))
        c = 1.0 / 3.0 + a.get("amp", 0.05) * rng.uniform(-1.0, 1.0, size=(2,) + p.shape)
        return [2.0 * c[0] - 1.0, 2.0 * c[1] - 1.0]
    raise ValueError(f"unknown three-phase initial condition {p.init!r}")


def initial_state(p: Problem) -> Dict[str, object]:
    """Return {'phi': cells, 'u': [faces per axis], 'p': cells} in float64;
    for three-phase problems 'phi' is the list [phi_1, phi_2]."""
    a = p.init_args
    if p.props.nphases == 3:
        phi = [np.ascontiguousarray(x, dtype=np.float64) for x in ternary_fields(p)]
    elif p.init == "drop":
        phi = phi_drop(p, a["centre"], a["radius"])
    elif p.init == "ellipse":
        phi = phi_ellipse(p, a["centre"], a["semi_axes"])
    elif p.init == "slab":
        phi = phi_slab(p, a["height"])
    elif p.init == "drops":
        cs_, rs_ = drop_set(p, a["seed"], a["count"], a["rmin"], a["rmax"], a["gap"])
        phi = phi_drops(p, cs_, rs_)
    elif p.init == "rt_surface":
        X = cell_centres(p.n, p.h)
        gz = a["amp"] * (np.cos(2 * np.pi * X[0]) + np.cos(2 * np.pi * X[2]))
        phi = interface(X[1] - a["h0"] - gz, p.props.Cn)
    elif p.init == "spinodal":
        phi = phi_spinodal(p, a.get("seed", 0), a.get("amp", 0.05))
    elif p.init == "const":
        phi = np.full(p.shape, float(a.get("value", 1.0)))
    else:
        raise ValueError(f"unknown initial condition {p.init!r}")
    if a.get("velocity") == "stream":
        u = velocity_streamfunction(p, a.get("vseed", 1), a.get("vamp", 1e-2))
    elif a.get("velocity") == "potential3d":
        u = velocity_potential3d(p, a.get("vseed", 1), a.get("vamp", 1e-2))
    else:
        u = [np.zeros(p.shape) for _ in range(p.dim)]
    if p.props.nphases != 3:
        phi = np.ascontiguousarray(phi, dtype=np.float64)
    return {"phi": phi,
            "u": [np.ascontiguousarray(x, dtype=np.float64) for x in u],
            "p": np.zeros(p.shape)}


# ---------------------------------------------------------------------------
# named problems
# ---------------------------------------------------------------------------

def static_drop(n: int = 64, steps: int = 100, **kw) -> Problem:
    """Static drop: unit periodic box, R = 0.25 centred, density and viscosity
    ratio 10 (carrier heavier), sigma = 1 (We = 1), Cn = 1.5 h, mobility 1e-3
    (Pe = 1/(M sigma) = 1000), Re = 10, no gravity, dt = 1e-4, u0 = 0."""
    h = 1.0 / n
    pr = Props(rho_minus=0.1, eta_minus=0.1, Re=10.0, We=1.0, Cn=1.5 * h,
               Pe=1000.0, inv_Fr=0.0, dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("static_drop_%d" % n, (n, n), h, (PERIODIC, PERIODIC), pr, steps,
                   "drop", {"centre": (0.5, 0.5), "radius": 0.25})


def rising_bubble(nx: int = 256, steps: int = 2000, **kw) -> Problem:
    """Rising bubble: non-dimensional box [0,2] x [0,4] (bubble diameter 1),
    nx x 2nx cells, periodic sides, no-slip top and bottom.  Bubble radius 0.5
    at (1,1); rho_-/rho_+ = 1e-3, eta_-/eta_+ = 1e-2; We = Eo = 10, Re = Ar = 35,
    Fr = 1 with gravity along -y; Cn = 1.5 h; 1/Pe = 3 Cn^2; dt = 2.5e-4."""
    h = 2.0 / nx
    Cn = 1.5 * h
    pr = Props(rho_minus=1e-3, eta_minus=1e-2, Re=35.0, We=10.0, Cn=Cn,
               Pe=1.0 / (3.0 * Cn * Cn), inv_Fr=1.0, dt=2.5e-4)
    pr = pr.copy(**kw)
    return Problem("rising_bubble_%dx%d" % (nx, 2 * nx), (nx, 2 * nx), h, (PERIODIC, WALL),
                   pr, steps, "drop", {"centre": (1.0, 1.0), "radius": 0.5})


def adjoint_drop(n: int = 128, steps: int = 400, sigma: float = 1.0, mobility: float = 1e-3, **kw) -> Problem:
    """Oscillating drop: unit periodic box, initial ellipse with semi-axes
    0.3 (x) / 0.2 (y), ratios 10/10, Re = 10, Cn = 1.5 h, dt = 1e-4.
    Surface tension sigma and mobility M enter as We = 1/sigma, Pe = 1/(M sigma)."""
    h = 1.0 / n
    pr = Props(rho_minus=0.1, eta_minus=0.1, Re=10.0, We=1.0 / sigma, Cn=1.5 * h,
               Pe=1.0 / (mobility * sigma), inv_Fr=0.0, dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("adjoint_drop_%d" % n, (n, n), h, (PERIODIC, PERIODIC), pr, steps,
                   "ellipse", {"centre": (0.5, 0.5), "semi_axes": (0.3, 0.2)})


def flat_interface(nx: int = 32, ny: int = 32, steps: int = 100, gravity: bool = True, **kw) -> Problem:
    """Flat interface at rest: x periodic, y walls, heavy carrier below."""
    h = 1.0 / nx
    pr = Props(rho_minus=0.1, eta_minus=0.1, Re=10.0, We=1.0, Cn=1.5 * h, Pe=1000.0,
               inv_Fr=1.0 if gravity else 0.0, dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("flat_%dx%d" % (nx, ny), (nx, ny), h, (PERIODIC, WALL), pr, steps,
                   "slab", {"height": 0.5 * ny * h})


def spinodal(n: int = 32, seed: int = 7, steps: int = 1000, bc=(PERIODIC, PERIODIC), **kw) -> Problem:
    h = 1.0 / n
    pr = Props(rho_minus=0.1, eta_minus=0.1, Re=10.0, We=1.0, Cn=1.5 * h, Pe=1000.0, dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("spinodal_%d" % n, (n,) * len(bc), h, tuple(bc), pr, steps,
                   "spinodal", {"seed": seed, "amp": 0.05})


def drop3d(n: int = 32, steps: int = 10, **kw) -> Problem:
    """3D periodic drop with a divergence-free random velocity perturbation."""
    h = 1.0 / n
    pr = Props(rho_minus=0.1, eta_minus=0.1, Re=10.0, We=1.0, Cn=1.5 * h, Pe=1000.0, dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("drop3d_%d" % n, (n, n, n), h, (PERIODIC,) * 3, pr, steps, "drop",
                   {"centre": (0.5, 0.5, 0.5), "radius": 0.25, "velocity": "potential3d",
                    "vseed": 3, "vamp": 1e-2})


def drops3d(n: int = 128, steps: int = 500, seed: int = 3, count: int = 16, **kw) -> Problem:
    """3D drops in a periodic unit box (two-phase version of the three-phase
    drop configuration): `count` drops of the phi=-1 fluid with seeded radii
    in [0.05, 0.12] and centres at least 6 Cn apart; density and viscosity
    ratio 100 (carrier heavier), sigma = 1 (We = 1), Re = 10, Cn = 1.5 h (the
    drop layout uses the 128^3 gap 6 x 1.5/128 at every resolution),
    1/Pe = 3 Cn^2, dt = 1e-4, divergence-free velocity perturbation of
    amplitude 1e-2 (Fourier modes 1 <= |k|^2 <= 4, seeded)."""
    h = 1.0 / n
    Cn = 1.5 * h
    pr = Props(rho_minus=0.01, eta_minus=0.01, Re=10.0, We=1.0, Cn=Cn, Pe=1.0 / (3.0 * Cn * Cn), dt=1e-4)
    pr = pr.copy(**kw)
    return Problem("drops3d_%d" % n, (n, n, n), h, (PERIODIC,) * 3, pr, steps, "drops",
                   {"seed": seed, "count": count, "rmin": 0.05, "rmax": 0.12, "gap": 6 * 1.5 / 128,
                    "velocity": "potential3d", "vseed": seed + 100, "vamp": 1e-2})


def lid_driven_cavity3d(n: int = 128, steps: int = 200, **kw) -> Problem:
    """Two-phase lid-driven cavity (the paper's 3D lid-driven cavity): unit
    cube with walls on every side, the two fluids in the lower and upper
    halves with a flat interface at y = 1/2 (equilibrium profile), density
    and viscosity ratio 1, Re = 100, We = 100, Cn = 1.5 h, 1/Pe = 3 Cn^2,
    fluid at rest; the top wall (y = 1) moves along x with
    u_x = 16 x (1 - x) z (1 - z) (zero at its edges), the other walls are
    no-slip.  dt = 1e-3 (advective CFL 0.128 at 128^3 with the lid speed 1)."""
    h = 1.0 / n
    Cn = 1.5 * h
    pr = Props(rho_minus=1.0, eta_minus=1.0, Re=100.0, We=100.0, Cn=Cn, Pe=1.0 / (3.0 * Cn * Cn), dt=1e-3)
    pr = pr.copy(**kw)
    return Problem("lid_driven_cavity3d_%d" % n, (n, n, n), h, (WALL,) * 3, pr, steps, "slab",
                   {"height": 0.5, "lid": "paper"})


def rayleigh_taylor3d(n: int = 64, steps: int = 200, **kw) -> Problem:
    """Reduced 3D Rayleigh-Taylor instability (one wavelength of the paper's
    3D initial condition): box [0,1] x [0,4] x [0,1] of n x 4n x n cells, walls
    on every side, the heavy fluid (phi = +1, the reference) above the
    interface y = h0 + g(x, z), h0 = 2, g = 0.05 (cos 2 pi x + cos 2 pi z);
    Atwood number 0.15 (rho_- = 0.85 / 1.15), viscosity ratio 1, Re = 1000,
    We = 1000, Fr = 1 with gravity along -y, Cn = 1.5 h, 1/Pe = 3 Cn^2,
    dt = 2.5e-3, fluid at rest."""
    h = 1.0 / n
    Cn = 1.5 * h
    pr = Props(rho_minus=0.85 / 1.15, eta_minus=1.0, Re=1000.0, We=1000.0, Cn=Cn, Pe=1.0 / (3.0 * Cn * Cn),
               inv_Fr=1.0, dt=2.5e-3)
    pr = pr.copy(**kw)
    return Problem("rayleigh_taylor3d_%d" % n, (n, 4 * n, n), h, (WALL,) * 3, pr, steps, "rt_surface",
                   {"h0": 2.0, "amp": 0.05})


def wall_velocity(p: Problem) -> Dict[Tuple[int, int, int], np.ndarray]:
    """Tangential velocities of moving walls: {(b, side, a): face array of
    component a whose layer next to wall (b, side) holds the wall speed}.
    Empty for problems whose walls are all at rest."""
    a = p.init_args
    if a.get("lid") == "paper":
        # u_x on the top wall y = 1 at the x-face positions (i h, 1, (k + 1/2) h)
        X = cell_centres(p.n, p.h)
        xf = X[0] - 0.5 * p.h
        z = X[2]
        return {(1, 1, 0): 16.0 * xf * (1.0 - xf) * z * (1.0 - z)}
    if a.get("lid") == "couette":
        return {(1, 1, 0): np.full(p.shape, float(a["speed"]))}
    return {}


def sample_surface_tensions(seed: int, lo: float = 0.5, hi: float = 1.5) -> Tuple[float, float, float]:
    """Pairwise surface tensions (sigma_12, sigma_13, sigma_23) ~ U[lo, hi]
    each, redrawn until every spreading coefficient
    Sigma_i = sigma_ij + sigma_ik - sigma_jk is positive."""
    rng = np.random.default_rng(seed)
    while True:
        s12, s13, s23 = (float(x) for x in rng.uniform(lo, hi, size=3))
        if min(s12 + s13 - s23, s12 + s23 - s13, s13 + s23 - s12) > 0.0:
            return (s12, s13, s23)


def ternary_drops3d(n: int = 128, steps: int = 500, seed: int = 3, count: int = 8, **kw) -> Problem:
    """Three-phase drops: unit periodic box, `count` drops of phase 1 and
    `count` of phase 2 (alternating in the seeded placement order, radii
    U[0.05, 0.12], surfaces at least 6 x 1.5/128 apart) in a carrier phase 3;
    pairwise surface tensions U[0.5, 1.5] (seeded, all spreading coefficients
    positive); densities (100, 10, 1), viscosities (1/Re) eta_i = 1e-2
    (Re = 1, eta_i = 1e-2); Cn = 1.5 h; 1/Pe = 3 Cn^2; dt = 1e-4; We = 1
    (pressure scale); divergence-free velocity perturbation of amplitude 1e-2
    (Fourier modes 1 <= |k|^2 <= 4, seeded)."""
    h = 1.0 / n
    Cn = 1.5 * h
    pr = Props(Re=1.0, We=1.0, Cn=Cn, Pe=1.0 / (3.0 * Cn * Cn), dt=1e-4, nphases=3,
               rho3=(100.0, 10.0, 1.0), eta3=(1e-2, 1e-2, 1e-2), sigma3=sample_surface_tensions(seed))
    pr = pr.copy(**kw)
    return Problem("ternary_drops3d_%d" % n, (n, n, n), h, (PERIODIC,) * 3, pr, steps, "ternary_drops",
                   {"seed": seed, "count": count, "rmin": 0.05, "rmax": 0.12, "gap": 6 * 1.5 / 128,
                    "velocity": "potential3d", "vseed": seed + 100, "vamp": 1e-2})


def ternary_problem(n: Tuple[int, ...], init: str, init_args: Dict, bc=None, steps: int = 10,
                    **kw) -> Problem:
    """A small three-phase test problem on a box of cell size 1/n[0]
    (defaults: Re = 10, We = 1, Cn = 1.5 h, Pe = 1000, dt = 1e-4, densities
    (1, 0.1, 0.5), viscosities (1, 0.1, 0.3), sigma (1, 0.8, 1.2))."""
    n = tuple(n)
    h = 1.0 / n[0]
    bc = tuple(bc) if bc is not None else (PERIODIC,) * len(n)
    pr = Props(Re=10.0, We=1.0, Cn=1.5 * h, Pe=1000.0, dt=1e-4, nphases=3, rho3=(1.0, 0.1, 0.5),
               eta3=(1.0, 0.1, 0.3), sigma3=(1.0, 0.8, 1.2))
    pr = pr.copy(**kw)
    return Problem("ternary_%s_%s" % (init, "x".join(map(str, n))), n, h, bc, pr, steps, init, dict(init_args))


def oscillating_drop(n: int, semi_axes, rho_ratio: float, eta_ratio: float, sigma: float = 1.0,
                     mobility: float = 1e-3, steps: int = 200, name: Optional[str] = None, **kw) -> Problem:
    """One member of the batched ensemble: unit periodic box, centred
    axis-aligned ellipse, density / viscosity ratios rho_+/rho_- and
    eta_+/eta_-, Re = 10, Cn = 1.5 h, We = 1/sigma, Pe = 1/(M sigma), and the
    capillary time-step bound dt = min(1e-4, 1/2 sqrt((rho_+ + rho_-) h^3 / (2 pi sigma)))."""
    h = 1.0 / n
    rho_minus = 1.0 / rho_ratio
    dt = min(1e-4, 0.5 * math.sqrt((1.0 + rho_minus) * h ** 3 / (2.0 * math.pi * sigma)))
    pr = Props(rho_minus=rho_minus, eta_minus=1.0 / eta_ratio, Re=10.0, We=1.0 / sigma, Cn=1.5 * h,
               Pe=1.0 / (mobility * sigma), inv_Fr=0.0, dt=dt)
    pr = pr.copy(**kw)
    return Problem(name or "osc_drop_%d" % n, (n, n), h, (PERIODIC, PERIODIC), pr, steps,
                   "ellipse", {"centre": (0.5, 0.5), "semi_axes": tuple(semi_axes)})


def ensemble(count: int = 512, seed: int = 4, sizes=(64, 96, 128, 192, 256), steps: int = 200,
             **kw) -> List[Problem]:
    """Batched ensemble of oscillating drops: n ~ U(sizes), semi-axes
    U[0.2, 0.3] each, rho_+/rho_- ~ logU[1, 1000], eta_+/eta_- ~ logU[1, 100]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        ax = rng.uniform(0.2, 0.3, size=2)
        rr = float(np.exp(rng.uniform(0.0, math.log(1000.0))))
        er = float(np.exp(rng.uniform(0.0, math.log(100.0))))
        out.append(oscillating_drop(n, ax, rr, er, steps=steps, name="ens%d_%d" % (i, n), **kw))
    return out


def ensemble_stratified(per_size: int = 3, seed: int = 4, sizes=(64, 96, 128, 192, 256), steps: int = 20,
                        **kw) -> List[Problem]:
    """A few members of every size (parity tests of the batched form): the
    first per_size members of each size drawn from the ensemble's generator."""
    pool = ensemble(count=64 * len(sizes) * per_size, seed=seed, sizes=sizes, steps=steps, **kw)
    out = []
    for n in sizes:
        out += [p for p in pool if p.n[0] == n][:per_size]
    return out


# Solver tolerances of the precision form (FP64 CG with the FP32 multigrid
# preconditioner): its budget is 1e-5 relative to the FP64 oracle, so the solves
# stop at these looser relative residuals.  Over the 500 steps of the 128^3
# three-phase drops the state stays within 1.5e-8 of the FP64 run at the
# parity tolerances (1e-9 / 1e-8 for momentum / pressure: 2.3e-7 with 1e-8 /
# 1e-7, 1.3e-5 with 1e-8 / 1e-6), three orders of magnitude inside the budget.
PRECISION_FORM_TOLERANCES = dict(rtol_ch=1e-10, rtol_mom=1e-9, rtol_p=1e-8)


def problem_by_name(name: str) -> Problem:
    table = {
        "static_drop": static_drop,
        "rising_bubble": rising_bubble,
        "adjoint_drop": adjoint_drop,
    }
    return table[name]()
