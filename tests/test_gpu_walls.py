"""Walls with inhomogeneous Dirichlet data (chns_set_wall_velocity) on the
GPU against the oracle: plane Couette flow, the paper's 3D lid-driven
cavity (reduced and full 128^3), and the reduced 3D Rayleigh-Taylor
instability (walls at rest, gravity)."""
import numpy as np
import pytest

import workloads as W
from oracle import MACGrid, Params, diagnostics, step as ostep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _gpu(prob, steps, init=None):
    import paper_2009_06628_amd as P
    g = P.grid_for_problem(prob)
    st = g.new_state(init if init is not None else W.initial_state(prob))
    stats = g.step(st, steps)
    torch.cuda.synchronize()
    return g, st, stats


def _oracle(prob, steps, init=None):
    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(prob.props)
    st = init if init is not None else W.initial_state(prob)
    for _ in range(steps):
        st = ostep(g, st, prm, wall_u=prob.wall_velocity)
    return g, st, prm


def _compare(sg, so, dim, tol):
    """Relative max-norm errors; velocity components against the largest
    velocity of any component (a component at rest to round-off, as u_y of
    plane Couette flow, is compared with that scale), p with its mean
    removed (skipped when the oracle's p is round-off)."""
    errs = {"phi": relerr(sg["phi"].cpu().numpy(), so["phi"])}
    umax = max(float(np.abs(so["u"][a]).max()) for a in range(dim))
    for a in range(dim):
        errs["u%d" % a] = float(np.abs(sg["u"][a].cpu().numpy() - so["u"][a]).max()) / umax
    pg = sg["p"].cpu().numpy()
    po = so["p"] - so["p"].mean()
    if np.abs(po).max() > 1e-10 * umax:
        errs["p"] = relerr(pg - pg.mean(), po)
    print("parity", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs


def test_couette_steady_profile_and_transient():
    n, U = 32, 0.7
    prob = W.Problem("couette", (16, n), 1.0 / n, (W.PERIODIC, W.WALL),
                     W.Props(rho_minus=1.0, eta_minus=1.0, Re=5.0, We=1.0, Cn=0.1, Pe=100.0, dt=1e-2),
                     1, "const", {"value": 1.0, "lid": "couette", "speed": U})
    shape = tuple(reversed(prob.n))
    j = np.broadcast_to(np.arange(n).reshape(n, 1), shape)
    lin = U * (j + 0.5) / n
    init = {"phi": np.ones(shape), "u": [np.ascontiguousarray(lin, dtype=float), np.zeros(shape)],
            "p": np.zeros(shape)}
    _, sg, _ = _gpu(prob, 20, init)
    assert np.abs(sg["u"][0].cpu().numpy() - lin).max() < 1e-13
    rest = {"phi": np.ones(shape), "u": [np.zeros(shape), np.zeros(shape)], "p": np.zeros(shape)}
    _, sg, _ = _gpu(prob, 50, rest)
    _, so, _ = _oracle(prob, 50, rest)
    _compare(sg, so, 2, 1e-12)


@pytest.mark.parametrize("case", ["lid_driven_cavity_16", "rayleigh_taylor_16x64x16"])
def test_reduced_3d_cases_match_oracle(case):
    if case.startswith("lid"):
        prob, steps = W.lid_driven_cavity3d(16, steps=30), 30
    else:
        prob, steps = W.rayleigh_taylor3d(16, steps=20), 20
    print(case, prob.n, flush=True)
    _, sg, stats = _gpu(prob, steps)
    og, so, prm = _oracle(prob, steps)
    _compare(sg, so, 3, 1e-9)
    d0 = diagnostics(og, W.initial_state(prob), prm)
    for key in ("mass_plus", "mass_minus"):
        assert abs(stats[key] - d0[key]) <= 1e-12 * d0[key]


def test_lid_driven_cavity_full_size_invariants():
    """128^3 lid-driven cavity, 20 steps: both phase masses to 1e-12, every
    wall's normal velocity 0, divergence at the solver tolerance, and the
    mirror symmetry z -> 1 - z of the lid (u_x, u_y, phi even, u_z odd)."""
    prob = W.lid_driven_cavity3d(128, steps=20)
    print("lid-driven cavity 128^3", flush=True)
    import paper_2009_06628_amd as P
    g = P.grid_for_problem(prob)
    st = g.new_state(W.initial_state(prob))
    s0 = g.step(st, 0)
    s1 = g.step(st, 20)
    for key in ("mass_plus", "mass_minus"):
        assert abs(s1[key] - s0[key]) <= 1e-12 * s0[key]
    assert s1["umax"] > 1e-2 and s1["divmax"] * prob.h <= 1e-8 * s1["umax"]
    u = [x.cpu().numpy() for x in st["u"]]
    assert np.all(u[0][:, :, 0] == 0) and np.all(u[1][:, 0, :] == 0) and np.all(u[2][0] == 0)
    for a in (0, 1):
        assert np.abs(u[a][::-1] - u[a]).max() <= 1e-9 * s1["umax"]
    mirrored = np.zeros_like(u[2])
    mirrored[1:] = -u[2][1:][::-1]
    assert np.abs(mirrored - u[2]).max() <= 1e-9 * s1["umax"]
