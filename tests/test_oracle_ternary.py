"""Pins of the three-phase oracle step (Algorithm T, oracle/ternary.py).

The paper is two-phase, so the three-phase step is pinned by what fixes it
independently of its own code: the reduction to the paper's binary step when
one phase is absent, invariance under relabelling the phases (the third phase
is implied by sum c = 1, so relabelling exercises a different code path for
each phase), the flat-interface energy of every pair, conservation of every
phase's mass, the consistent-flux continuity identity, well-balance of flat
layers under gravity and energy decay without flow.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import MACGrid, Params, step as bstep
from oracle import ternary as T


def _setup(prob):
    g = MACGrid(prob.n, prob.h, prob.periodic)
    return g, T.Params3.from_props(prob.props), W.initial_state(prob)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_spreading_and_weights():
    s = (0.7, 1.1, 0.9)
    S = T.spreading(s)
    # Sigma_i + Sigma_j = 2 sigma_ij for every pair
    assert math.isclose(S[0] + S[1], 2 * s[0]) and math.isclose(S[0] + S[2], 2 * s[1])
    assert math.isclose(S[1] + S[2], 2 * s[2])
    w = T.weights(s)
    assert math.isclose(sum(w), 1.0, rel_tol=1e-15)
    # w_i Sigma_i is the same for every phase (Sigma_T / 3)
    assert max(w[i] * S[i] for i in range(3)) - min(w[i] * S[i] for i in range(3)) < 1e-15
    with pytest.raises(ValueError):
        T.weights((0.5, 0.5, 1.5))


@pytest.mark.parametrize("bc", [(W.PERIODIC, W.PERIODIC), (W.PERIODIC, W.WALL)])
def test_third_phase_absent_reduces_to_binary_step(bc):
    """c_3 = 0 (phi_2 = -phi_1): the three-phase step is the paper's binary
    step for phi = phi_1 with rho_- = rho_2, eta_- = eta_2 (rho_1 = eta_1 = 1)
    and 1/We = sigma_12; phase 3 stays absent."""
    n = (32, 32)
    prob = W.ternary_problem(n, "ternary_pair", {"inside": 1, "outside": 0, "centre": (0.5, 0.45), "radius": 0.22,
                                                 "velocity": "stream", "vseed": 4, "vamp": 0.2},
                             bc=bc, rho3=(1.0, 0.1, 7.0), eta3=(1.0, 0.2, 3.0), sigma3=(1.0 / 1.3, 0.9, 1.1),
                             We=1.3, inv_Fr=1.0 if bc[1] == W.WALL else 0.0)
    g, prm3, st3 = _setup(prob)
    prm2 = Params(0.1, 0.2, prob.props.Re, 1.3, prob.props.Cn, prob.props.Pe, prob.props.inv_Fr, prob.props.dt)
    st2 = {"phi": st3["phi"][0].copy(), "u": [x.copy() for x in st3["u"]], "p": st3["p"].copy()}
    assert np.array_equal(st3["phi"][1], -st3["phi"][0])
    for _ in range(5):
        st3 = T.step3(g, st3, prm3)
        st2 = bstep(g, st2, prm2)
    assert _rel(st3["phi"][0], st2["phi"]) <= 1e-12
    assert np.abs(T.third(*st3["phi"]) + 1.0).max() <= 1e-14
    for a in range(2):
        assert _rel(st3["u"][a], st2["u"][a]) <= 1e-11
    assert _rel(st3["p"], st2["p"]) <= 1e-11
    assert _rel(st3["mu"][0], st2["mu"]) <= 1e-12


def _relabel(prob, perm):
    """The same physical problem with phases relabelled: new phase k is old
    phase perm[k]."""
    pr = prob.props
    s = {(0, 1): pr.sigma3[0], (0, 2): pr.sigma3[1], (1, 2): pr.sigma3[2]}
    sig = lambda i, j: s[(min(i, j), max(i, j))]
    return pr.copy(rho3=tuple(pr.rho3[perm[k]] for k in range(3)), eta3=tuple(pr.eta3[perm[k]] for k in range(3)),
                   sigma3=(sig(perm[0], perm[1]), sig(perm[0], perm[2]), sig(perm[1], perm[2])))


@pytest.mark.parametrize("perm", [(2, 1, 0), (1, 2, 0)])
def test_relabelling_the_phases_gives_the_same_flow(perm):
    """Drops of phases 1 and 2 in phase 3 with flow, walls and gravity, run
    with the phases relabelled (the stored pair then includes the former
    implied phase): every phase field, u and p agree (to the divergence
    residual of the projection, ~1e-13)."""
    prob = W.ternary_problem((32, 32), "ternary_drops",
                             {"seed": 9, "count": 2, "rmin": 0.1, "rmax": 0.14, "gap": 0.1,
                              "velocity": "stream", "vseed": 6, "vamp": 0.3},
                             bc=(W.PERIODIC, W.WALL), inv_Fr=0.5)
    g, prm, st = _setup(prob)
    phis = [st["phi"][0], st["phi"][1], T.third(*st["phi"])]
    prm_r = T.Params3.from_props(_relabel(prob, perm))
    st_r = {"phi": [phis[perm[0]].copy(), phis[perm[1]].copy()], "u": [x.copy() for x in st["u"]],
            "p": st["p"].copy()}
    for _ in range(5):
        st = T.step3(g, st, prm)
        st_r = T.step3(g, st_r, prm_r)
    phis = [st["phi"][0], st["phi"][1], T.third(*st["phi"])]
    phis_r = [st_r["phi"][0], st_r["phi"][1], T.third(*st_r["phi"])]
    for k in range(3):
        assert np.abs(phis_r[k] - phis[perm[k]]).max() <= 1e-11
    for a in range(2):
        assert _rel(st_r["u"][a], st["u"][a]) <= 1e-10
    assert _rel(st_r["p"], st["p"]) <= 1e-10


@pytest.mark.parametrize("pair", [(0, 1), (0, 2), (1, 2)])
def test_flat_pair_interface_energy_is_its_surface_tension(pair):
    """A flat i|j interface (equilibrium profile, third phase absent) has free
    energy per unit length (2 sqrt2 / 3) sigma_ij -- the binary step's
    effective surface tension with 1/We = sigma_ij -- within 1 %."""
    g = MACGrid((4, 64), 1.0 / 64, (True, False))
    prm = T.Params3((1.0, 1.0, 1.0), (1.0, 1.0, 1.0), (0.7, 1.1, 0.9), 10.0, 1.0, 4.0 / 64, 1000.0, 0.0, 1e-4)
    y = g.coords()[1]
    Ly = 1.0
    phi_i = -np.tanh((y - 0.5 * Ly) / (math.sqrt(2) * prm.Cn))
    phis = [None, None, None]
    i, j = pair
    k = 3 - i - j
    phis[i], phis[j], phis[k] = phi_i, -phi_i, np.full(g.shape, -1.0)
    if k != 2:   # store phases 1, 2 (phase 3 is implied)
        assert np.abs(T.third(phis[0], phis[1]) - phis[2]).max() < 1e-15
    d = T.diagnostics3(g, {"phi": [phis[0], phis[1]], "u": [np.zeros(g.shape)] * 2, "p": np.zeros(g.shape)}, prm)
    Lx = 4.0 / 64
    sig = {(0, 1): prm.sigma[0], (0, 2): prm.sigma[1], (1, 2): prm.sigma[2]}[pair]
    assert abs(d["free"] / Lx / ((2 * math.sqrt(2) / 3) * sig) - 1.0) < 0.01


def test_every_phase_mass_is_conserved():
    """Proposition mass_conservation for each phase: drops of phases 1 and 2
    in phase 3 between walls with gravity and flow, 20 steps: the three
    masses stay to 1e-12, the wall normal velocity 0, and the implied phase 3
    follows its own flux-form update up to dt |D u^n|."""
    prob = W.ternary_problem((32, 32), "ternary_drops",
                             {"seed": 5, "count": 2, "rmin": 0.1, "rmax": 0.14, "gap": 0.1,
                              "velocity": "stream", "vseed": 2, "vamp": 0.3},
                             bc=(W.PERIODIC, W.WALL), inv_Fr=1.0)
    g, prm, st = _setup(prob)
    d0 = T.diagnostics3(g, st, prm)
    kM = 1.0 / (prm.Pe * prm.Cn)
    for n in range(20):
        new = T.step3(g, st, prm)
        if n == 3:
            p3 = T.third(*st["phi"])
            mu3 = -new["mu"][0] - new["mu"][1]
            F = [st["u"][a] * g.avg(p3, a) - kM * g.grad(mu3, a) for a in range(2)]
            own = p3 - prm.dt * g.div(F)
            bound = prm.dt * np.abs(g.div(st["u"])).max() + 1e-14
            assert np.abs(T.third(*new["phi"]) - own).max() <= 2 * bound
        st = new
    d1 = T.diagnostics3(g, st, prm)
    for k in ("mass1", "mass2", "mass3"):
        assert abs(d1[k] - d0[k]) <= 1e-12 * d0[k]
    assert d1["umax"] > 1e-3
    for a in range(2):
        assert np.all(st["u"][a][g.wall_face_mask(a)] == 0.0)


def test_continuity_consistency():
    """rho_lin(phi^{n+1}) - rho_lin(phi^n) + dt D m - dt K D u^n = 0 with
    K = rho_3 + sum_{i=1,2} (rho_i - rho_3)/2: the three-phase mass flux
    m = rho_lin u + J, J = -(kM/2) sum_i rho_i G mu~_i, satisfies the
    continuity equation given the flux-form phase updates."""
    prob = W.ternary_problem((32, 32), "ternary_drops",
                             {"seed": 5, "count": 2, "rmin": 0.1, "rmax": 0.14, "gap": 0.1,
                              "velocity": "stream", "vseed": 3, "vamp": 0.3},
                             bc=(W.PERIODIC, W.WALL), rho3=(3.0, 0.2, 1.0))
    g, prm, st0 = _setup(prob)
    st1 = T.step3(g, st0, prm)
    lin = lambda s: T.mixture(prm, [s["phi"][0], s["phi"][1], T.third(*s["phi"])], "rho", pull=False)
    K = prm.rho[2] + 0.5 * ((prm.rho[0] - prm.rho[2]) + (prm.rho[1] - prm.rho[2]))
    res = lin(st1) - lin(st0) + prm.dt * g.div(st1["m"]) - prm.dt * K * g.div(st0["u"])
    assert np.abs(res).max() < 1e-13


def test_flat_layers_stay_at_rest():
    """Well-balance: three flat layers (phase 1 at the bottom, then 2, then 3)
    between no-slip walls under gravity: every force depends on y only and
    is a discrete gradient, so u stays 0 over 50 steps."""
    prob = W.ternary_problem((16, 32), "ternary_layers", {"y1": 0.6, "y2": 1.3}, bc=(W.PERIODIC, W.WALL),
                             inv_Fr=1.0, rho3=(2.0, 1.0, 0.3))
    g, prm, st = _setup(prob)
    for _ in range(50):
        st = T.step3(g, st, prm)
    assert max(np.abs(x).max() for x in st["u"]) <= 1e-12
    assert np.abs(st["p"]).max() > 1e-3


def test_energy_decays_without_flow():
    """Three-phase spinodal mixture with u = 0 (the CH part of Algorithm T):
    the free energy does not increase over 400 steps and falls overall."""
    prob = W.ternary_problem((32, 32), "ternary_mix", {"seed": 12, "amp": 0.1}, Pe=100.0, dt=2e-4)
    g, prm, st = _setup(prob)
    E = [T.diagnostics3(g, st, prm)["free"]]
    for _ in range(400):
        st = T.step3(g, st, prm, ch_only=True)
        E.append(T.diagnostics3(g, st, prm)["free"])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-14 * np.abs(E[:-1]))
    assert E[-1] < 0.9 * E[0]
