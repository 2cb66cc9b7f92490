"""Pins of the energy-law step monitor (oracle/energy.py): each term against
a closed form, the vanishing of every term for a state at rest, and the
monitor on the static drop."""
import math

import numpy as np

import workloads as W
from oracle import MACGrid, Params
from oracle import energy as E


def _tg(g, A=1.0):
    h = g.h
    i, j = g.index(0), g.index(1)
    ux = A * np.sin(2 * np.pi * i * h) * np.cos(2 * np.pi * (j + 0.5) * h)
    uy = -A * np.cos(2 * np.pi * (i + 0.5) * h) * np.sin(2 * np.pi * j * h)
    return [ux, uy]


def test_viscous_dissipation_of_eigenmodes():
    """K u = -(1/Re) L u for constant eta: a Taylor-Green mode (periodic) and
    a wall shear profile sin(pi (j + 1/2)/n) (no-slip ghost rule) are
    eigenvectors, so u^T K u h^d = -(eta lam / Re) |u|^2 h^d."""
    n, Re, eta = 16, 7.0, 2.5
    g = MACGrid((n, n), 1.0 / n, (True, True))
    u = _tg(g)
    lam = 2 * (2 * np.cos(2 * np.pi * g.h) - 2) / g.h ** 2
    ref = -eta * lam / Re * float(np.sum(u[0] ** 2 + u[1] ** 2)) * g.h ** 2
    got = E.viscous_dissipation(g, u, np.full(g.shape, eta), Re)
    assert math.isclose(got, ref, rel_tol=1e-12)
    gw = MACGrid((8, n), 1.0 / n, (True, False))
    j = gw.index(1)
    ux = np.sin(np.pi * (j + 0.5) / n)
    lam_w = (2 * np.cos(np.pi / n) - 2) / gw.h ** 2
    ref = -eta * lam_w / Re * float(np.sum(ux ** 2)) * gw.h ** 2
    got = E.viscous_dissipation(gw, [ux, np.zeros(gw.shape)], np.full(gw.shape, eta), Re)
    assert math.isclose(got, ref, rel_tol=1e-12)


def test_chemical_dissipation_closed_form():
    """mu = cos(2 pi x) on a periodic n x n grid: sum (G mu)^2 h^2 =
    (4 sin^2(pi h) / h^2) (n^2 / 2) h^2."""
    n = 32
    g = MACGrid((n, n), 1.0 / n, (True, True))
    prm = Params(0.1, 0.1, 10.0, 2.0, 0.05, 300.0, 0.0, 1e-4)
    mu = np.cos(2 * np.pi * g.coords()[0])
    ref = 4 * np.sin(np.pi * g.h) ** 2 / g.h ** 2 * (n * n / 2) * g.h ** 2 / (prm.Pe * prm.Cn ** 2 * prm.We)
    assert math.isclose(E.chemical_dissipation(g, mu, prm), ref, rel_tol=1e-12)


def test_cubic_and_inertia_bounds_closed_form():
    g = MACGrid((8, 8), 1.0 / 8, (True, False))
    prm = Params(0.1, 0.1, 10.0, 2.0, 0.05, 300.0, 0.0, 1e-4)
    phi0, phi1 = np.full(g.shape, 0.2), np.full(g.shape, -0.3)
    ref = 6 * 0.3 * 0.5 ** 3 / (24 * prm.We * prm.Cn)
    assert math.isclose(E.cubic_bound(g, phi0, phi1, prm), ref, rel_tol=1e-12)
    U = 0.7
    u0 = [np.zeros(g.shape), np.zeros(g.shape)]
    u1 = [np.full(g.shape, U), np.zeros(g.shape)]
    assert math.isclose(E.inertia_bound(g, np.full(g.shape, 1.0), np.full(g.shape, 1.5), u0, u1),
                        0.5 * U * U / 8, rel_tol=1e-12)


def test_monitor_at_rest_is_zero():
    g = MACGrid((16, 16), 1.0 / 16, (True, False))
    prm = Params(0.1, 0.1, 10.0, 1.0, 0.1, 100.0, 0.0, 1e-3)
    st = {"phi": np.full(g.shape, 0.4), "u": [np.zeros(g.shape)] * 2, "p": np.zeros(g.shape)}
    _, m = E.step_monitor(g, st, prm)
    assert m["visc"] == 0.0 and m["cubic"] < 1e-40 and m["inert"] == 0.0
    assert m["chem"] < 1e-25
    assert m["holds"]


def test_monitor_on_the_static_drop():
    """Static drop with a small seeded flow: the dissipation dominates the
    two bounds by a wide margin at dt = 1e-4 (dt_max >> dt), and the
    discrete energy falls."""
    prob = W.static_drop(32, steps=1)
    prob.init_args = dict(prob.init_args, velocity="stream", vseed=3, vamp=0.05)
    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(prob.props)
    st = W.initial_state(prob)
    for _ in range(3):
        st, m = E.step_monitor(g, st, prm)
        assert m["holds"] and m["dt_max"] > 10 * prm.dt
        assert m["visc"] > 0 and m["chem"] > 0 and m["cubic"] > 0 and m["inert"] > 0
        assert m["energy_after"] < m["energy_before"]
