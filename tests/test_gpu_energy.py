"""Energy-law step monitor (chns_step_monitor) against the oracle's
(oracle/energy.py) on the same seeded inputs: every term, the step
condition and the energies before and after the step."""
import numpy as np
import pytest

import workloads as W
from oracle import MACGrid, Params
from oracle import energy as E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cases():
    drop = W.static_drop(32, steps=3)
    drop.init_args = dict(drop.init_args, velocity="stream", vseed=3, vamp=0.05)
    bub = W.rising_bubble(32, steps=3)
    bub.init_args = dict(bub.init_args, velocity="stream", vseed=5, vamp=0.1)
    d3 = W.drop3d(16, steps=3)
    d3.init_args = dict(d3.init_args, vamp=0.05)
    return {"drop2d": drop, "bubble_walls": bub, "drop3d": d3}


@pytest.mark.parametrize("case", ["drop2d", "bubble_walls", "drop3d"])
def test_energy_monitor_matches_oracle(case):
    import paper_2009_06628_amd as P
    prob = _cases()[case]
    print("energy monitor", case, prob.n, flush=True)
    g = P.grid_for_problem(prob)
    st = g.new_state(W.initial_state(prob))
    og = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(prob.props)
    so = W.initial_state(prob)
    for k in range(3):
        mg = g.step_monitor(st)
        so, mo = E.step_monitor(og, so, prm)
        print(k, {key: (mg[key], mo[key]) for key in ("visc", "chem", "cubic", "inert", "dt_max")}, flush=True)
        for key in ("visc", "chem"):
            assert abs(mg[key] - mo[key]) <= 1e-10 * abs(mo[key]), key
        for key in ("cubic", "inert"):
            assert abs(mg[key] - mo[key]) <= 1e-6 * abs(mo[key]) + 1e-30, key
        assert abs(mg["dt_max"] - mo["dt_max"]) <= 1e-6 * mo["dt_max"]
        assert mg["holds"] == mo["holds"]
        for key in ("energy_before", "energy_after"):
            assert abs(mg[key] - mo[key]) <= 1e-11 * abs(mo[key]), key
    # the monitored steps are the plain steps: state parity with the oracle
    err = np.abs(st["phi"].cpu().numpy() - so["phi"]).max()
    assert err <= 1e-12
