"""GPU (HIP, gfx950) path vs the FP64 CPU oracle, element by element.

Bar: relative max-norm  max|gpu - oracle| / max|oracle|  <= 1e-9 after 100
steps (the stated target), tighter for single operators and single steps.
Pressure is compared with its mean removed (gauge).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import MACGrid, Params, step as ostep, diagnostics
from oracle import chns as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    import paper_2009_06628_amd as P
    return P


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()


def run_gpu(prob, steps, init=None):
    P = _lib()
    g = P.grid_for_problem(prob)
    st = g.new_state(init if init is not None else W.initial_state(prob))
    stats = g.step(st, steps) if steps > 0 else None
    torch.cuda.synchronize()
    return g, st, stats


def run_oracle(prob, steps, init=None):
    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(prob.props)
    st = init if init is not None else W.initial_state(prob)
    for _ in range(steps):
        st = ostep(g, st, prm)
    return g, st, prm


def compare_states(sg, so, dim, tol, tol_u=None, tol_p=None):
    errs = {"phi": relerr(to_np(sg["phi"]), so["phi"])}
    for a in range(dim):
        errs["u%d" % a] = relerr(to_np(sg["u"][a]), so["u"][a]) if np.abs(so["u"][a]).max() > 0 else \
            float(np.abs(to_np(sg["u"][a])).max())
    pg = to_np(sg["p"])
    errs["p"] = relerr(pg - pg.mean(), so["p"] - so["p"].mean())
    if "mu" in so:
        errs["mu"] = relerr(to_np(sg["mu"]), so["mu"])
    print("parity", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        lim = tol
        if k == "p" and tol_p is not None:
            lim = tol_p
        if k.startswith("u") and tol_u is not None:
            lim = tol_u
        assert v <= lim, (k, v, lim)
    return errs


# ---------------------------------------------------------------------------
# single operators
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,per", [((40, 24), (True, False)), ((64, 64), (True, True)), ((18, 10), (False, False)),
                                   ((16, 8, 12), (True, False, True))])
def test_pressure_operator_matches_oracle(n, per):
    P = _lib()
    rng = np.random.default_rng(7)
    og = MACGrid(n, 1.0 / n[0], per)
    rho = rng.uniform(1e-3, 1.0, size=og.shape)
    x = rng.normal(size=og.shape)
    ref = (O.pressure_matrix(og, [og.avg(rho, a) for a in range(og.dim)]) @ x.ravel()).reshape(og.shape)
    bc = ["periodic" if p else "wall" for p in per]
    g = P.create_grid(n, 1.0 / n[0], bc)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    y = dev(np.zeros(og.shape))
    g.apply_pressure_operator(dev(rho), dev(x), y)
    assert relerr(to_np(y), ref) <= 1e-14


@pytest.mark.parametrize("n,per", [((64, 128), (True, False)), ((96, 96), (True, True)), ((80, 48), (False, False)),
                                   ((96, 40), (False, True)), ((32, 16, 24), (True, True, False)),
                                   ((40, 20, 12), (False, False, True))])
def test_solve_pressure_matches_oracle(n, per):
    P = _lib()
    rng = np.random.default_rng(11)
    og = MACGrid(n, 1.0 / n[0], per)
    # smooth density field with contrast 1000 (a bubble), random rhs
    X = og.coords()
    r2 = sum((X[a] - 0.5 * og.n[a] * og.h) ** 2 for a in range(og.dim))
    phi = np.tanh((np.sqrt(r2) - 0.25) / (math.sqrt(2) * 3 * og.h))
    rho = 0.5 * (1 - 1e-3) * phi + 0.5 * (1 + 1e-3)
    rhs = rng.normal(size=og.shape)
    rhs -= rhs.mean()
    ref = O.pressure_solve(og, [og.avg(rho, a) for a in range(og.dim)], rhs)
    bc = ["periodic" if p else "wall" for p in per]
    g = P.create_grid(n, 1.0 / n[0], bc)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    p = dev(np.zeros(og.shape))
    out = g.solve_pressure(dev(rho), dev(rhs), p, rtol=1e-13, max_iter=300)
    print("pressure solve", n, out, flush=True)
    assert out["rc"] == 0
    assert relerr(to_np(p), ref) <= 1e-9


@pytest.mark.parametrize("n,per", [((32, 16, 24), (True, True, False)), ((40, 20, 36), (False, False, True)),
                                   ((36, 20, 40), (True, False, True))])
def test_march_sweeps_match_grid_stride_and_oracle(n, per):
    """3D smoothing and residual sweeps marching along z (used by default on
    levels of 2^24 cells and more), forced onto every level with
    CHNS_OPT_MARCH_SWEEP_CELLS = 1 on grids with ragged x / y tiles and
    several z chunks (which also makes the CG apply form the pressure
    coefficients from the density): the pressure solve is bit for bit that of
    the grid-stride sweeps and stored coefficients (same per-cell arithmetic)
    and matches the oracle."""
    P = _lib()
    rng = np.random.default_rng(12)
    og = MACGrid(n, 1.0 / n[0], per)
    X = og.coords()
    r2 = sum((X[a] - 0.5 * og.n[a] * og.h) ** 2 for a in range(og.dim))
    phi = np.tanh((np.sqrt(r2) - 0.25) / (math.sqrt(2) * 3 * og.h))
    rho = 0.5 * (1 - 1e-2) * phi + 0.5 * (1 + 1e-2)
    rhs = rng.normal(size=og.shape)
    rhs -= rhs.mean()
    ref = O.pressure_solve(og, [og.avg(rho, a) for a in range(og.dim)], rhs)
    bc = ["periodic" if p else "wall" for p in per]
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    sols = []
    for cells in (1 << 24, 1):
        g = P.create_grid(n, 1.0 / n[0], bc)
        g.set_option(P.CHNS_OPT_MARCH_SWEEP_CELLS, cells)
        p = dev(np.zeros(og.shape))
        out = g.solve_pressure(dev(rho), dev(rhs), p, rtol=1e-13, max_iter=300)
        print("pressure solve", n, "march cells", cells, out, flush=True)
        assert out["rc"] == 0
        sols.append(p)
    assert torch.equal(sols[0], sols[1])
    assert relerr(to_np(sols[1]), ref) <= 1e-9


def test_march_sweeps_whole_step_bitwise():
    """Ten steps of the 3D drop with every level's sweeps marching along z
    equal the grid-stride run bit for bit (momentum, pressure and, through
    MG-PCG, the CH solve)."""
    P = _lib()
    prob = W.drop3d(32, steps=10)
    out = []
    for cells in (1 << 24, 1):
        g = P.grid_for_problem(prob)
        g.set_option(P.CHNS_OPT_MARCH_SWEEP_CELLS, cells)
        g.set_option(P.CHNS_OPT_CH_SOLVER, P.CHNS_CH_PCG)
        st = g.new_state(W.initial_state(prob))
        g.step(st, 10)
        out.append(st)
    for k in ("phi", "p", "mu"):
        assert torch.equal(out[0][k], out[1][k]), k
    for a in range(3):
        assert torch.equal(out[0]["u"][a], out[1]["u"][a]), a


@pytest.mark.parametrize("n,per", [((36, 20, 40), (False, True, False)), ((32, 32, 32), (True, True, True)),
                                   ((48, 24, 32), (True, False, True))])
@pytest.mark.parametrize("precision", [0, 1])
def test_tile_cycle_matches_grid_stride_and_oracle(n, per, precision):
    """3D V-cycle passes over 8^3-cell tiles with recomputed halos (one
    launch per level and side), forced onto every level above the
    single-workgroup part with a large CHNS_OPT_TILE_CYCLE_CELLS, on grids
    with ragged tiles and walls: the pressure solve is bit for bit that of
    the grid-wide passes (tile cells 0) in both precision forms and matches
    the oracle."""
    P = _lib()
    rng = np.random.default_rng(13)
    og = MACGrid(n, 1.0 / n[0], per)
    X = og.coords()
    r2 = sum((X[a] - 0.5 * og.n[a] * og.h) ** 2 for a in range(og.dim))
    phi = np.tanh((np.sqrt(r2) - 0.25) / (math.sqrt(2) * 3 * og.h))
    rho = 0.5 * (1 - 1e-2) * phi + 0.5 * (1 + 1e-2)
    rhs = rng.normal(size=og.shape)
    rhs -= rhs.mean()
    ref = O.pressure_solve(og, [og.avg(rho, a) for a in range(og.dim)], rhs)
    bc = ["periodic" if p else "wall" for p in per]
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    sols = []
    for cells in (0, 1 << 30):
        g = P.create_grid(n, 1.0 / n[0], bc, precision=precision)
        g.set_option(P.CHNS_OPT_TILE_CYCLE_CELLS, cells)
        p = dev(np.zeros(og.shape))
        out = g.solve_pressure(dev(rho), dev(rhs), p, rtol=1e-12, max_iter=300)
        print("pressure solve", n, "precision", precision, "tile cells", cells, out, flush=True)
        assert out["rc"] == 0
        sols.append(p)
    assert torch.equal(sols[0], sols[1])
    assert relerr(to_np(sols[1]), ref) <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
def test_tile_cycle_whole_step_bitwise(precision):
    """Five steps of the 3D drop (CH by MG-PCG, truncated momentum cycles)
    with the tile passes on every eligible level equal the run with the
    grid-wide passes only, bit for bit."""
    P = _lib()
    prob = W.drop3d(32, steps=5)
    if precision:
        prob = W.drop3d(32, steps=5, **W.PRECISION_FORM_TOLERANCES)
    out = []
    for cells in (0, 1 << 30):
        g = P.grid_for_problem(prob, precision)
        g.set_option(P.CHNS_OPT_TILE_CYCLE_CELLS, cells)
        g.set_option(P.CHNS_OPT_CH_SOLVER, P.CHNS_CH_PCG)
        st = g.new_state(W.initial_state(prob))
        g.step(st, 5)
        out.append(st)
    for k in ("phi", "p", "mu"):
        assert torch.equal(out[0][k], out[1][k]), k
    for a in range(3):
        assert torch.equal(out[0]["u"][a], out[1]["u"][a]), a


# ---------------------------------------------------------------------------
# whole steps
# ---------------------------------------------------------------------------

def test_one_step_static_drop():
    prob = W.static_drop(64, steps=1)
    prob.init_args = dict(prob.init_args, velocity="stream", vseed=4, vamp=0.05)
    _, sg, stats = run_gpu(prob, 1)
    _, so, _ = run_oracle(prob, 1)
    print("stats", stats, flush=True)
    compare_states(sg, so, 2, 1e-11)


def test_one_step_bubble_walls():
    prob = W.rising_bubble(64, steps=1)
    prob.init_args = dict(prob.init_args, velocity="stream", vseed=6, vamp=0.1)
    _, sg, stats = run_gpu(prob, 1)
    _, so, _ = run_oracle(prob, 1)
    print("stats", stats, flush=True)
    compare_states(sg, so, 2, 1e-11)


def test_static_drop_100_steps_parity_and_invariants():
    """Static drop 64^2, density / viscosity ratio 10, sigma 1, Cn = 1.5 h,
    M = 1e-3, dt = 1e-4, 100 steps: parity 1e-9, mass to 1e-12."""
    prob = W.static_drop(64, steps=100)
    g, sg, stats = run_gpu(prob, 100)
    og, so, prm = run_oracle(prob, 100)
    compare_states(sg, so, 2, 1e-9)
    d0 = diagnostics(og, W.initial_state(prob), prm)
    assert abs(stats["mass_minus"] - d0["mass_minus"]) / d0["mass_minus"] <= 1e-12
    assert abs(stats["mass_plus"] - d0["mass_plus"]) / d0["mass_plus"] <= 1e-12
    do = diagnostics(og, so, prm)
    assert abs(stats["energy"] - do["energy"]) <= 1e-10 * abs(do["energy"])


def test_bubble_reduced_100_steps_parity():
    """Rising bubble physics (ratios 1000 / 100, Eo 10, Ar 35, walls) on a
    64 x 128 grid, 100 steps."""
    prob = W.rising_bubble(64, steps=100)
    g, sg, stats = run_gpu(prob, 100)
    og, so, prm = run_oracle(prob, 100)
    print("stats", stats, flush=True)
    compare_states(sg, so, 2, 1e-9)


def test_rising_bubble_full_size_one_step_and_invariants():
    """Full 256 x 512 rising-bubble grid: one step against the oracle, then
    20 more steps checked by invariants (mass, walls, divergence)."""
    prob = W.rising_bubble(256, steps=1)
    g, sg, stats = run_gpu(prob, 1)
    og, so, prm = run_oracle(prob, 1)
    # velocity after one step from rest at density ratio 1000: the oracle's
    # own pressure solve is only reproducible to ~2e-10 in this norm
    compare_states(sg, so, 2, 1e-10, tol_u=1e-9)
    d0 = diagnostics(og, W.initial_state(prob), prm)
    stats = g.step(sg, 20)
    assert abs(stats["mass_minus"] - d0["mass_minus"]) / d0["mass_minus"] <= 1e-12
    assert stats["divmax"] * og.h <= 1e-10 * max(stats["umax"], 1e-3)
    uy = to_np(sg["u"][1])
    assert np.all(uy[0, :] == 0.0)


def test_drop3d_parity():
    prob = W.drop3d(16, steps=5)
    _, sg, stats = run_gpu(prob, 5)
    _, so, _ = run_oracle(prob, 5)
    print("stats", stats, flush=True)
    compare_states(sg, so, 3, 1e-10)


@pytest.mark.parametrize("Re,level", [(50.0, 1), (1000.0, 0)])
def test_drop3d_truncated_momentum_cycle_parity(Re, level):
    """Momentum operator dominated by its diagonal shift rho_min / dt = 1e3
    at 32^3: against 2 d eta_max / (Re h_l^2), Re = 50 gives ratio 8.1 on the
    grid (< 10) and 32.6 on the 16^3 level (>= 30), so the 3D momentum
    V-cycles end there with a symmetric Gauss-Seidel sweep; Re = 1000 gives
    ratio 163 on the grid (>= 10), where the preconditioner is that sweep on
    the grid alone.  20 steps against the oracle."""
    prob = W.drop3d(32, steps=20, Re=Re)
    ratio = [(0.1 / prob.props.dt) / (6.0 * 1.0 / (prob.props.Re * (prob.h * 2 ** l) ** 2)) for l in range(2)]
    assert (ratio[0] >= 10.0) == (level == 0) and ratio[1] >= 30.0
    _, sg, stats = run_gpu(prob, 20)
    _, so, _ = run_oracle(prob, 20)
    print("stats", stats, flush=True)
    compare_states(sg, so, 3, 1e-10)


def test_flat_interface_stays_at_rest_gpu():
    prob = W.flat_interface(32, 32, steps=100, gravity=True)
    _, sg, stats = run_gpu(prob, 100)
    assert max(float(np.abs(to_np(x)).max()) for x in sg["u"]) <= 1e-12


def test_deterministic_bitwise():
    prob = W.rising_bubble(64, steps=10)
    _, s1, _ = run_gpu(prob, 10)
    _, s2, _ = run_gpu(prob, 10)
    for k in ("phi", "p", "mu"):
        assert torch.equal(s1[k], s2[k])
    for a in range(2):
        assert torch.equal(s1["u"][a], s2["u"][a])


@pytest.mark.parametrize("case", ["bubble2d", "drops3d", "drops3d_96"])
def test_ch_direct_solve_matches_mg_pcg(case):
    """The Cahn-Hilliard system is solved directly (axis eigenbases, FP64
    transforms) by default and by MG-PCG with the CHNS_OPT_CH_SOLVER option;
    the states must
    agree to the PCG tolerance (1e-10 per solve) after several steps, and
    the direct solve must report one application."""
    P = _lib()
    # 96^3: the axis transforms take 64-wide output tiles (matrix-core
    # kernel) with a ragged last tile along every axis
    prob = {"bubble2d": W.rising_bubble(64, steps=20), "drops3d": W.drops3d(32, steps=4),
            "drops3d_96": W.drops3d(96, steps=4)}[case]
    steps = 20 if case == "bubble2d" else 4
    init = W.initial_state(prob)
    out = []
    for solver in ("direct", "pcg"):
        print("CH solver", case, solver, flush=True)
        g = P.grid_for_problem(prob)
        g.set_option(P.CHNS_OPT_CH_SOLVER, P.CHNS_CH_PCG if solver == "pcg" else P.CHNS_CH_DIRECT)
        st = g.new_state(init)
        stats = g.step(st, steps)
        out.append((st, stats))
    (a, sa), (b, sb) = out
    assert sa["iters_ch"] == 1 and sb["iters_ch"] > 1
    assert relerr(to_np(a["phi"]), to_np(b["phi"])) < 1e-8
    for d in range(len(a["u"])):
        assert relerr(to_np(a["u"][d]), to_np(b["u"][d])) < 1e-8, d
    pa, pb = to_np(a["p"]), to_np(b["p"])
    assert relerr(pa - pa.mean(), pb - pb.mean()) < 1e-8


def _fft_case(case):
    drops = {"seed": 5, "count": 2, "rmin": 0.04, "rmax": 0.06, "gap": 0.05, "velocity": "stream",
             "vseed": 9, "vamp": 0.05}
    return {"drops3d_32": lambda: W.drops3d(32, steps=4),
            "ternary_64x32x16": lambda: W.ternary_problem((64, 32, 16), "ternary_drops",
                                                          dict(drops, velocity="potential3d"), steps=4),
            "ternary_32x32x24": lambda: W.ternary_problem((32, 32, 24), "ternary_drops",
                                                          dict(drops, velocity="potential3d"), steps=4),
            "ternary2d_32x16": lambda: W.ternary_problem((32, 16), "ternary_drops", drops, steps=4),
            "bubble2d_64": lambda: W.rising_bubble(64, steps=4),
            "spinodal2d_128": lambda: W.spinodal(128, steps=4)}[case]()


@pytest.mark.parametrize("case", ["drops3d_32", "ternary_64x32x16", "ternary_32x32x24", "ternary2d_32x16",
                                  "bubble2d_64", "spinodal2d_128"])
def test_ch_fft_matches_dense_basis(case):
    """The direct CH solve transforms periodic power-of-two axes by radix-2
    FFT (the last axis with the division fused in, when it is one of them)
    and every other axis by the product with the dense basis; forcing the
    dense product on every axis (CHNS_CH_DIRECT_DENSE) must give the same
    states to rounding after four steps.  Cases: every axis FFT (32^3; 64 x
    32 x 16 with 16 on the fused axis; 2D 128^2), a non-power-of-two last
    axis (32 x 32 x 24: FFT on x, y, dense z and the separate division), a
    walled axis (bubble: FFT x, dense y), and workgroups with fewer pencils
    than they pair (2D 32 x 16: 16 of 128 and 32 of 256)."""
    P = _lib()
    prob = _fft_case(case)
    init = W.initial_state(prob)
    out = []
    for solver in (P.CHNS_CH_DIRECT, P.CHNS_CH_DIRECT_DENSE):
        g = P.grid_for_problem(prob)
        g.set_option(P.CHNS_OPT_CH_SOLVER, solver)
        st = g.new_state(init)
        stats = g.step(st, 4)
        print("CH transform", case, solver, stats["iters_ch"], flush=True)
        out.append(st)
    a, b = out
    phis = a["phi"] if isinstance(a["phi"], (list, tuple)) else [a["phi"]]
    phib = b["phi"] if isinstance(b["phi"], (list, tuple)) else [b["phi"]]
    for x, y in zip(phis, phib):
        assert relerr(to_np(x), to_np(y)) < 1e-11
    for d in range(len(a["u"])):
        assert relerr(to_np(a["u"][d]), to_np(b["u"][d])) < 1e-10, d
    pa, pb = to_np(a["p"]), to_np(b["p"])
    assert relerr(pa - pa.mean(), pb - pb.mean()) < 1e-10


@pytest.mark.parametrize("case", ["bubble2d", "drops3d"])
def test_time_guess_meets_the_tolerances(case):
    """CHNS_OPT_TIME_GUESS (default on) starts the momentum and pressure
    solves from their last solutions extrapolated in time: after 10 steps
    the state agrees with the plain guesses (u^n, p^n) to the solver
    tolerances, with no more CG iterations in the last step."""
    P = _lib()
    prob = W.rising_bubble(64, steps=10) if case == "bubble2d" else W.drop3d(32, steps=10)
    init = W.initial_state(prob)
    out = []
    for guess in (1, 0):
        g = P.grid_for_problem(prob)
        g.set_option(P.CHNS_OPT_TIME_GUESS, guess)
        st = g.new_state(init)
        g.step(st, 9)
        stats = g.step(st, 1)
        print("time guess", case, guess, stats["iters_p"], stats["iters_mom"], flush=True)
        out.append((st, stats))
    (a, sa), (b, sb) = out
    assert sa["iters_p"] <= sb["iters_p"] and sum(sa["iters_mom"]) <= sum(sb["iters_mom"])
    assert relerr(to_np(a["phi"]), to_np(b["phi"])) < 1e-9
    for d in range(len(a["u"])):
        assert relerr(to_np(a["u"][d]), to_np(b["u"][d])) < 1e-8, d
    pa, pb = to_np(a["p"]), to_np(b["p"])
    assert relerr(pa - pa.mean(), pb - pb.mean()) < 1e-8


def test_time_guess_restarts_on_another_state():
    """A handle that stepped one state and is then given another (whose
    pressure is not the handle's last solution) restarts its guess history
    there: the new state's steps are bit for bit those of a fresh handle."""
    P = _lib()
    pa, pb = W.drop3d(32, steps=3), W.drop3d(32, steps=2, Re=20.0)
    g = P.grid_for_problem(pa)
    sa = g.new_state(W.initial_state(pa))
    g.step(sa, 3)
    g.set_properties(pb.props)
    sb = g.new_state(W.initial_state(pb))
    g.step(sb, 2)
    f = P.grid_for_problem(pb)
    sf = f.new_state(W.initial_state(pb))
    f.step(sf, 2)
    for k in ("phi", "p", "mu"):
        assert torch.equal(sb[k], sf[k]), k
    for d in range(3):
        assert torch.equal(sb["u"][d], sf["u"][d]), d


@pytest.mark.parametrize("case", ["bubble2d", "drops3d"])
def test_concurrent_momentum_matches_serial_bitwise(case):
    """The momentum components run on their own streams and host threads; with
    the per-kernel timing on, or with CHNS_OPT_SERIAL_COMPONENTS, they run one
    after another on the handle's stream.  All orders must give the same
    state bit for bit."""
    P = _lib()
    prob = W.rising_bubble(64, steps=6) if case == "bubble2d" else W.drops3d(32, steps=3)
    steps = 6 if case == "bubble2d" else 3
    init = W.initial_state(prob)
    out = []
    for mode in ("timing", "serial", "concurrent"):
        g = P.grid_for_problem(prob)
        st = g.new_state(init)
        g.set_timing(mode == "timing")
        g.set_option(P.CHNS_OPT_SERIAL_COMPONENTS, 1 if mode == "serial" else 0)
        g.step(st, steps)
        torch.cuda.synchronize()
        g.set_timing(False)
        out.append(st)
    a = out[-1]
    for b in out[:-1]:
        for k in ("phi", "p", "mu"):
            assert torch.equal(a[k], b[k]), k
        for d in range(len(a["u"])):
            assert torch.equal(a["u"][d], b["u"][d]), d


def test_error_paths():
    P = _lib()
    prob = W.static_drop(32, steps=1)
    g = P.grid_for_problem(prob)
    st = g.new_state(W.initial_state(prob))
    # max_iter = 1: the step completes with the ENOCONV warning
    g.set_properties(prob.props.copy(max_iter=1))
    out = g.step(st, 1, allow_noconv=True)
    assert out["rc"] == P.CHNS_ENOCONV and out["unconverged"] != 0
    # a NaN in phi is reported, not propagated silently
    g.set_properties(prob.props)
    st = g.new_state(W.initial_state(prob))
    st["phi"][3, 5] = float("nan")
    with pytest.raises(P.CHNSError) as ei:
        g.step(st, 1)
    assert ei.value.code == P.CHNS_ENONFINITE


def test_ragged_and_small_grids():
    """Sizes that are not multiples of the 256-thread blocks, grids that are
    their own coarsest level, and a 3D walled box."""
    for prob in [W.static_drop(24, steps=3), W.spinodal(20, steps=3), W.rising_bubble(48, steps=3)]:
        _, sg, _ = run_gpu(prob, 3)
        _, so, _ = run_oracle(prob, 3)
        compare_states(sg, so, 2, 1e-10, tol_u=1e-9)


# ---------------------------------------------------------------------------
# full-size code paths
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["walls768", "drop3d_112"])
def test_one_step_past_the_kernel_grid_caps(case):
    """Sizes where the launch shapes change: more than 262,144 cells (kernels
    writing per-block partials loop over several cells per thread), more
    than 1,048,576 cells in 3D (every grid-stride sweep does), and more than
    1024 level-0 tiles in 2D (the CG update leaves the level-0 tile passes).
    One step against the oracle."""
    if case == "walls768":
        n = 768
        prob = W.Problem("walls768", (n, n), 1.0 / n, (W.WALL, W.WALL), W.static_drop(n).props, 1, "drop",
                         {"centre": (0.5, 0.45), "radius": 0.25, "velocity": "stream", "vseed": 3, "vamp": 0.05})
        assert (n // 32) * (n // 16) > 1024 and n * n > 262144
    else:
        prob = W.drop3d(112, steps=1)
        assert prob.cells > 1048576
    print("full-size one step", case, prob.n, flush=True)
    _, sg, stats = run_gpu(prob, 1)
    _, so, _ = run_oracle(prob, 1)
    print("stats", stats, flush=True)
    compare_states(sg, so, prob.dim, 1e-10)


def test_rising_bubble_full_size_100_steps_parity():
    """The full 256 x 512 rising-bubble configuration (density ratio 1000,
    viscosity ratio 100, walls, gravity) from its initial state: 100 steps
    against the oracle at the 1e-9 bar, phase masses to 1e-12."""
    prob = W.rising_bubble(256, steps=100)
    print("bubble 256x512, 100 steps", flush=True)
    g, sg, stats = run_gpu(prob, 100)
    og, so, prm = run_oracle(prob, 100)
    compare_states(sg, so, 2, 1e-9)
    d0 = diagnostics(og, W.initial_state(prob), prm)
    for key in ("mass_plus", "mass_minus"):
        assert abs(stats[key] - d0[key]) <= 1e-12 * d0[key]
