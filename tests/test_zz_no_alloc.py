"""The pressure solve that allocates nothing (chns_solve_pressure_noalloc)
against the handle-based chns_solve_pressure: same operator, kernels and
results, on two calls in a row (the second on a smaller grid, so it runs on
what the first left in the shared device array)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(n, bc, seed, ratio):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    # smooth density field with the given ratio (a tanh drop) and a random rhs
    X = np.meshgrid(*[(np.arange(m) + 0.5) / m for m in reversed(n)], indexing="ij")
    r2 = sum((x - 0.5) ** 2 for x in X)
    phi = np.tanh((np.sqrt(r2) - 0.25) / 0.03)
    rho = 0.5 * (1 + 1 / ratio) + 0.5 * (1 - 1 / ratio) * phi
    rhs = rng.standard_normal(shape)
    return rho, rhs


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_pressure_matches_handle_solve(precision):
    import paper_2009_06628_amd as P
    lib = P.load_library()
    assert lib.chns_solve_pressure_noalloc_capacity() == 32 << 20
    dev = torch.device("cuda:0")
    cases = [((128, 256), ("periodic", "wall"), 11, 1000.0),
             ((32, 32, 32), ("periodic", "periodic", "wall"), 12, 100.0),
             ((64, 48), ("wall", "wall"), 13, 10.0)]
    for (n, bc, seed, ratio) in cases:   # largest first: later calls reuse the array
        print(f"noalloc case n={n} bc={bc} precision={precision}", flush=True)
        h = 1.0 / n[0]
        rho, rhs = _case(n, bc, seed, ratio)
        t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
        rho_t, rhs_t = t(rho), t(rhs)
        g = P.create_grid(n, h, bc, precision)
        p_ref = torch.zeros_like(rho_t)
        r_ref = g.solve_pressure(rho_t, rhs_t, p_ref, rtol=1e-12, max_iter=300)
        p_new = torch.zeros_like(rho_t)
        r_new = P.solve_pressure_noalloc(n, h, bc, rho_t, rhs_t, p_new, rtol=1e-12, max_iter=300,
                                         precision=precision)
        torch.cuda.synchronize()
        assert r_ref["rc"] == 0 and r_new["rc"] == 0
        assert r_new["iters"] == r_ref["iters"]
        a, b = p_new.cpu().numpy(), p_ref.cpu().numpy()
        err = np.abs(a - b).max() / np.abs(b).max()
        print(f"  iters {r_new['iters']} rel diff {err:.3e}", flush=True)
        assert err <= 1e-12
        # rhs is not modified
        assert np.array_equal(rhs_t.cpu().numpy(), rhs)
        del g


def test_noalloc_rejects_oversized_grid():
    import paper_2009_06628_amd as P
    dev = torch.device("cuda:0")
    n = (1024, 1024)
    z = torch.zeros((1024, 1024), dtype=torch.float64, device=dev)
    with pytest.raises(P.CHNSError) as ei:
        P.solve_pressure_noalloc(n, 1 / 1024, ("periodic", "periodic"), z + 1, z, z.clone())
    assert ei.value.code == P.CHNS_EINVAL
