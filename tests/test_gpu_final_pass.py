"""Labels and byproduct modes taken from the z-update that ends the inner loop (final_pass = 0,
8 < L <= 64) against the separate final pass (final_pass = 1, the same arithmetic on the same
input): every output of a fit, an assignment and an SLK-MS fit is bit-identical between the two,
whether the device's expectation of the last pass held (no final pass run), failed (a loose
tolerance ends the loop at the second pass, before any pass expects to be the last one), or the
pass count is fixed (the last pass allowed always writes them).  Only `final_passes` differs."""
import numpy as np
import pytest

import gen
from test_gpu_parity import _say, to_dev

pytestmark = pytest.mark.gpu

CASES = [dict(n=3001, d=32, L=12, K=10, seed=21), dict(n=5000, d=64, L=50, K=10, seed=22)]


def same(a, b):
    ra = {k: v for k, v in a["result"].items() if k != "final_passes"}
    rb = {k: v for k, v in b["result"].items() if k != "final_passes"}
    assert ra == rb, (a["result"], b["result"])
    assert a["z"].equal(b["z"]) and a["labels"].equal(b["labels"])
    for key in ("modes", "modes_next", "bound_trace", "modes_used"):
        if a.get(key) is None:
            continue
        if isinstance(a[key], np.ndarray):
            assert np.array_equal(a[key], b[key]), key
        else:
            assert a[key].equal(b[key]), key


@pytest.fixture(scope="module", params=range(len(CASES)), ids=lambda i: f"L{CASES[i]['L']}")
def problem(request, slk, torch):
    kw = CASES[request.param]
    inst = gen.gaussian_mixture(**kw)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=kw["K"], reorder=True)
    yield inst, x, g
    g.close()


def test_fit(problem, slk):
    inst, x, g = problem
    a = slk.fit(x, g, inst.init_modes, lam=1.0)
    b = slk.fit(x, g, inst.init_modes, lam=1.0, final_pass=1)
    same(a, b)
    ra, rb = a["result"], b["result"]
    _say(f"[final_pass] L={inst.L}: {ra['outer_iters']} outer, {ra['inner_iters_total']} z-updates, "
         f"{ra['final_passes']} final passes (forced: {rb['final_passes']})")
    assert rb["final_passes"] == rb["outer_iters"]
    assert ra["final_passes"] < ra["outer_iters"]


def test_assign_loose_tolerance_falls_back(problem, slk):
    inst, x, g = problem
    a = slk.assign(x, g, inst.init_modes, lam=1.0, tol=10.0)
    b = slk.assign(x, g, inst.init_modes, lam=1.0, tol=10.0, final_pass=1)
    same(a, b)
    # the loop ends at pass index 1; only passes from index 2 on predict from the bound
    assert a["result"]["inner_iters_last"] == 2
    assert a["result"]["final_passes"] == 1 and b["result"]["final_passes"] == 1


@pytest.mark.parametrize("passes", [1, 5])
def test_assign_fixed_passes(problem, slk, passes):
    inst, x, g = problem
    a = slk.assign(x, g, inst.init_modes, lam=1.0, fixed_inner=passes)
    b = slk.assign(x, g, inst.init_modes, lam=1.0, fixed_inner=passes, final_pass=1)
    same(a, b)
    assert a["result"]["final_passes"] == 0 and b["result"]["final_passes"] == 1


def test_fit_ms(problem, slk, torch):
    inst, x, g = problem
    m0 = x[inst.init_modes.astype(np.int64)].contiguous()
    a = slk.fit_ms(x, g, m0, lam=1.0, max_outer=3)
    b = slk.fit_ms(x, g, m0, lam=1.0, max_outer=3, final_pass=1)
    same(a, b)
    assert a["ms_steps"] == b["ms_steps"]
    assert b["result"]["final_passes"] == b["result"]["outer_iters"]
