"""Rows of very high degree (hubs of the kNN graph) against the FP64 oracle.

A kNN graph's symmetrised rows can be far longer than k (a point that is among the nearest
neighbours of many others).  The library updates rows of degree above its heavy-row
threshold with a whole work-group each; these tests build hubs of degree 140 to 1,510 on
purpose and check the z-update, one outer iteration, the energy and the labels against the
oracle, for row widths that take each lane-group size of the float4 path (L = 5, 12, 24, 50)
and the wide path (L = 70)."""
import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import ZTOL, check_outer, rel_gap, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu

WIDTHS = [5, 12, 24, 50, 70]


@pytest.fixture(scope="module")
def hubs():
    inst = gen.star_hubs()
    idx, d2 = orc.knn(inst.X, inst.K, block=256)
    rp, ci = orc.symmetrize(idx, inst.N)
    return dict(inst=inst, idx=idx, d2=d2, rp=rp, ci=ci, s2=orc.sigma2_from_knn(d2))


def modes_for(inst, L):
    return np.random.default_rng(100 + L).choice(inst.N, L, replace=False).astype(np.int32)


def graph(slk, torch, h, reorder):
    return slk.Graph.from_knn(to_dev(torch, h["idx"], torch.int32), to_dev(torch, h["d2"], torch.float64),
                              reorder=reorder)


def test_hub_degrees(hubs, slk, torch):
    g = graph(slk, torch, hubs, True)
    info = g.info()
    assert info["max_degree"] == int(np.diff(hubs["rp"]).max()) >= 1500
    assert int((np.diff(hubs["rp"]) > 128).sum()) >= 4


@pytest.mark.parametrize("L", WIDTHS)
@pytest.mark.parametrize("reorder", [False, True])
def test_hub_inner_step(hubs, slk, torch, L, reorder):
    inst = hubs["inst"]
    g = graph(slk, torch, hubs, reorder)
    A = orc.unary(inst.X, modes_for(inst, L), hubs["s2"]).astype(np.float32)
    Z = np.random.default_rng(L).dirichlet(np.ones(L), size=inst.N).astype(np.float32)
    z_out, bound = slk.inner_step(g, to_dev(torch, A, torch.float32), to_dev(torch, Z, torch.float32), lam=0.05)
    W = orc.csr_matrix(hubs["rp"], hubs["ci"], inst.N)
    A64, Z64 = A.astype(np.float64), Z.astype(np.float64)
    B = orc.pairwise(W, Z64)
    np.testing.assert_allclose(z_out.cpu().numpy(), orc.softmax_rows(A64 + 0.05 * B), atol=ZTOL)
    R = orc.relaxed_bound(Z64, A64, B, 0.05)
    assert abs(bound - R) <= 1e-5 * abs(R) + 1e-6


@pytest.mark.parametrize("L", WIDTHS)
def test_hub_assign_lockstep(hubs, slk, torch, L):
    inst = hubs["inst"]
    g = graph(slk, torch, hubs, True)
    modes = modes_for(inst, L)
    lam = 0.05
    out = orc.assign(inst.X, hubs["rp"], hubs["ci"], modes, hubs["s2"], lam)
    x = to_dev(torch, inst.X, torch.float32)
    res = slk.assign(x, g, modes, lam=lam, fixed_inner=out["n_pass"])
    inst_L = gen.Instance(inst.name, inst.X, L, inst.K, lam, modes, inst.labels_true, inst.seed)
    check_outer(res, out, inst_L, hubs["rp"], hubs["ci"], lam, trajectory_ztol(out, hubs["rp"], hubs["ci"], lam))
    np.testing.assert_allclose(res["bound_trace"], out["R_trace"], rtol=1e-5, atol=1e-6)


def test_hub_energy(hubs, slk, torch):
    inst = hubs["inst"]
    g = graph(slk, torch, hubs, True)
    rng = np.random.default_rng(5)
    lab = rng.integers(0, inst.L, size=inst.N).astype(np.int32)
    x = to_dev(torch, inst.X, torch.float32)
    e = slk.energy(x, g, to_dev(torch, lab, torch.int32), inst.init_modes, lam=0.3)
    A = orc.unary(inst.X, inst.init_modes, hubs["s2"])
    E, cut = orc.energy(A, lab, hubs["rp"], hubs["ci"], 0.3)
    assert e["cut"] == cut
    assert rel_gap(e["energy_fp64"], E) <= 1e-12
    assert rel_gap(e["energy"], E) <= 1e-5


def test_hub_reorder_and_determinism(hubs, slk, torch):
    """The locality order (which renumbers the hubs) only changes the order of the neighbour
    sums; repeated calls are bit-identical."""
    inst = hubs["inst"]
    x = to_dev(torch, inst.X, torch.float32)
    g0, g1 = graph(slk, torch, hubs, False), graph(slk, torch, hubs, True)
    a = slk.assign(x, g0, inst.init_modes, lam=0.05, fixed_inner=8)
    b = slk.assign(x, g1, inst.init_modes, lam=0.05, fixed_inner=8)
    assert (a["z"] - b["z"]).abs().max().item() <= ZTOL
    assert np.mean(a["labels"].cpu().numpy() == b["labels"].cpu().numpy()) >= 0.999
    c = slk.assign(x, g1, inst.init_modes, lam=0.05, fixed_inner=8)
    assert torch.equal(b["z"], c["z"]) and torch.equal(b["labels"], c["labels"])
    assert np.array_equal(b["modes_next"], c["modes_next"]) and b["result"] == c["result"]
