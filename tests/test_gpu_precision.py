"""The BF16-X path: points rounded to bfloat16 once, for the kNN distances and the unary term.

It must be exactly the FP32 path run on the rounded points (so it inherits that path's parity
with the FP64 oracle, here checked again against the oracle on the rounded points), and its
FP64 energy recheck must evaluate the original FP32 points.  Its error against the FP32 problem
is stated, not assumed: at the C1 mixture the two paths reach the same modes and labels, with a
relative energy gap within 1e-4."""
import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import ETOL, ZTOL, rel_gap, round_bf16, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    inst = gen.make("mixture-2k")
    Xb = round_bf16(inst.X)
    idx, d2 = orc.knn(Xb, inst.K, block=256)
    rp, ci = orc.symmetrize(idx, inst.N)
    return dict(inst=inst, Xb=Xb, rp=rp, ci=ci, s2=orc.sigma2_from_knn(d2))


def test_bf16_path_is_fp32_path_on_rounded_points(c1, slk, torch):
    inst = c1["inst"]
    x = to_dev(torch, inst.X, torch.float32)
    xb = to_dev(torch, c1["Xb"], torch.float32)
    gb = slk.Graph.build_knn(x, k=inst.K, method="exact", prec="bf16")
    g32 = slk.Graph.build_knn(xb, k=inst.K, method="exact")
    a = slk.fit(x, gb, inst.init_modes, lam=inst.lam, prec="bf16")
    b = slk.fit(xb, g32, inst.init_modes, lam=inst.lam)
    assert torch.equal(a["z"], b["z"]) and torch.equal(a["labels"], b["labels"])
    assert np.array_equal(a["modes"], b["modes"])
    ra, rb = a["result"], b["result"]
    assert ra["energy"] == rb["energy"] and ra["cut"] == rb["cut"]
    # the recheck of the BF16 run evaluates the original points (at the converged modes)
    assert ra["converged"] == 1
    E_true, _ = orc.energy(orc.unary(inst.X, a["modes"], gb.info()["sigma2"]), a["labels"].cpu().numpy(),
                           c1["rp"], c1["ci"], inst.lam)
    assert rel_gap(ra["energy_fp64"], E_true) <= ETOL


def test_bf16_assign_against_oracle_on_rounded_points(c1, slk, torch):
    inst = c1["inst"]
    x = to_dev(torch, inst.X, torch.float32)
    gb = slk.Graph.build_knn(x, k=inst.K, method="mfma", prec="bf16")
    out = orc.assign(c1["Xb"], c1["rp"], c1["ci"], inst.init_modes, c1["s2"], inst.lam)
    res = slk.assign(x, gb, inst.init_modes, lam=inst.lam, fixed_inner=out["n_pass"], prec="bf16")
    ztol = trajectory_ztol(out, c1["rp"], c1["ci"], inst.lam)
    assert np.abs(res["z"].cpu().numpy() - out["Z"]).max() <= ztol
    lab = res["labels"].cpu().numpy()
    # labels equal wherever the oracle's top two logits are resolvable in FP32 (at the initial
    # modes two modes can sit in one cluster and tie), else inside the near-tie set
    S = out["S"]
    srt = np.sort(S, axis=1)
    deg = np.diff(c1["rp"]).astype(np.float64)
    slack = 1e-6 + 64 * np.spacing(np.abs(srt[:, -1]).astype(np.float32)).astype(np.float64) + inst.lam * deg * ztol
    resolvable = (srt[:, -1] - srt[:, -2]) > slack
    assert np.mean(lab[resolvable] == out["labels"][resolvable]) >= 0.999
    assert np.all(S[np.arange(len(lab)), lab] >= srt[:, -1] - slack)
    E_b, cut = orc.energy(out["A"], lab, c1["rp"], c1["ci"], inst.lam)
    assert res["result"]["cut"] == cut
    assert rel_gap(res["result"]["energy"], E_b) <= 1e-5
    E_true = orc.energy_of(inst.X, c1["rp"], c1["ci"], lab, inst.init_modes, c1["s2"], inst.lam)[0]
    assert rel_gap(res["result"]["energy_fp64"], E_true) <= ETOL


def test_bf16_energy_error_against_fp32_problem(slk, torch):
    """Both paths' solutions evaluated on the FP32 problem (FP32 graph, FP64 unary term)."""
    inst = gen.make("mixture-2k")
    x = to_dev(torch, inst.X, torch.float32)
    g32 = slk.Graph.build_knn(x, k=inst.K, method="exact")
    gb = slk.Graph.build_knn(x, k=inst.K, method="exact", prec="bf16")
    a = slk.fit(x, g32, inst.init_modes, lam=inst.lam)
    b = slk.fit(x, gb, inst.init_modes, lam=inst.lam, prec="bf16")
    ea = slk.energy(x, g32, a["labels"], a["modes"], lam=inst.lam)
    eb = slk.energy(x, g32, b["labels"], b["modes"], lam=inst.lam)
    assert rel_gap(eb["energy_fp64"], ea["energy_fp64"]) <= 1e-4
    assert np.mean(a["labels"].cpu().numpy() == b["labels"].cpu().numpy()) >= 0.999
