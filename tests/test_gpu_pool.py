"""Reuse of the library's device memory pool: calls that run on memory freed by earlier calls
(with other sizes in between, and after slk_pool_trim) return bit-identical results, and the
FP32 fit still matches the FP64 oracle's energy at its labels and modes."""
import math

import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import _say, rel_gap, to_dev

pytestmark = pytest.mark.gpu


def _fit(slk, torch, inst, method="exact"):
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=inst.K, method=method)
    out = slk.fit(x, g, inst.init_modes, lam=inst.lam)
    ex = g.export()
    res = dict(z=out["z"].cpu().numpy(), labels=out["labels"].cpu().numpy(), modes=np.asarray(out["modes"]).copy(),
               result=out["result"], knn_idx=ex["knn_idx"].cpu().numpy(), knn_d2=ex["knn_d2"].cpu().numpy(),
               sigma2=g.info()["sigma2"])
    g.close()
    return res


def _same(a, b):
    for k in ("z", "labels", "modes", "knn_idx", "knn_d2"):
        assert np.array_equal(a[k], b[k]), k
    assert a["result"] == b["result"]
    assert a["sigma2"] == b["sigma2"]


def test_reuse_across_sizes_and_trim(slk, torch):
    small = gen.make("mixture-2k")
    other = gen.gaussian_mixture(n=5003, d=24, L=9, K=7, seed=21, name="other-5003")
    _say("[pool] mixture-2k, then other-5003 (MFMA kNN), then mixture-2k again, trim, again")
    first = _fit(slk, torch, small)
    o1 = _fit(slk, torch, other, method="mfma")
    second = _fit(slk, torch, small)
    _same(first, second)
    slk.pool_trim()
    third = _fit(slk, torch, small)
    _same(first, third)
    o2 = _fit(slk, torch, other, method="mfma")
    _same(o1, o2)
    # the reused-memory fit is still the oracle's fit at its own labels and modes
    r = third["result"]
    rp, ci = orc.symmetrize(third["knn_idx"].astype(np.int64), small.N)
    lab = third["labels"].astype(np.int64)
    assert r["cut"] == orc.cut_count(rp, ci, lab)
    if r["converged"]:
        d = small.X[third["modes"][lab]].astype(np.float64) - small.X.astype(np.float64)
        U = math.fsum(np.exp(-(d * d).sum(axis=1) / (2.0 * third["sigma2"])).tolist())
        assert rel_gap(r["energy_fp64"], -U + small.lam * r["cut"]) <= 1e-9


def test_trim_is_repeatable(slk, torch):
    slk.pool_trim()
    slk.pool_trim()
