"""Out-of-sample assignment (slk_predict) against the FP64 oracle (oracle/extend.py).

Bar: the queries' neighbour lists bit-identical (exact and MFMA searches), |dZ| <= 1e-5 per
entry, labels equal wherever the oracle's top two logits are resolvable in FP32."""
import numpy as np
import pytest

import gen
from oracle import extend, slk as orc
from test_gpu_parity import ZTOL, round_bf16, to_dev

pytestmark = pytest.mark.gpu


def queries(inst, m, seed):
    rng = np.random.default_rng(seed)
    base = inst.X[rng.integers(0, inst.N, m)]
    return (base + rng.normal(0, 0.5, base.shape)).astype(np.float32)


def check(z, lab, nn, ref, lam, k):
    assert np.array_equal(nn.cpu().numpy(), ref["idx"])
    assert np.abs(z.cpu().numpy() - ref["Z"]).max() <= ZTOL
    S = ref["S"]
    srt = np.sort(S, axis=1)
    second = srt[:, -2] if S.shape[1] > 1 else np.full(len(S), -np.inf)
    slack = 1e-6 + 64 * np.spacing(np.abs(srt[:, -1]).astype(np.float32)) + lam * k * 1e-6
    res = (srt[:, -1] - second) > slack
    lab = lab.cpu().numpy()
    assert np.array_equal(lab[res], ref["labels"][res])
    assert np.all(S[np.arange(len(lab)), lab] >= srt[:, -1] - slack)


@pytest.mark.parametrize("L,m,k,method", [(5, 37, 10, "exact"), (5, 1001, 10, "mfma"), (12, 300, 1, "exact"),
                                          (40, 513, 7, "mfma"), (70, 200, 10, "exact"),
                                          (6, 12003, 10, "exact")])
def test_predict_against_oracle(slk, torch, L, m, k, method):
    inst = gen.gaussian_mixture(n=1500, d=12, L=L, K=10, seed=50 + L)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=10, method="exact")
    fit = slk.assign(x, g, inst.init_modes, lam=inst.lam, fixed_inner=6)
    Z = fit["z"]
    Y = queries(inst, m, seed=L)
    s2 = g.info()["sigma2"]
    z, lab, nn = slk.predict(x, Z, inst.init_modes, to_dev(torch, Y, torch.float32), k=k, lam=0.8, sigma2=s2,
                             method=method)
    ref = extend.predict(inst.X, Z.cpu().numpy().astype(np.float64), inst.init_modes, Y, k, s2, 0.8)
    check(z, lab, nn, ref, 0.8, k)


@pytest.mark.parametrize("m", [4095, 4101])
def test_predict_exact_widths(slk, torch, m):
    """Queries into 20,000 x 64 points (5 MiB): the exact search runs 4 queries per work-group
    below 4,096 queries and 8 from there.  Z is any row-stochastic matrix (seeded); each query's
    result depends on that query alone, so the oracle checks a sample: the first and last 40
    queries and 200 drawn at random."""
    inst = gen.gaussian_mixture(n=20000, d=64, L=6, K=10, seed=81)
    rng = np.random.default_rng(m)
    Zh = rng.random((inst.N, 6)) + 0.05
    Zh = (Zh / Zh.sum(axis=1, keepdims=True)).astype(np.float32)
    x = to_dev(torch, inst.X, torch.float32)
    Y = queries(inst, m, seed=m)
    z, lab, nn = slk.predict(x, to_dev(torch, Zh, torch.float32), inst.init_modes, to_dev(torch, Y, torch.float32),
                             k=10, lam=0.8, sigma2=2000.0, method="exact")
    rows = np.unique(np.concatenate([np.arange(40), np.arange(m - 40, m), rng.integers(0, m, 200)]))
    ref = extend.predict(inst.X, Zh.astype(np.float64), inst.init_modes, Y[rows], 10, 2000.0, 0.8)
    r = torch.as_tensor(rows, device="cuda")
    check(z[r], lab[r], nn[r], ref, 0.8, 10)


def test_predict_long_scan(slk, torch):
    """40,001 queries (the plain MFMA search, not the split one) into 2^19 + 777 points of 48
    coordinates: the candidate search tests whole key tiles before merging (long scans), with no
    point excluded and fewer queries than keys.  Z is a seeded row-stochastic matrix; the oracle
    checks the first and last 20 queries and 60 drawn at random."""
    n, m = (1 << 19) + 777, 40001
    assert slk.tune_lookup(n, 48, 6)["knn_long_scan"] == 1
    inst = gen.gaussian_mixture(n=n, d=48, L=6, K=10, seed=83)
    rng = np.random.default_rng(7)
    Zh = rng.random((n, 6)) + 0.05
    Zh = (Zh / Zh.sum(axis=1, keepdims=True)).astype(np.float32)
    x = to_dev(torch, inst.X, torch.float32)
    Y = queries(inst, m, seed=9)
    z, lab, nn = slk.predict(x, to_dev(torch, Zh, torch.float32), inst.init_modes, to_dev(torch, Y, torch.float32),
                             k=10, lam=0.8, sigma2=200.0, method="mfma")
    rows = np.unique(np.concatenate([np.arange(20), np.arange(m - 20, m), rng.integers(0, m, 60)]))
    ref = extend.predict(inst.X, Zh.astype(np.float64), inst.init_modes, Y[rows], 10, 200.0, 0.8)
    r = torch.as_tensor(rows, device="cuda")
    check(z[r], lab[r], nn[r], ref, 0.8, 10)


def test_predict_bf16_points(slk, torch):
    inst = gen.gaussian_mixture(n=1200, d=20, L=6, K=10, seed=61)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=10, method="exact")
    Z = slk.assign(x, g, inst.init_modes, lam=1.0, fixed_inner=5)["z"]
    Y = queries(inst, 400, seed=3)
    s2 = g.info()["sigma2"]
    for method in ("exact", "mfma"):
        z, lab, nn = slk.predict(x, Z, inst.init_modes, to_dev(torch, Y, torch.float32), k=10, lam=1.0, sigma2=s2,
                                 method=method, prec="bf16")
        ref = extend.predict(round_bf16(inst.X), Z.cpu().numpy().astype(np.float64), inst.init_modes, round_bf16(Y),
                             10, s2, 1.0)
        check(z, lab, nn, ref, 1.0, 10)


def test_predict_copy_of_fitted_point(slk, torch):
    """A query equal to a fitted point has that point as its first neighbour (distance 0)."""
    inst = gen.gaussian_mixture(n=800, d=8, L=4, K=8, seed=71)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=8, method="exact")
    Z = slk.assign(x, g, inst.init_modes, lam=1.0, fixed_inner=4)["z"]
    rows = np.array([0, 5, 799])
    _, _, nn = slk.predict(x, Z, inst.init_modes, x[torch.as_tensor(rows, device="cuda")], k=9, lam=1.0,
                           graph=g, method="mfma")
    nn = nn.cpu().numpy()
    own = g.export()["knn_idx"].cpu().numpy()[rows]
    assert np.array_equal(nn[:, 0], rows) and np.array_equal(nn[:, 1:], own)


def test_predict_rejects_bad_arguments(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    inst = gen.gaussian_mixture(n=100, d=4, L=3, K=5, seed=1)
    x = to_dev(torch, inst.X, torch.float32)
    Z = torch.full((100, 3), 1.0 / 3, device="cuda")
    y = x[:4].clone()
    with pytest.raises(SlkError):
        slk.predict(x, Z, inst.init_modes, y, k=0, sigma2=1.0)
    with pytest.raises(SlkError):
        slk.predict(x, Z, [0, 1, 100], y, k=3, sigma2=1.0)
    with pytest.raises(SlkError):
        slk.predict(x, Z, inst.init_modes, y, k=3, sigma2=float("inf"))
