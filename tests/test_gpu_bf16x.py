"""BF16-X (SLK_PREC_BF16X): the unary distance contraction on bf16 MFMA (three-term bf16 split of
tile-centred points, FP32 accumulation) against the FP64 oracle on the FP32 points.

The unary term is held to a bound derived from the arithmetic, per entry (p, l), with
y = x_p - c and w = m_l - c for the reference c of p's tile (the first of its 32 rows):
  |d2_gpu - d2| <= 2 (3 * 2^-27 + (6D/16 + 32) 2^-24) |y| |w| + (D + 8) 2^-24 (|y|^2 + |w|^2)
(split residuals and dropped products, FP32 accumulation of the MFMA products, FP32 norms and
centring), so |a_gpu - a| <= a (exp(bound / (2 sigma^2)) - 1) + 2^-21 a, and Z^0 = softmax(a) moves
by at most twice the largest error of its row.  The z-updates that follow run at the FP32 parity
bar from the GPU's own unary term, and the fit's FP64 energy recheck is exact at its labels."""
import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import CASES, ZTOL, _say, make_case, oracle_graph, rel_gap, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu

UCASES = [("mixture-2k", {}), ("ragged-1001-L7", dict(n=1001, d=9, L=7, K=5, seed=8)),
          ("wide-L70", dict(n=700, d=6, L=70, K=6, seed=9)), ("d64", dict(n=3001, d=64, L=6, K=8, seed=11)),
          ("L200", dict(n=1500, d=40, L=200, K=6, seed=12)), ("d130", dict(n=777, d=130, L=33, K=5, seed=13))]


def unary_bound(X, modes, s2):
    X64 = X.astype(np.float64)
    N, D = X64.shape
    M = X64[np.asarray(modes)]
    out = np.empty((N, len(modes)))
    for t0 in range(0, N, 32):
        T = X64[t0:t0 + 32]
        c = X64[t0]
        ny = np.sqrt(((T - c) ** 2).sum(axis=1))[:, None]
        nw = np.sqrt(((M - c) ** 2).sum(axis=1))[None, :]
        out[t0:t0 + 32] = (2 * (3 * 2.0 ** -27 + (6 * D / 16 + 32) * 2.0 ** -24) * ny * nw
                           + (D + 8) * 2.0 ** -24 * (ny ** 2 + nw ** 2))
    return np.expm1(out / (2 * s2)) + 2.0 ** -21


@pytest.mark.parametrize("name,kw", UCASES)
def test_bf16x_unary_within_its_bound(name, kw, slk, torch):
    inst = make_case(name, kw)
    modes = inst.init_modes
    s2 = oracle_graph(inst)[4]
    a, z0 = slk.unary(to_dev(torch, inst.X, torch.float32), modes, s2, prec="bf16x")
    A = orc.unary(inst.X, modes, s2)
    err = np.abs(a.cpu().numpy() - A)
    bound = A * unary_bound(inst.X, modes, s2)
    _say(f"[bf16x unary] {name}: max rel err {np.max(err / np.maximum(A, 1e-300)):.2e}, "
         f"largest err / bound {np.max(err / np.maximum(bound, 1e-300)):.3f}")
    assert np.all(err <= bound + 1e-40)
    zb = 2 * bound.max(axis=1, keepdims=True) + 1e-6
    assert np.all(np.abs(z0.cpu().numpy() - orc.softmax_rows(A)) <= zb)


@pytest.fixture(scope="module", params=[c[0] for c in CASES if c[0] != "L1"])
def case(request, torch):
    name = request.param
    inst = make_case(name, dict(CASES)[name])
    idx, d2, rp, ci, s2 = oracle_graph(inst)
    return dict(inst=inst, idx=idx, d2=d2, rp=rp, ci=ci, s2=s2, x=to_dev(torch, inst.X, torch.float32))


def test_bf16x_lockstep_fit(case, slk, torch):
    """Outer iterations in lock-step (the GPU's modes, the oracle's pass counts) with the oracle
    iterating from the GPU's BF16-X unary term: Z, resolvable labels, modes in the tie sets, the
    FP64 energy recheck exact at the GPU's labels and modes."""
    inst = case["inst"]
    g = slk.Graph.from_knn(to_dev(torch, case["idx"], torch.int32), to_dev(torch, case["d2"], torch.float64))
    modes = inst.init_modes.copy()
    for t in range(20):
        a, _ = slk.unary(case["x"], modes, case["s2"], prec="bf16x")
        A_gpu = a.cpu().numpy().astype(np.float64)
        out = orc.assign(inst.X, case["rp"], case["ci"], modes, case["s2"], inst.lam, A=A_gpu)
        res = slk.assign(case["x"], g, modes, lam=inst.lam, fixed_inner=out["n_pass"], prec="bf16x")
        z = res["z"].cpu().numpy()
        dz = float(np.abs(z - out["Z"]).max())
        ztol = trajectory_ztol(out, case["rp"], case["ci"], inst.lam, dz)
        lab = res["labels"].cpu().numpy()
        S = out["S"]
        srt = np.sort(S, axis=1)
        top = srt[:, -1]
        second = srt[:, -2] if inst.L > 1 else np.full(inst.N, -np.inf)
        slack = 1e-6 + 64 * np.spacing(np.abs(top).astype(np.float32)).astype(np.float64) \
            + inst.lam * np.diff(case["rp"]) * ztol
        resolvable = (top - second) > slack
        _say(f"[bf16x lockstep] {inst.name} outer {t}: passes={out['n_pass']} max|dZ|={dz:.2e} ztol={ztol:.2e}")
        assert dz <= ztol
        assert np.mean(lab[resolvable] == out["labels"][resolvable]) >= 0.999
        assert np.all(S[np.arange(inst.N), lab] >= top - slack)
        r = res["result"]
        E64, cut = orc.energy(orc.unary(inst.X, modes, case["s2"]), lab, case["rp"], case["ci"], inst.lam)
        assert r["cut"] == cut and rel_gap(r["energy_fp64"], E64) <= 1e-12
        E_at, _ = orc.energy(A_gpu, lab, case["rp"], case["ci"], inst.lam)
        assert rel_gap(r["energy"], E_at) <= 1e-6
        nxt = res["modes_next"].astype(np.int64)
        V = out["V"]
        for l in range(inst.L):
            vb = V[out["modes_next"][l], l]
            assert nxt[l] in out["ties"][l] or V[nxt[l], l] >= vb - orc.tie_eps(vb) - 2 * inst.lam * ztol * np.diff(case["rp"]).max()
        if np.array_equal(nxt, modes):
            break
        modes = nxt
