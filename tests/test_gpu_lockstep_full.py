"""Whole SLK-BO fits at full size, in lock-step with the FP64 oracle (Algorithm 1 end to end):
large-1m in the benchmark's launch configuration (MFMA kNN, locality order, lambda = 1) and
images-70k at lambda = 0.5, 1 and 2.

The GPU runs its own fit.  The oracle then runs each of its outer iterations from the same modes,
with the GPU's pass count (reading R10: FP32 and FP64 can stop a pass apart) on the GPU's graph,
which is checked first: sampled kNN rows bit-identical to the oracle's, the CSR equal to the
oracle's OR-symmetrisation of the GPU's lists, sigma^2 equal to the oracle's estimator.  Per outer
iteration: all N x L entries of Z (1e-5, or the float32 reference's own distance where larger),
labels equal on the resolvable rows (>= 99.9%) and inside the near-tie set elsewhere, the GPU's
byproduct modes inside the oracle's tie sets (the next outer iteration starts from them), the cut
exact, the FP64 energy of the GPU's labels within 1e-6 of the oracle's, the bound trace within
1e-5.  The oracle's row-wise steps run over row blocks on a thread pool (tests/par_oracle.py;
bit-identical to oracle.slk.assign)."""
import numpy as np
import pytest

import gen
import par_oracle
from oracle import slk as orc
from test_gpu_parity import ZTOL, _say, check_outer, gpu_outer_history, rel_gap, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu

CASES = [("large-1m", 1.0), ("images-70k", 0.5), ("images-70k", 1.0), ("images-70k", 2.0)]
_BUILT = {}


@pytest.fixture(scope="module")
def pool():
    p = par_oracle.RowPool()
    yield p
    p.close()


@pytest.fixture(scope="module")
def built(slk, torch):
    yield _BUILT
    for v in _BUILT.values():
        v["g"].close()
    _BUILT.clear()


def get(built, name, slk, torch):
    if name in built:
        return built[name]
    for other in list(built):
        built.pop(other)["g"].close()
    inst = gen.make(name)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=inst.K, method="mfma", reorder=(name == "large-1m"))
    info = g.info()
    ex = g.export()
    knn_idx = ex["knn_idx"].cpu().numpy().astype(np.int64)
    knn_d2 = ex["knn_d2"].cpu().numpy()
    rp, ci = orc.symmetrize(knn_idx, inst.N)
    assert np.array_equal(ex["row_ptr"].cpu().numpy(), rp) and np.array_equal(ex["col_idx"].cpu().numpy(), ci)
    s2 = orc.sigma2_from_knn(knn_d2)
    assert rel_gap(info["sigma2"], s2) <= 1e-12
    rows = np.random.default_rng(4).choice(inst.N, 8, replace=False)
    oi, od = orc.knn(inst.X, inst.K, rows=rows, block=8)
    assert np.array_equal(knn_idx[rows], oi) and np.array_equal(knn_d2[rows], od)
    X64 = inst.X.astype(np.float64)
    built[name] = dict(inst=inst, x=x, g=g, rp=rp, ci=ci, s2=s2, X64=X64, XT=np.ascontiguousarray(X64.T),
                       W=orc.csr_matrix(rp, ci, inst.N))
    _say(f"[full] {name}: graph checked (nnz={len(ci)}, sigma2={s2:.6f})")
    return built[name]


@pytest.mark.parametrize("name,lam", CASES)
def test_fit_lockstep_full(name, lam, built, pool, slk, torch):
    b = get(built, name, slk, torch)
    inst, x, g, rp, ci = b["inst"], b["x"], b["g"], b["rp"], b["ci"]
    res = slk.fit(x, g, inst.init_modes, lam=lam)
    r = res["result"]
    hist = gpu_outer_history(slk, x, g, inst.init_modes, lam)
    last = hist[-1][1]
    assert len(hist) == r["outer_iters"]
    assert torch.equal(last["labels"], res["labels"]) and torch.equal(last["z"], res["z"])
    assert last["result"]["energy_fp64"] == r["energy_fp64"] and last["result"]["cut"] == r["cut"]
    inst_l = gen.Instance(inst.name, inst.X, inst.L, inst.K, lam, inst.init_modes, inst.labels_true, inst.seed)
    for t, (m, rt) in enumerate(hist):
        n_pass = rt["result"]["inner_iters_last"]
        out = par_oracle.assign(pool, b["X64"], rp, ci, m, b["s2"], lam, n_pass, W=b["W"], XT=b["XT"])
        dz = float(np.abs(rt["z"].cpu().numpy() - out["Z"]).max())
        ztol = trajectory_ztol(out, rp, ci, lam, dz)
        lab = rt["labels"].cpu().numpy()
        st = check_outer(rt, out, inst_l, rp, ci, lam, ztol)
        _say(f"[full] {name} lam={lam} outer {t}: passes={n_pass} max|dZ|={dz:.2e} ztol={ztol:.2e} labels: "
             f"{st['agree_all']:.6f} of all rows, {st['agree_resolvable']:.6f} of the {st['resolvable']} resolvable; "
             f"E_gpu={rt['result']['energy_fp64']:.6f}, the oracle's own labels {out['E']:.6f}")
        np.testing.assert_allclose(rt["bound_trace"], out["R_trace"], rtol=1e-5, atol=1e-6)
    E_at, _ = orc.energy(out["A"], lab, rp, ci, lam)
    assert rel_gap(r["energy_fp64"], E_at) <= 1e-6
