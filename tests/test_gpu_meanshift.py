"""SLK-MS on the GPU (slk_mean_shift, slk_fit_ms) against the FP64 oracle (oracle/extend.py).

Tolerance of a mode.  One mean-shift step is a weighted mean of the points; the GPU forms the
weights z * k in FP32 from the unary kernel (relative error within 2e-5, the unary test's
bound) and sums them in FP32 per 1,024-point block, then in FP64.  A relative weight error e
moves a weighted mean by at most 2e times the largest |x_pc - m_lc| among weighted points, so a
step lands within MTOL = 1e-4 * extent of the oracle's, extent = max |x_pc| + max |m_lc|
(5x the weight bound).  Steps taken from each side's own previous modes stay inside the same
bound near a fixed point (a step contracts toward the mode), so fixed-count runs use 2 * MTOL.
Assignments after a z-update block are held to the trajectory tolerance of the SLK-BO tests."""
import numpy as np
import pytest

import gen
from oracle import extend, slk as orc
from test_gpu_parity import ETOL, ZTOL, _say, oracle_graph, rel_gap, round_bf16, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu


def extent(X, M):
    return float(np.abs(X).max() + np.abs(M).max())


def start(inst):
    return inst.X[inst.init_modes].astype(np.float32)


def soft_z(inst, seed):
    return np.random.default_rng(seed).dirichlet(np.ones(inst.L), size=inst.N).astype(np.float32)


MS_CASES = [(3000, 12, 5, 1), (2500, 150, 7, 2), (37, 3, 3, 3), (1100, 9, 64, 4), (500, 4, 1, 5), (2049, 33, 20, 6)]


@pytest.mark.parametrize("n,d,L,seed", MS_CASES)
def test_mean_shift_one_step(slk, torch, n, d, L, seed):
    inst = gen.gaussian_mixture(n=n, d=d, L=L, K=8, seed=seed)
    s2 = 4.0 * d
    Z = soft_z(inst, seed)
    M0 = start(inst)
    m, it = slk.mean_shift(to_dev(torch, inst.X, torch.float32), to_dev(torch, Z, torch.float32),
                           to_dev(torch, M0, torch.float32), s2, tol=0.0, max_iter=1)
    ref = extend.mean_shift_step(inst.X, Z.astype(np.float64), M0, s2)
    err = np.abs(m.cpu().numpy() - ref).max()
    tol = 1e-4 * extent(inst.X, M0)
    _say(f"[ms step] n={n} d={d} L={L}: err={err:.2e} tol={tol:.2e}")
    assert it == 1 and err <= tol


@pytest.mark.parametrize("n,d,L,seed", MS_CASES[:4])
def test_mean_shift_fixed_steps(slk, torch, n, d, L, seed):
    inst = gen.gaussian_mixture(n=n, d=d, L=L, K=8, seed=seed)
    s2 = 4.0 * d
    Z = soft_z(inst, seed)
    M0 = start(inst)
    m, it = slk.mean_shift(to_dev(torch, inst.X, torch.float32), to_dev(torch, Z, torch.float32),
                           to_dev(torch, M0, torch.float32), s2, tol=0.0, max_iter=6)
    ref, rit = extend.mean_shift(inst.X, Z.astype(np.float64), M0, s2, tol=0.0, max_iter=6)
    err = np.abs(m.cpu().numpy() - ref).max()
    _say(f"[ms 6 steps] n={n} d={d} L={L}: err={err:.2e}")
    assert it == rit == 6 and err <= 2e-4 * extent(inst.X, M0)


def test_mean_shift_converges_to_oracle_fixed_point(slk, torch):
    inst = gen.gaussian_mixture(n=2000, d=8, L=4, K=8, seed=21)
    s2 = 6.0
    Z = np.eye(inst.L, dtype=np.float32)[inst.labels_true]
    M0 = start(inst)
    m, it = slk.mean_shift(to_dev(torch, inst.X, torch.float32), to_dev(torch, Z, torch.float32),
                           to_dev(torch, M0, torch.float32), s2, tol=1e-6, max_iter=500)
    ref, rit = extend.mean_shift(inst.X, Z.astype(np.float64), M0, s2, tol=1e-6, max_iter=500)
    m = m.cpu().numpy()
    _say(f"[ms converge] steps gpu={it} oracle={rit} err={np.abs(m - ref).max():.2e}")
    assert it < 500 and rit < 500
    assert np.abs(m - ref).max() <= 2e-4 * extent(inst.X, M0)
    # a fixed point of the oracle's step, to the same tolerance
    again = extend.mean_shift_step(inst.X, Z.astype(np.float64), m, s2)
    assert np.abs(again - m).max() <= 2e-4 * extent(inst.X, M0)


def test_mean_shift_zero_weight_cluster_keeps_its_mode(slk, torch):
    inst = gen.gaussian_mixture(n=1500, d=10, L=4, K=8, seed=31)
    Z = soft_z(inst, 1)
    Z[:, 2] = 0.0
    M0 = start(inst)
    m, _ = slk.mean_shift(to_dev(torch, inst.X, torch.float32), to_dev(torch, Z, torch.float32),
                          to_dev(torch, M0, torch.float32), 40.0, tol=0.0, max_iter=3)
    m = m.cpu().numpy()
    assert np.array_equal(m[2], M0[2])
    ref, _ = extend.mean_shift(inst.X, Z.astype(np.float64), M0, 40.0, tol=0.0, max_iter=3)
    assert np.abs(m - ref).max() <= 2e-4 * extent(inst.X, M0)


def test_mean_shift_bf16_points(slk, torch):
    inst = gen.gaussian_mixture(n=2100, d=24, L=6, K=8, seed=41)
    Z = soft_z(inst, 2)
    M0 = start(inst) + np.float32(0.123)        # mode vectors off the bf16 grid stay as they are
    m, _ = slk.mean_shift(to_dev(torch, inst.X, torch.float32), to_dev(torch, Z, torch.float32),
                          to_dev(torch, M0, torch.float32), 96.0, tol=0.0, max_iter=2, prec="bf16")
    Xr = round_bf16(inst.X)
    ref, _ = extend.mean_shift(Xr, Z.astype(np.float64), M0, 96.0, tol=0.0, max_iter=2)
    assert np.abs(m.cpu().numpy() - ref).max() <= 2e-4 * extent(Xr, M0)


def test_mean_shift_rejects_bad_arguments(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    x = torch.zeros((100, 4), device="cuda")
    z = torch.full((100, 65), 1.0 / 65, device="cuda")
    with pytest.raises(SlkError):
        slk.mean_shift(x, z, torch.zeros((65, 4), device="cuda"), 1.0)
    z = z[:, :3].contiguous()
    m0 = torch.zeros((3, 4), device="cuda")
    with pytest.raises(SlkError):
        slk.mean_shift(x, z, m0, 0.0)
    with pytest.raises(SlkError):
        slk.mean_shift(x, z, m0, 1.0, max_iter=0)
    with pytest.raises(SlkError):
        slk.mean_shift(x, z, m0, 1.0, tol=-1.0)


# ------------------------------------------------------------------- SLK-MS fit

def check_stage(res, inst, rp, ci, s2, lam, n_inner, ms_steps):
    """The GPU's last outer iteration against the oracle run from the GPU's own inputs to it:
    the z-update block at the GPU's modes_used (assignment, labels, cut, energy), then the
    mean-shift from the GPU's Z and modes_used (modes)."""
    Mu = res["modes_used"].cpu().numpy().astype(np.float64)
    out = orc.assign(inst.X, rp, ci, None, s2, lam, n_inner=n_inner, A=extend.unary_at(inst.X, Mu, s2))
    ztol = trajectory_ztol(out, rp, ci, lam)
    z = res["z"].cpu().numpy()
    dz = np.abs(z - out["Z"]).max()
    assert dz <= ztol, (dz, ztol)
    lab = res["labels"].cpu().numpy()
    S = out["S"]
    srt = np.sort(S, axis=1)
    second = srt[:, -2] if S.shape[1] > 1 else np.full(len(S), -np.inf)
    deg = np.diff(rp).astype(np.float64)
    slack = 1e-6 + 64 * np.spacing(np.abs(srt[:, -1]).astype(np.float32)) + lam * deg * ztol
    res_rows = (srt[:, -1] - second) > slack
    assert np.mean(lab[res_rows] == out["labels"][res_rows]) >= 0.999
    E_at, cut_at = orc.energy(out["A"], lab, rp, ci, lam)
    r = res["result"]
    assert r["cut"] == cut_at
    assert rel_gap(r["energy_fp64"], E_at) <= ETOL
    ref, _ = extend.mean_shift(inst.X, z.astype(np.float64), Mu, s2, tol=0.0, max_iter=ms_steps)
    err = np.abs(res["modes"].cpu().numpy() - ref).max()
    assert err <= 2e-4 * extent(inst.X, Mu), err
    return dz, err


@pytest.mark.parametrize("name,kw,reorder", [
    ("mixture", dict(n=2000, d=16, L=5, K=10, seed=0), False),
    ("ragged-reordered", dict(n=1001, d=9, L=7, K=5, seed=8), True),
    ("wide-d", dict(n=1300, d=130, L=4, K=8, seed=12), True),
    ("L1", dict(n=200, d=4, L=1, K=5, seed=10), False),
])
def test_fit_ms_stagewise(slk, torch, name, kw, reorder):
    inst = gen.gaussian_mixture(**kw, name=name)
    idx, d2, rp, ci, s2 = oracle_graph(inst)
    g = slk.Graph.from_knn(to_dev(torch, idx, torch.int32), to_dev(torch, d2, torch.float64), reorder=reorder)
    x = to_dev(torch, inst.X, torch.float32)
    M0 = start(inst)
    for outer in (1, 3):
        res = slk.fit_ms(x, g, to_dev(torch, M0, torch.float32), lam=inst.lam, fixed_inner=7, max_outer=outer,
                         ms_tol=0.0, ms_max_iter=4)
        r = res["result"]
        assert r["outer_iters"] == outer and res["ms_steps"] == 4 * outer
        if outer == 1:
            assert np.array_equal(res["modes_used"].cpu().numpy(), M0)
        dz, err = check_stage(res, inst, rp, ci, s2, inst.lam, 7, 4)
        _say(f"[fit_ms] {name} outer={outer}: dz={dz:.2e} dm={err:.2e}")


def test_fit_ms_free_running(slk, torch):
    """Run to convergence on both sides from the same start: the same clustering and the same
    modes (to the fixed-point tolerance), and the GPU's final modes a fixed point of the
    oracle's mean-shift for the GPU's Z.  The start takes one point of every generating
    component: from two seeds in one component both modes climb to nearly the same place and
    the split of that component between them is decided by rounding (a degenerate start that
    the stagewise test covers instead)."""
    inst = gen.gaussian_mixture(n=2000, d=16, L=5, K=10, seed=0)
    idx, d2, rp, ci, s2 = oracle_graph(inst)
    g = slk.Graph.from_knn(to_dev(torch, idx, torch.int32), to_dev(torch, d2, torch.float64))
    M0 = inst.X[[int(np.nonzero(inst.labels_true == l)[0][0]) for l in range(inst.L)]].astype(np.float32)
    res = slk.fit_ms(to_dev(torch, inst.X, torch.float32), g, to_dev(torch, M0, torch.float32), lam=inst.lam,
                     ms_tol=1e-6, ms_max_iter=200)
    ref = extend.fit_ms(inst.X, rp, ci, M0, s2, inst.lam, ms_tol=1e-6, ms_max=200)
    r = res["result"]
    _say(f"[fit_ms free] gpu outer={r['outer_iters']} conv={r['converged']} oracle outer={ref['outer_iters']} "
         f"conv={ref['converged']}")
    assert r["converged"] and ref["converged"]
    lab = res["labels"].cpu().numpy()
    assert np.mean(lab == ref["labels"]) >= 0.999
    m = res["modes"].cpu().numpy()
    tol = 2e-4 * extent(inst.X, M0)
    assert np.abs(m - ref["modes"]).max() <= tol
    again = extend.mean_shift_step(inst.X, res["z"].cpu().numpy().astype(np.float64), m, s2)
    assert np.abs(again - m).max() <= tol


def test_fit_ms_free_running_random_start(slk, torch):
    """From the random start of reading R12, where two seeds fall into one generating component
    (twice at this seed: the seeds come from components 3, 2, 3, 0, 2): both sides converge, each
    pair of modes of one component to two points ~0.27 apart, and the rows of those components
    have two logits equal to within FP32 resolution, so their split between the pair is decided by
    rounding on either side.  Held to: modes within the fixed-point tolerance, labels equal on the
    rows the oracle resolves and inside its near-tie set elsewhere, energy within 1e-6."""
    inst = gen.gaussian_mixture(n=2000, d=16, L=5, K=10, seed=0)
    idx, d2, rp, ci, s2 = oracle_graph(inst)
    g = slk.Graph.from_knn(to_dev(torch, idx, torch.int32), to_dev(torch, d2, torch.float64))
    M0 = start(inst)
    res = slk.fit_ms(to_dev(torch, inst.X, torch.float32), g, to_dev(torch, M0, torch.float32), lam=inst.lam,
                     ms_tol=1e-6, ms_max_iter=200)
    ref = extend.fit_ms(inst.X, rp, ci, M0, s2, inst.lam, ms_tol=1e-6, ms_max=200)
    r = res["result"]
    assert r["converged"] and ref["converged"]
    m = res["modes"].cpu().numpy()
    assert np.abs(m - ref["modes"]).max() <= 2e-4 * extent(inst.X, M0)
    lab = res["labels"].cpu().numpy()
    S = ref["S"]
    srt = np.sort(S, axis=1)
    top, second = srt[:, -1], srt[:, -2]
    slack = 1e-6 + 64 * np.spacing(np.abs(top).astype(np.float32)).astype(np.float64) + inst.lam * np.diff(rp) * ZTOL
    resolvable = (top - second) > slack
    _say(f"[fit_ms random start] seeds' components {inst.labels_true[inst.init_modes].tolist()}, resolvable rows "
         f"{int(resolvable.sum())}, labels equal on all rows {np.mean(lab == ref['labels']):.3f}")
    assert np.mean(lab[resolvable] == ref["labels"][resolvable]) >= 0.999
    assert np.all(S[np.arange(inst.N), lab] >= top - slack)
    assert rel_gap(r["energy_fp64"], ref["E"]) <= ETOL


def test_fit_ms_rejects_bad_arguments(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    inst = gen.gaussian_mixture(n=300, d=4, L=3, K=5, seed=1)
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=5, method="exact")
    m0 = to_dev(torch, start(inst), torch.float32)
    with pytest.raises(SlkError):
        slk.fit_ms(x, g, m0, ms_max_iter=0)
    with pytest.raises(SlkError):
        slk.fit_ms(x, g, m0, ms_tol=-1.0)
    with pytest.raises(SlkError):
        slk.fit_ms(x, g, torch.zeros((65, 4), device="cuda"))
