"""The served and batched form (slk_server_*, slk_fit_batched) on the GPU.

Every job keeps the work-groups, tiles and reduction order of its own slk_fit, so the tests
require its outputs to be bit-identical to a solo fit whether it runs alone or in a mix of
uneven jobs that join and leave while others run; one job is also checked against the FP64
oracle directly."""
import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import check_outer, rel_gap, to_dev, trajectory_ztol

pytestmark = pytest.mark.gpu


def small_stream(n_jobs=10, seed=7):
    specs = gen.job_stream(n_jobs=n_jobs, rate=100.0, seed=seed, n_lo=200, n_hi=4000, dims=(8, 16, 40),
                           L_lo=2, L_hi=40, K=10)
    return [gen.materialise(sp, K=10) for sp in specs]


def solo(slk, torch, inst, method="auto"):
    x = to_dev(torch, inst.X, torch.float32)
    g = slk.Graph.build_knn(x, k=inst.K, method=method)
    return slk.fit(x, g, inst.init_modes, lam=inst.lam)


def same(a, b):
    assert b["status"] == 0, b["status"]
    # the served form always runs the separate final pass; everything else is identical
    ra = {k: v for k, v in a["result"].items() if k != "final_passes"}
    rb = {k: v for k, v in b["result"].items() if k != "final_passes"}
    assert ra == rb, (a["result"], b["result"])
    assert np.array_equal(a["modes"], b["modes"])
    assert a["z"].equal(b["z"]) and a["labels"].equal(b["labels"])


def test_fit_batched_matches_solo(slk, torch):
    insts = small_stream()
    probs = [dict(x=to_dev(torch, i.X, torch.float32), init_modes=i.init_modes, lam=i.lam, k=i.K) for i in insts]
    outs = slk.fit_batched(probs, max_jobs=16, passes_per_step=2)
    for inst, out in zip(insts, outs):
        same(solo(slk, torch, inst), out)


@pytest.mark.parametrize("max_jobs,passes", [(3, 1), (4, 3)])
def test_server_continuous_admission(slk, torch, max_jobs, passes):
    """Jobs arrive while others run (a few per step), the slot count forces admission as
    slots free up, and every result equals the job's solo fit."""
    insts = small_stream(n_jobs=9, seed=11)
    xs = [to_dev(torch, i.X, torch.float32) for i in insts]
    sv = slk.Server(max_jobs=max_jobs, passes_per_step=passes)
    tickets, outs, seen_active = {}, {}, []
    nxt, steps = 0, 0
    while len(outs) < len(insts):
        if nxt < len(insts) and steps % 2 == 0:
            for _ in range(2):
                if nxt < len(insts):
                    i = insts[nxt]
                    tickets[sv.submit(xs[nxt], i.init_modes, lam=i.lam, k=i.K)] = nxt
                    nxt += 1
        outs.update(sv.step())
        seen_active.append(sv.active)
        steps += 1
        assert steps < 5000
    sv.close()
    assert max(seen_active) == max_jobs            # the slots filled up
    assert sum(1 for a in seen_active if a > 1) > 3  # jobs overlapped on the device
    for t, k in tickets.items():
        same(solo(slk, torch, insts[k]), outs[t])


def test_server_memory_budget_serialises(slk, torch):
    insts = small_stream(n_jobs=4, seed=13)
    sv = slk.Server(max_jobs=8, passes_per_step=2, memory_budget=1)
    xs = [to_dev(torch, i.X, torch.float32) for i in insts]
    tickets = {sv.submit(x, i.init_modes, lam=i.lam, k=i.K): j for j, (x, i) in enumerate(zip(xs, insts))}
    outs = {}
    while len(outs) < len(insts):
        outs.update(sv.step())
        assert sv.active <= 1                       # a 1-byte budget admits one job at a time
    sv.close()
    for t, k in tickets.items():
        same(solo(slk, torch, insts[k]), outs[t])


def test_served_job_against_oracle(slk, torch):
    inst = gen.gaussian_mixture(n=900, d=6, L=4, K=8, seed=31, name="served")
    idx, d2 = orc.knn(inst.X, inst.K, block=256)
    rp, ci = orc.symmetrize(idx, inst.N)
    s2 = orc.sigma2_from_knn(d2)
    x = to_dev(torch, inst.X, torch.float32)
    out = slk.fit_batched([dict(x=x, init_modes=inst.init_modes, lam=inst.lam, k=inst.K, method="exact")])[0]
    r = out["result"]
    assert out["status"] == 0 and r["converged"] == 1
    ref = orc.assign(inst.X, rp, ci, out["modes"], s2, inst.lam, n_inner=r["inner_iters_last"])
    res = dict(out, modes_next=out["modes"])
    check_outer(res, ref, inst, rp, ci, inst.lam, trajectory_ztol(ref, rp, ci, inst.lam))


def test_server_rejects_bad_jobs(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    inst = gen.gaussian_mixture(n=300, d=4, L=3, K=5, seed=3)
    x = to_dev(torch, inst.X, torch.float32)
    sv = slk.Server(max_jobs=2)
    with pytest.raises(SlkError) as e:
        sv.submit(x, np.arange(65), k=5)            # L > 64: not served
    assert e.value.status == 5
    with pytest.raises(SlkError) as e:
        sv.submit(x, [1, 1, 2], k=5)                # duplicate modes
    assert e.value.status == 1
    with pytest.raises(SlkError):
        sv.submit(x, [0, 1, 400], k=5)              # out of range
    with pytest.raises(SlkError):
        sv.submit(x, [0, 1, 2], k=300)              # k >= n
    t = sv.submit(x, inst.init_modes, k=5)          # the server still works
    outs = {}
    while not outs:
        outs = sv.step()
    assert outs[t]["status"] == 0
    sv.close()


def test_build_knn_batched_identical_to_single_builds(slk, torch):
    """slk_build_knn_batched: the exact searches of several problems share one launch; every graph
    equals its own slk_build_knn (lists, FP64 distances, CSR, sigma^2), also with the locality
    order, bf16 points and a problem large enough for the MFMA path in the same call."""
    probs = []
    rng = np.random.default_rng(3)
    for j, (n, d, k) in enumerate([(300, 8, 5), (1777, 16, 10), (64, 3, 7), (2500, 40, 10), (999, 12, 6)]):
        inst = gen.gaussian_mixture(n=n, d=d, L=3, K=k, seed=40 + j)
        probs.append(dict(x=to_dev(torch, inst.X, torch.float32), k=k, reorder=bool(j % 2),
                          prec="bf16" if j == 4 else "fp32"))
    big = gen.gaussian_mixture(n=12000, d=64, L=4, K=10, seed=49)
    probs.append(dict(x=to_dev(torch, big.X, torch.float32), k=10, method="auto"))
    graphs = slk.Graph.build_knn_batched(probs)
    for pr, g in zip(probs, graphs):
        ref = slk.Graph.build_knn(pr["x"], k=pr["k"], reorder=pr.get("reorder", False), prec=pr.get("prec", "fp32"),
                                  method=pr.get("method", "auto"))
        a, b = g.export(), ref.export()
        for key in ("knn_idx", "knn_d2", "row_ptr", "col_idx", "perm"):
            assert torch.equal(a[key], b[key]), key
        assert g.info() == ref.info()
        g.close()
        ref.close()


@pytest.mark.parametrize("replay", [True, False])
def test_server_graph_replay_and_grouped_builds(slk, torch, replay):
    """Twelve small jobs submitted together on a server created on a (capturable) torch stream:
    their graphs are built in shared exact-search launches, and with graph replay the steps whose
    launch sequence repeats run from captured HIP graphs (replayed many times, with the server's
    own copies and synchronisations in between); every result equals the job's solo fit either
    way.  A server on the null stream launches directly (the null stream cannot be captured)."""
    insts = [gen.gaussian_mixture(n=1500, d=16, L=6, K=10, seed=60 + j) for j in range(12)]
    xs = [to_dev(torch, i.X, torch.float32) for i in insts]
    kw = dict(fixed_inner=24, max_outer=2)   # the jobs step in lock-step through 12 equal inner steps
    torch.cuda.synchronize()
    with torch.cuda.stream(torch.cuda.Stream()):   # replay needs a stream that can be captured
        sv = slk.Server(max_jobs=16, passes_per_step=2, builders=1, graph_replay=replay)
        tickets = {sv.submit(x, i.init_modes, lam=i.lam, k=i.K, **kw): j for j, (x, i) in enumerate(zip(xs, insts))}
        outs = {}
        while len(outs) < len(insts):
            outs.update(sv.step())
        st = sv.stats()
        sv.close()
    torch.cuda.synchronize()
    assert st["grouped_builds"] >= 1, st
    if replay:
        assert st["graph_captures"] >= 1 and st["graph_launches"] >= st["graph_captures"] + 10, st
    else:
        assert st["graph_launches"] == 0
    for t, k in tickets.items():
        x = xs[k]
        g = slk.Graph.build_knn(x, k=insts[k].K)
        same(slk.fit(x, g, insts[k].init_modes, lam=insts[k].lam, **kw), outs[t])
