"""Benchmark of the SLK-BO iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large-1m]

One step = one SLK-BO fit (Algorithm 1: unary term, inner z-updates until the bound
settles, labels, byproduct modes, energy with its FP64 recheck, outer loop until the modes
stop changing) on the resident points and the resident kNN graph.  The graph itself
(MFMA kNN + FP64 re-rank, symmetrisation, sigma^2) is built once before the timed steps
and reported in the "knn" object with its MFMA roofline.

`value` is the whole-fit algorithmic throughput: the bytes every kernel of the fit must
move by its definition (counted per launch, see ALG_BYTES below) divided by the fit's wall
time.  `roofline` is for the dominant kernel, the fused z-update (iter_kernel), timed live
with HIP events on its launch stream over the timed steps.  `cpu_baseline` times the FP64
oracle's z-update on the host over a bounded number of passes of the same workload.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense bf16 MFMA
METRIC = "SLK-iteration GB/s (% HBM peak) at N=1M; batched solves/s + p99 latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------- bytes
def bytes_iter(N, nnz, L):
    """One z-update (iter_kernel): row_ptr, col_idx, A and Z^i read once, Z^{i+1} written."""
    return 4 * (N + 1) + 4 * nnz + 12 * N * L


def bytes_final(N, nnz, L):
    """Final pass: as a z-update, plus int32 labels in two orders."""
    return bytes_iter(N, nnz, L) + 8 * N


def bytes_unary(N, D, L):
    """Unary term: X read, A and Z^0 written."""
    return 4 * N * D + 8 * N * L


def bytes_energy(N, nnz, D, fp64):
    """Energy: row_ptr, col_idx, labels, A[p, l_p]; X as well for the FP64 recheck."""
    return 4 * (N + 1) + 4 * nnz + 8 * N + (4 * N * D if fp64 else 0)


def fit_bytes(N, D, L, nnz, inner_total, outer):
    """Every launch of a fit: per outer iteration the unary term, the z-updates, the final pass
    and the energy; once per fit the FP64 energy recheck."""
    return (inner_total * bytes_iter(N, nnz, L)
            + outer * (bytes_final(N, nnz, L) + bytes_unary(N, D, L) + bytes_energy(N, nnz, D, False))
            + bytes_energy(N, nnz, D, True))


def traffic_entry(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(f"{kernel}:{workload}")
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_1810_13044_amd", "csrc", ent["source"])
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return ent["bytes_per_launch"] if h == ent["source_sha"] else None


def cpu_baseline(graph, A, Z0, lam, N, nnz, L, budget_s=20.0):
    """The FP64 oracle's z-update (CSR x Z, softmax, bound) on the host, bounded passes."""
    from oracle import slk as orc
    ex = graph.export()
    rp = ex["row_ptr"].cpu().numpy()
    ci = ex["col_idx"].cpu().numpy()
    W = orc.csr_matrix(rp, ci, N)
    A64 = A.cpu().numpy().astype(np.float64)
    Z = Z0.cpu().numpy().astype(np.float64)
    times = []
    t_all = time.perf_counter()
    while len(times) < 2 or (time.perf_counter() - t_all < budget_s and len(times) < 10):
        t0 = time.perf_counter()
        B = orc.pairwise(W, Z)
        S = A64 + lam * B
        orc.relaxed_bound(Z, A64, B, lam)
        Z = orc.softmax_rows(S)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": round(bytes_iter(N, nnz, L) / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} FP64 oracle z-updates (SciPy CSR x dense Z, NumPy softmax and bound, "
                      f"single thread) over the full N={N} graph; median {t:.3f} s per pass; "
                      f"host has {os.cpu_count()} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large-1m")
    ap.add_argument("--n", type=int, default=0, help="override N (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reorder", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_1810_13044_amd as slk

    torch.cuda.set_device(0)
    kw = {"n": args.n} if args.n else {}
    t0 = time.perf_counter()
    inst = gen.make(args.workload, **kw)
    N, D, L, K = inst.N, inst.D, inst.L, inst.K
    log(f"[bench] workload {args.workload}: N={N} D={D} L={L} K={K} generated in {time.perf_counter() - t0:.1f}s")
    x = torch.from_numpy(inst.X).to("cuda")
    torch.cuda.synchronize()

    # ---- graph (a1-a3), once
    slk.timing_enable(True)
    t0 = time.perf_counter()
    g = slk.Graph.build_knn(x, k=K, method="mfma", reorder=bool(args.reorder))
    torch.cuda.synchronize()
    knn_s = time.perf_counter() - t0
    info = g.info()
    n_cand, cand_ms = slk.timing_read("cand_kernel")
    knn_flops = 2.0 * N * N * D
    log(f"[bench] kNN graph in {knn_s:.2f}s (cand_kernel {cand_ms:.1f} ms): nnz={info['nnz']} "
        f"sigma2={info['sigma2']:.4f} certified={info['rows_certified']} fallback={info['rows_fallback']}")
    nnz = info["nnz"]

    if args.copy_mib:
        buf = torch.empty(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        buf2 = buf.clone()
        torch.cuda.synchronize()
        del buf, buf2

    # ---- fit (a4-a8): warmup, then timed steps
    lam = inst.lam
    for i in range(args.warmup):
        r = slk.fit(x, g, inst.init_modes, lam=lam)
        log(f"[bench] warmup {i}: {r['result']}")
    torch.cuda.synchronize()
    slk.timing_enable(True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(slk.fit(x, g, inst.init_modes, lam=lam)["result"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_iter, iter_ms = slk.timing_read("iter_kernel")
    kern = {k: slk.timing_read(k) for k in ("unary_kernel", "iter_kernel", "iter_kernel_after_stop", "final_kernel",
                                            "energy_kernel")}
    slk.timing_enable(False)
    r0 = results[0]
    assert all(r == r0 for r in results), "fit results differ between steps"
    log(f"[bench] fit: {r0}")
    if n_iter != r0["inner_iters_total"] * args.steps:
        log(f"[bench] warning: {n_iter} timed z-updates for {r0['inner_iters_total'] * args.steps} passes")
    ms_step = wall / args.steps * 1e3
    total_bytes = fit_bytes(N, D, L, nnz, r0["inner_iters_total"], r0["outer_iters"])
    value = total_bytes / (ms_step / 1e3) / 1e9
    iter_avg_ms = iter_ms / max(n_iter, 1)
    achieved = bytes_iter(N, nnz, L) / (iter_avg_ms / 1e3) / 1e9
    log(f"[bench] {args.steps} fits in {wall:.3f}s ({ms_step:.2f} ms/fit); iter_kernel avg {iter_avg_ms * 1e3:.1f} us "
        f"over {n_iter} launches -> {achieved:.0f} GB/s; kernels {kern}")

    cpu = None
    if not args.no_cpu_baseline:
        a, z0 = slk.unary(x, inst.init_modes, info["sigma2"])
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(g, a, z0, lam, N, nnz, L)
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: N={N} D={D} L={L} k_n={K} lambda={lam}, seeded synthetic "
                        f"(anisotropic Gaussian mixture); one step = one SLK-BO fit on the resident kNN graph",
            "N": N, "D": D, "L": L, "k": K, "nnz": nnz, "lambda": lam, "reorder": bool(args.reorder),
            "outer_iters": r0["outer_iters"], "inner_iters_total": r0["inner_iters_total"],
        },
        "roofline": {
            "kernel": "iter_kernel (fused CSR SpMM + row softmax + bound partials)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_entry("iter_kernel", args.workload),
            "alg_bytes_per_launch": bytes_iter(N, nnz, L),
            "avg_launch_us": round(iter_avg_ms * 1e3, 2),
            "launches": n_iter,
        },
        "cpu_baseline": cpu,
        "knn": {
            "method": "bf16x3 MFMA Gram candidates + FP64 re-rank + certificate",
            "build_s": round(knn_s, 3),
            "cand_kernel_ms": round(cand_ms, 2),
            "alg_tflops": round(knn_flops / (cand_ms / 1e3) / 1e12, 1) if cand_ms else None,
            "mfma_tflops_issued": round(3 * knn_flops / (cand_ms / 1e3) / 1e12, 1) if cand_ms else None,
            "peak_tflops": BF16_PEAK_TFLOPS,
            "frac_issued": round(3 * knn_flops / (cand_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS, 4) if cand_ms else None,
            "rows_certified": info["rows_certified"],
            "rows_fallback": info["rows_fallback"],
        },
        "fit": {k: r0[k] for k in ("energy", "energy_fp64", "bound", "cut", "n_distinct_modes", "converged")},
        "kernels_ms": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in kern.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
