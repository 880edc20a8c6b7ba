"""Autotuner of the z-update's tile shape (row batches per wave in a work-group's tile).

    python -m paper_1810_13044_amd.tune [--out paper_1810_13044_amd/csrc/tune_table.h]

Runs on the GPU.  For every lane-group class of L (1, 2, 4, 8, 16 lanes per row) and a ladder of
row counts it builds a seeded Gaussian-mixture problem with its exact kNN graph in the locality
order (64 dimensions, mixture components of about 20,000 points as in the large benchmark
workload, at most 64), times the z-update (HIP events, slk timing) at 1, 2, 4 and 8 batches per
wave, and writes
the fastest choice per size range as the C table the library compiles in (tune_table.h).  Rebuild
the library afterwards.  Every call of the library - single fits and the served form - takes its
tile shapes from that table.
"""
from __future__ import annotations

import argparse
import datetime
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CLASSES = [(1, 4), (2, 8), (4, 16), (8, 32), (16, 50)]       # (lanes per row, L measured)
SIZES = [2_000, 5_000, 12_000, 30_000, 70_000, 150_000, 400_000, 1_000_000]
STEPS = (1, 2, 4, 8)


def measure(slk, torch, x, g, modes, lam, passes=12, reps=3):
    slk.assign(x, g, modes, lam=lam, fixed_inner=passes, trace=False)
    torch.cuda.synchronize()
    slk.timing_enable(True)
    for _ in range(reps):
        slk.assign(x, g, modes, lam=lam, fixed_inner=passes, trace=False)
    torch.cuda.synchronize()
    n_it, ms = slk.timing_read("iter_kernel")
    slk.timing_enable(False)
    return ms / max(n_it, 1) * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(PKG, "csrc", "tune_table.h"))
    ap.add_argument("--sizes", default=",".join(str(v) for v in SIZES))
    args = ap.parse_args()
    import torch
    import gen
    import paper_1810_13044_amd as slk

    sizes = [int(v) for v in args.sizes.split(",")]
    best = {}          # (g, n) -> (wave_steps, {ws: us})
    for n in sizes:
        inst = gen.gaussian_mixture(n=n, d=64, L=int(min(64, max(4, n // 20_000))), K=10, seed=97)
        x = torch.from_numpy(inst.X).to("cuda")
        g = slk.Graph.build_knn(x, k=10, reorder=True)
        for gcls, L in CLASSES:
            modes = np.random.default_rng(n + L).choice(n, L, replace=False)
            t = {}
            for ws in STEPS:
                slk.tune_override(ws)
                t[ws] = measure(slk, torch, x, g, modes, 1.0)
            slk.tune_override(0)
            pick = min(STEPS, key=lambda w: t[w])
            best[(gcls, n)] = (pick, t)
            print(f"[tune] n={n} L={L} (g={gcls}): " + ", ".join(f"{w}: {t[w]:.1f} us" for w in STEPS)
                  + f" -> {pick}", flush=True)
        g.close()
        del x
    dev = torch.cuda.get_device_name(0)
    stamp = datetime.date.today().isoformat()
    lines = []
    for gcls, _L in CLASSES:
        for i, n in enumerate(sizes):
            n_max = "INT64_MAX" if i + 1 == len(sizes) else str(int(np.sqrt(n * sizes[i + 1])))
            lines.append(f"    {{{gcls}, {n_max}, {best[(gcls, n)][0]}}},")
    meas = "\n".join(f"//   g={gc:2d} n={n:>9}: " + ", ".join(f"{w}: {t[w]:.1f}" for w in STEPS)
                     for (gc, n), (_p, t) in sorted(best.items()))
    text = f"""// Tile shapes of the z-update and final pass (row batches per wave in a work-group's tile), by
// lane-group class g (lanes per row: 1, 2, 4, 8, 16 for L <= 4, 8, 16, 32, 64) and row count:
// the first entry of the class with n <= n_max applies.  Written by paper_1810_13044_amd/tune.py.
// Measured z-update time per launch in microseconds at 1, 2, 4, 8 batches per wave:
{meas}
#pragma once
#include <stdint.h>

namespace slk {{
struct TuneZEntry {{
  int32_t g;
  int64_t n_max;
  int32_t wave_steps;
}};
constexpr TuneZEntry kTuneZ[] = {{
{chr(10).join(lines)}
}};
constexpr const char* kTuneSource = "tune.py on {dev} ({stamp})";
}}  // namespace slk
"""
    with open(args.out, "w") as f:
        f.write(text)
    print(f"[tune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
