"""Autotuner of the level-test launch shapes.

The level kernels take their work in items of consecutive ranks of one
edge; how many ranks a wave takes per item, how fast the rank windows
grow, how many items an edge gets in the first window, how many
workgroups may share a CU and how long a conditioning prefix the
shared-prefix kernels factor once change only the speed, never the
results.  This
tool measures candidate values on seeded synthetic workloads, keeps per
level the value with the smallest device time of that level's tests
(coordinate descent, one field at a time), and writes the table the Python
binding loads into every context (``tuning_gfx950.json`` next to the
library).

    python -m paper_2109_04626_amd.autotune [--out PATH] [--reps 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))

CANDIDATES = {
    "shared_prefix_depth": [2, 3],
    "shared_ranks_per_wave": [1024, 2048, 4096, 8192, 16384, 32768, 65536],
    "test_ranks_per_wave": [256, 512, 2048, 8192],
    "window_growth": [4, 8, 16],
    "first_window_items": [1, 2],
    "max_blocks_per_cu": [0, 4],
}


def _workloads(fpc, ctx):
    """Callables returning one result (or a list of results) each."""
    import torch

    import semdata

    runs = []
    for name, seed in (("er_p1000_n10000_d4", 0), ("ba_p1000_n10000_m2", 2000), ("er_p95_n5000_d12", 0)):
        X, _, cfg = semdata.workload(name, seed)
        Xd = torch.from_numpy(X).cuda()
        runs.append((f"{name} seed {seed}",
                     lambda Xd=Xd, cfg=cfg: [fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"],
                                                              precision=fpc.FPC_PREC_MIXED)]))
    base, boots, datas, cfg = semdata.batched_workload(n_boot=16, n_data=4)
    bd = torch.from_numpy(base).cuda()
    inst = [(bd, torch.from_numpy(r).cuda()) for r in boots] + [(torch.from_numpy(d).cuda(), None) for d in datas]
    runs.append(("16 bootstraps + 4 data sets (batched)",
                 lambda: fpc.fpc_skeleton_batch(ctx, inst, alpha=cfg["alpha"], max_level=cfg["max_level"],
                                                precision=fpc.FPC_PREC_MIXED)))
    return runs


def _level_times(results) -> dict:
    """Device time of each level's tests (the first level excluded); in a
    batch every instance reports the shared launches, so take one each."""
    t = {}
    seen = set()
    for r in results:
        for x in r["levels"][1:]:
            key = (x["level"], round(x["kernel_ms"], 6), round(x["level_ms"], 6))
            if key in seen:
                continue
            seen.add(key)
            t[x["level"]] = t.get(x["level"], 0.0) + x["kernel_ms"]
    return t


def measure(fpc, ctx, runs, reps: int) -> dict:
    """Per-level device ms summed over the workloads (min over reps)."""
    tot = {}
    for _, fn in runs:
        best = None
        for _ in range(reps):
            lt = _level_times(fn())
            best = lt if best is None else {l: min(best.get(l, 1e30), v) for l, v in lt.items()}
        for l, v in best.items():
            tot[l] = tot.get(l, 0.0) + v
    return tot


def tune(reps: int = 2, verbose: bool = True) -> dict:
    import torch

    import paper_2109_04626_amd as fpc

    ctx = fpc.Context(0, tuning="default")
    runs = _workloads(fpc, ctx)
    for _, fn in runs:  # warm every kernel and buffer
        fn()
    torch.cuda.synchronize()
    table = fpc.fpc_get_tuning(ctx)
    L = fpc.FPC_TUNE_LEVELS
    base = measure(fpc, ctx, runs, reps)
    if verbose:
        print(f"[tune] defaults: {sum(base.values()):.2f} ms {sorted(base.items())}", flush=True)
    log = {"defaults": base}
    for field, cands in CANDIDATES.items():
        per_val = {}
        for v in cands:
            trial = {k: list(x) for k, x in table.items()}
            trial[field] = [v] * L
            if field == "shared_prefix_depth":  # the triple kernel needs l >= 3
                trial[field] = [min(v, 2) if l < 3 else v for l in range(L)]
            fpc.fpc_set_tuning(ctx, trial)
            per_val[v] = measure(fpc, ctx, runs, reps)
            if verbose:
                print(f"[tune] {field}={v}: {sum(per_val[v].values()):.2f} ms", flush=True)
        levels = sorted({l for m in per_val.values() for l in m})
        for l in levels:
            best = min(cands, key=lambda v: per_val[v].get(l, 1e30))
            if field == "shared_prefix_depth" and l < 3:
                best = 2
            table[field][min(l, L - 1)] = best
        fpc.fpc_set_tuning(ctx, table)
        log[field] = {str(v): per_val[v] for v in cands}
    final = measure(fpc, ctx, runs, reps)
    if verbose:
        print(f"[tune] tuned: {sum(final.values()):.2f} ms {sorted(final.items())}", flush=True)
    out = {
        "device": torch.cuda.get_device_name(0),
        "workloads": [name for name, _ in runs],
        "objective": "device ms of each level's test launches, summed over the workloads (min of reps)",
        "default_ms": sum(base.values()),
        "tuned_ms": sum(final.values()),
        "tuning": table,
        "search": log,
    }
    ctx.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning_gfx950.json"))
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    t0 = time.time()
    out = tune(args.reps)
    out["seconds"] = time.time() - t0
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("default_ms", "tuned_ms", "seconds")}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
