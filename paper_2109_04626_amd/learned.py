"""Learned order of the candidate lists: data collection, training and
evaluation, all through the C ABI (the network's passes are the library's
HIP kernels).

The plain method (lexicographic order over candidates sorted by id) runs
on seeded scale-free SEM data with FPC_FLAG_LOG_FEATURES; every candidate
of every edge deleted after the first level becomes one row (features,
label = "in the separating set that was found").  The network learns to
score candidates; with FPC_ORDER_LEARNED each level enumerates subsets
over the list sorted by decreasing score, so subsets of likely separators
are tested first.  The skeleton cannot change (stable schedule); only the
number of tests before each edge's first separating set does.

    python -m paper_2109_04626_amd.learned train  --out model.npy
    python -m paper_2109_04626_amd.learned eval   --model model.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "ranker_ba.npy")

# training and evaluation workload: Barabasi-Albert DAGs (m = 2), n = 10000,
# alpha = 0.01, levels after the first capped at 3; training graphs have p
# uniform in [200, 1000], evaluation graphs p = 1000
WORKLOAD = "ba_p1000_n10000_m2"
TRAIN_SEEDS = range(1000, 1200)
EVAL_SEEDS = range(2000, 2020)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the flat layout of fpc_mlp_params."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((3, 64)) * np.sqrt(2.0 / 3)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = rng.standard_normal(64) * np.sqrt(1.0 / 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3, [0.0]]).astype(np.float32)


def _data(seed: int, **over):
    import semdata

    X, sem, cfg = semdata.workload(WORKLOAD, seed, **over)
    return X, cfg


def collect(ctx, seeds, p_lo: int = 200, p_hi: int = 1000, verbose: bool = True):
    """Feature/label rows from plain runs on seeded BA graphs."""
    import torch

    import paper_2109_04626_amd as fpc

    xs, ys = [], []
    for s in seeds:
        p = int(np.random.default_rng([s, 7]).integers(p_lo, p_hi + 1))
        X, cfg = _data(s, p=p)
        res = fpc.fpc_skeleton(ctx, torch.from_numpy(X).cuda(), alpha=cfg["alpha"], max_level=cfg["max_level"],
                               precision=fpc.FPC_PREC_MIXED, flags=fpc.FPC_FLAG_LOG_FEATURES)
        if res["log"] is not None:
            xs.append(res["log"]["x"])
            ys.append(res["log"]["y"].astype(np.float32))
        if verbose:
            rows = 0 if res["log"] is None else len(res["log"]["y"])
            print(f"[collect] seed {s} p={p}: {rows} rows, {res['total_tests']} tests", flush=True)
    return np.concatenate(xs), np.concatenate(ys)


def train(ctx, X: np.ndarray, y: np.ndarray, epochs: int = 10, batch: int = 65536, lr: float = 3e-3,
          seed: int = 0, verbose: bool = True):
    """Adam on the mean binary cross-entropy, minibatches on the GPU."""
    import torch

    import paper_2109_04626_amd as fpc

    model = fpc.fpc_mlp_init(ctx, init_params(seed))
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(y))).cuda()
        losses = []
        for b0 in range(0, len(y), batch):
            idx = perm[b0:b0 + batch]
            losses.append(fpc.fpc_mlp_train_step(ctx, Xd[idx].contiguous(), yd[idx].contiguous(), model, lr))
        hist.append(float(np.mean(losses)))
        if verbose:
            print(f"[train] epoch {ep}: loss {hist[-1]:.5f}", flush=True)
    return model, hist


def evaluate(ctx, model, seeds=EVAL_SEEDS, verbose: bool = True) -> dict:
    """Lexicographic vs learned order on held-out seeds (mixed precision)."""
    import torch

    import paper_2109_04626_amd as fpc

    rows = []
    for s in seeds:
        Xh, cfg = _data(s)
        X = torch.from_numpy(Xh).cuda()

        def run(m=None):
            return fpc.fpc_skeleton(ctx, X, alpha=cfg["alpha"], max_level=cfg["max_level"],
                                    precision=fpc.FPC_PREC_MIXED, order_model=m)

        run(), run(model)  # warm
        ta, tb = [], []
        for rep in range(4):  # median time of each form; each form runs first in half of the pairs
            first_lex = rep % 2 == 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = run() if first_lex else run(model)
            t1 = time.perf_counter()
            y = run(model) if first_lex else run()
            t2 = time.perf_counter()
            a, b = (x, y) if first_lex else (y, x)
            ta.append((t1 - t0) if first_lex else (t2 - t1))
            tb.append((t2 - t1) if first_lex else (t1 - t0))
        same = bool(np.array_equal(a["adj"], b["adj"]) and np.array_equal(a["sep_level"], b["sep_level"]))
        lv_a = sum(x["tests_executed"] for x in a["levels"][1:])
        lv_b = sum(x["tests_executed"] for x in b["levels"][1:])
        rows.append(dict(seed=s, same_skeleton=same, tests_lex=lv_a, tests_learned=lv_b,
                         ms_lex=float(np.median(ta)) * 1e3, ms_learned=float(np.median(tb)) * 1e3,
                         kernel_ms_lex=sum(x["test_kernel_ms"] for x in a["levels"][1:]),
                         kernel_ms_learned=sum(x["test_kernel_ms"] for x in b["levels"][1:])))
        if verbose:
            print(f"[eval] seed {s}: tests {lv_a} -> {lv_b}, ms {rows[-1]['ms_lex']:.1f} -> "
                  f"{rows[-1]['ms_learned']:.1f}, same skeleton {same}", flush=True)
    tl = sum(r["tests_lex"] for r in rows)
    tb = sum(r["tests_learned"] for r in rows)
    return dict(rows=rows, tests_lex=tl, tests_learned=tb, test_ratio=tb / max(tl, 1),
                ms_lex=sum(r["ms_lex"] for r in rows), ms_learned=sum(r["ms_learned"] for r in rows),
                kernel_ms_lex=sum(r["kernel_ms_lex"] for r in rows),
                kernel_ms_learned=sum(r["kernel_ms_learned"] for r in rows),
                all_same=all(r["same_skeleton"] for r in rows))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--model", default=DEFAULT_MODEL)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--seeds", type=int, default=len(TRAIN_SEEDS))
    ap.add_argument("--eval-seeds", type=int, default=len(EVAL_SEEDS))
    ap.add_argument("--epochs", type=int, default=10)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2109_04626_amd as fpc

    ctx = fpc.Context(0)
    if args.cmd == "train":
        X, y = collect(ctx, list(TRAIN_SEEDS)[: args.seeds])
        print(f"[train] {len(y)} rows, {y.mean():.4f} positive", flush=True)
        model, hist = train(ctx, X, y, epochs=args.epochs)
        np.save(args.out, fpc.fpc_mlp_get(ctx, model))
        print(json.dumps({"rows": int(len(y)), "loss": hist}), flush=True)
    else:
        model = fpc.fpc_mlp_init(ctx, np.load(args.model))
        out = evaluate(ctx, model, list(EVAL_SEEDS)[: args.eval_seeds])
        print(json.dumps({k: v for k, v in out.items() if k != "rows"}), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
