"""Write the oracle's results for the full-size workloads used by the GPU
parity tests.  Calls only oracle/ and the input generators.

    python tests/golden/make_goldens.py [name ...]

Each file <workload>_seed<k>.npz (batched_data<d>_seed0.npz for data set d
of the many-instance workload) holds the FP64 oracle's skeleton edge
list, the level at which each deleted pair went, the separating sets of
LIST kind (ALL_BUT kind = every other variable), per-level counts and the
smallest |z - q| seen (tie monitor).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import semdata  # noqa: E402

GOLDENS = [("er_p1000_n10000_d4", 0), ("er_p95_n5000_d12", 0), ("er_p95_n20000_d8_paper", 0)]
# independent data sets of the many-instance workload (semdata.batched_workload,
# full size): d = 2, 7, 12 have p = 120, 778, 1939
BATCHED_GOLDENS = [2, 7, 12]


def batched_data(d: int):
    """Data set d of the many-instance workload and its configuration."""
    _, _, datas, cfg = semdata.batched_workload(n_boot=0, n_data=d + 1)
    X = datas[d]
    return X, dict(p=X.shape[1], n=cfg["n"], alpha=cfg["alpha"], max_level=cfg["max_level"])


def make(name: str, seed: int) -> str:
    if name.startswith("batched_data"):
        X, cfg = batched_data(int(name[len("batched_data"):]))
    else:
        X, sem, cfg = semdata.workload(name, seed)
    t0 = time.time()
    C = oracle.corr(X.astype(np.float64))
    res = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"], max_level=cfg["max_level"])
    p = cfg["p"]
    iu, ju = np.nonzero(np.triu(res["adj"], 1))
    keys = sorted(res["sepsets"])
    sep_pairs = np.array(keys, dtype=np.int32).reshape(-1, 2)
    sep_nodes = np.array([res["sepsets"][k] for k in keys], dtype=np.int32).reshape(len(keys), -1) \
        if keys and len({len(v) for v in res["sepsets"].values()}) == 1 else None
    flat = np.concatenate([np.array(res["sepsets"][k], np.int32) for k in keys]) if keys else np.zeros(0, np.int32)
    off = np.cumsum([0] + [len(res["sepsets"][k]) for k in keys]).astype(np.int64)
    out = os.path.join(HERE, f"{name}_seed{seed}.npz")
    np.savez_compressed(out, edges=np.stack([iu, ju], 1).astype(np.int32),
                        sep_level=res["sep_level"].astype(np.int16), sep_kind=res["sep_kind"],
                        sep_pairs=sep_pairs, sep_off=off, sep_flat=flat,
                        levels=res["levels"], total_tests=res["total_tests"],
                        min_margin=res["min_margin"], q=res["q"], p=p, n=cfg["n"],
                        max_level=cfg["max_level"], alpha=cfg["alpha"])
    del sep_nodes
    print(f"{out}: {len(iu)} edges, {res['total_tests']} tests, min margin {res['min_margin']:.3e}, "
          f"{time.time() - t0:.1f} s", flush=True)
    return out


def load(name: str, seed: int) -> dict:
    """Golden results as a dict shaped like oracle.skeleton's."""
    z = np.load(os.path.join(HERE, f"{name}_seed{seed}.npz"), allow_pickle=False)
    p = int(z["p"])
    adj = np.zeros((p, p), np.uint8)
    e = z["edges"]
    adj[e[:, 0], e[:, 1]] = 1
    adj[e[:, 1], e[:, 0]] = 1
    sepsets = {}
    pairs, flat, off = z["sep_pairs"], z["sep_flat"], z["sep_off"]  # each member read (decompressed) once
    for k, (i, j) in enumerate(pairs.tolist()):
        sepsets[(i, j)] = flat[off[k]:off[k + 1]].tolist()
    return dict(adj=adj, sep_level=z["sep_level"].astype(np.int32), sep_kind=z["sep_kind"], sepsets=sepsets,
                levels=z["levels"], total_tests=int(z["total_tests"]), min_margin=float(z["min_margin"]),
                q=float(z["q"]), p=p, n=int(z["n"]), max_level=int(z["max_level"]), alpha=float(z["alpha"]))


if __name__ == "__main__":
    want = sys.argv[1:]
    for name, seed in GOLDENS + [(f"batched_data{d}", 0) for d in BATCHED_GOLDENS]:
        if not want or name in want:
            make(name, seed)
