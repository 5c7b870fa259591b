"""Launch tuning (fpc_set_tuning) changes speed only: the skeleton and the
separating sets are the same under extreme launch shapes, and the shipped
autotuned table loads and validates (GPU only)."""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import oracle
import semdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fpc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_04626_amd as m

    return m


EXTREME = {
    "test_ranks_per_wave": [64] * 17,
    "shared_ranks_per_wave": [100] * 17,
    "window_growth": [2] * 17,
    "first_window_items": [3] * 17,
    "max_blocks_per_cu": [1] * 17,
    "shared_prefix_depth": [2] * 17,  # the pair kernel at every level
}


@pytest.mark.parametrize("prec", [0, 1])
def test_results_do_not_depend_on_launch_shapes(fpc, prec):
    p, n = 90, 3000
    _say(f"[tuning] p={p} n={n} prec={prec}")
    sem = semdata.make_sem(p, 51, degree=5.0)
    X = semdata.sample(sem, n, 51)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=0.01, max_level=6)
    Xd = torch.from_numpy(X).cuda()
    with fpc.Context(0, tuning="default") as a, fpc.Context(0, tuning=EXTREME) as b:
        assert fpc.fpc_get_tuning(b)["window_growth"] == [2] * 17
        ra = fpc.fpc_skeleton(a, Xd, alpha=0.01, max_level=6, precision=prec)
        rb = fpc.fpc_skeleton(b, Xd, alpha=0.01, max_level=6, precision=prec)
        for r in (ra, rb):
            assert np.array_equal(r["adj"], ref["adj"])
            assert np.array_equal(r["sep_level"], ref["sep_level"])
        assert ra["sepsets"] == rb["sepsets"]
        if prec == 0:
            assert rb["sepsets"] == ref["sepsets"]
        # batch under the extreme shapes too
        got = fpc.fpc_skeleton_batch(b, [(Xd, None), (Xd[:1500], None)], alpha=0.01, max_level=6, precision=prec)
        assert got[0]["sepsets"] == ra["sepsets"]
        one = fpc.fpc_skeleton(a, Xd[:1500].contiguous(), alpha=0.01, max_level=6, precision=prec)
        assert got[1]["sepsets"] == one["sepsets"] and np.array_equal(got[1]["adj"], one["adj"])


def test_tuning_rejects_out_of_range(fpc):
    with fpc.Context(0, tuning="default") as c:
        before = fpc.fpc_get_tuning(c)
        for field, bad in (("test_ranks_per_wave", 10), ("window_growth", 1), ("first_window_items", 0),
                           ("max_blocks_per_cu", -1), ("shared_prefix_depth", 3)):
            t = {field: [bad] * 17}
            with pytest.raises(fpc.FastPCError):
                fpc.fpc_set_tuning(c, t)
        assert fpc.fpc_get_tuning(c) == before
        fpc.fpc_set_tuning(c, None)
        assert fpc.fpc_get_tuning(c) == before


def test_shipped_table_loads(fpc):
    if not os.path.exists(fpc.TUNING_TABLE):
        pytest.skip("no autotuned table shipped")
    with open(fpc.TUNING_TABLE) as f:
        tab = json.load(f)["tuning"]
    with fpc.Context(0) as c:
        assert fpc.fpc_get_tuning(c) == {k: list(v) for k, v in tab.items()}


def test_recheck_queue_sizes_do_not_change_results(fpc):
    """A tiny recheck queue overflows: the level runs again with a 4x queue
    (still mixed), and past the cap in FP64; the results stay the same."""
    p, n = 90, 3000
    _say(f"[recheck queue] p={p} n={n}")
    sem = semdata.make_sem(p, 52, degree=5.0)
    X = semdata.sample(sem, n, 52)
    ref = oracle.skeleton(oracle.corr(X), n, alpha=0.01, max_level=6)
    Xd = torch.from_numpy(X).cuda()
    kw = dict(alpha=0.01, max_level=6, precision=fpc.FPC_PREC_MIXED, recheck_margin=3.0)  # a wide band
    with fpc.Context(0) as c:
        base = fpc.fpc_skeleton(c, Xd, **kw)
        assert sum(x["tests_rechecked"] for x in base["levels"]) > 200
        assert np.array_equal(base["adj"], ref["adj"])
        for init, cap in ((16, 1 << 20), (16, 64)):  # growth in the mixed form; the cap, then FP64
            fpc.fpc_set_recheck_queue(c, init, cap)
            got = fpc.fpc_skeleton(c, Xd, **kw)
            assert got["total_tests"] > base["total_tests"]  # the overflowed launches ran too
            # ... and their launches and device time are counted with them
            lb = {x["level"]: x for x in base["levels"]}
            rerun = [x for x in got["levels"] if x["level"] in lb and x["tests_executed"] > lb[x["level"]]["tests_executed"]]
            assert rerun and all(x["test_launches"] > lb[x["level"]]["test_launches"] for x in rerun)
            assert np.array_equal(got["adj"], ref["adj"])
            assert np.array_equal(got["sep_level"], base["sep_level"])
            assert got["sepsets"] == base["sepsets"]
        for bad in ((0, 10), (10, 5), (1, 1 << 40)):
            with pytest.raises(fpc.FastPCError):
                fpc.fpc_set_recheck_queue(c, *bad)
