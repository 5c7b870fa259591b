"""Checkpoint and resume at level boundaries (fpc_params.stop_after_levels,
fpc_params.resume), through the C ABI (GPU only).

Under the stable schedule the graph and separating sets at a level end fix
every later level, so a run stopped after k levels and resumed from its
state must end as the uninterrupted run: skeleton, separating sets and the
per-level rows (level, largest set, eligible edges, possible and required
tests, deletions).  Checked for every k in both schedules and precisions,
with the learned order, across a file round trip, and across the boundary
between the library and the oracle (either one stops, the other resumes).
Also the error paths: a checkpoint of another p, feature logging with
resume, batch calls, and the allocation-failure hook.
"""
from __future__ import annotations

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


@pytest.fixture(scope="module")
def ctx(fpc):
    c = fpc.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rows(res):
    return [(x["level"], x["max_cand"], x["edges_eligible"], x["tests_possible"], x["deleted"], x["tests_required"])
            for x in res["levels"]]


def same(a, b, tag):
    assert np.array_equal(a["adj"], b["adj"]), f"{tag}: skeletons differ"
    assert np.array_equal(a["sep_level"], b["sep_level"]), f"{tag}: separating-set levels differ"
    assert np.array_equal(a["sep_kind"], b["sep_kind"]), f"{tag}: kinds differ"
    assert a["sepsets"] == b["sepsets"], f"{tag}: separating sets differ"
    assert rows(a) == rows(b), f"{tag}: levels differ"
    assert a["next_level"] == b["next_level"] == -1


def data(p=40, seed=15, degree=5.0, n=2000):
    sem = semdata.make_sem(p, seed, degree=degree)
    return semdata.sample(sem, n, seed)


@pytest.mark.parametrize("schedule,prec,max_level", [(0, 0, -1), (0, 1, 4), (1, 0, -1), (1, 1, 3)],
                         ids=["reverse-fp64", "reverse-mixed-cap4", "forward-fp64", "forward-mixed-cap3"])
def test_stop_and_resume_at_every_boundary(fpc, ctx, schedule, prec, max_level):
    X = data()
    Xd = dev(X)
    kw = dict(alpha=0.01, max_level=max_level, precision=prec, schedule=schedule)
    full = fpc.fpc_skeleton(ctx, Xd, **kw)
    nlev = len(full["levels"])
    _say(f"[resume] schedule={schedule} prec={prec} cap={max_level}: levels {[x['level'] for x in full['levels']]}")
    assert nlev >= 3
    for k in range(1, nlev + 1):
        part = fpc.fpc_skeleton(ctx, Xd, stop_after_levels=k, **kw)
        assert len(part["levels"]) == k
        assert rows(part) == rows(full)[:k]
        assert np.all(part["adj"] >= full["adj"])  # deletions only accumulate
        assert part["next_level"] == (full["levels"][k]["level"] if k < nlev else -1)
        res = fpc.fpc_skeleton(ctx, Xd, resume=part, **kw)
        same(res, full, f"resume after {k} levels")
        if part["next_level"] >= 0:  # one level at a time from there
            step = fpc.fpc_skeleton(ctx, Xd, resume=part, stop_after_levels=1, **kw)
            assert len(step["levels"]) == k + 1
            same(fpc.fpc_skeleton(ctx, Xd, resume=step, **kw), full, f"resume after {k} + 1 levels")


def test_resume_with_the_learned_order(fpc, ctx):
    """The learned order's features use the first level's partial
    correlations, recomputed on resume."""
    p = np.zeros(fpc.fpc_mlp_params(), np.float32)
    p[64] = 4.0  # feature 1 (first-level |r|) -> unit 0
    p[256] = 1.0
    p[4416] = 1.0
    p[:192] += (0.05 * np.random.default_rng(2).standard_normal(192)).astype(np.float32)
    model = fpc.fpc_mlp_init(ctx, p)
    Xd = dev(data(60, 16, 5.0, 3000))
    kw = dict(alpha=0.01, max_level=5, precision=1, order_model=model)
    full = fpc.fpc_skeleton(ctx, Xd, **kw)
    for k in (1, 2, 3):
        part = fpc.fpc_skeleton(ctx, Xd, stop_after_levels=k, **kw)
        same(fpc.fpc_skeleton(ctx, Xd, resume=part, **kw), full, f"learned, resume after {k}")


def test_checkpoint_file_round_trip(fpc, ctx, tmp_path):
    Xd = dev(data())
    kw = dict(alpha=0.01, max_level=-1, precision=1)
    full = fpc.fpc_skeleton(ctx, Xd, **kw)
    part = fpc.fpc_skeleton(ctx, Xd, stop_after_levels=2, **kw)
    path = str(tmp_path / "ck.npz")
    fpc.save_checkpoint(path, part)
    st = fpc.load_checkpoint(path)
    assert st["next_level"] == part["next_level"] and len(st["levels"]) == 2
    assert st["levels"][1]["tests_required"] == part["levels"][1]["tests_required"]
    same(fpc.fpc_skeleton(ctx, Xd, resume=st, **kw), full, "from file")


def _oracle_state(ref):
    """A library checkpoint dict from an oracle result stopped at a boundary."""
    p = ref["p"]
    P = p * (p - 1) // 2
    iu, ju = np.triu_indices(p, 1)
    kind = ref["sep_kind"]
    lists = [ref["sepsets"][(int(iu[k]), int(ju[k]))] if kind[k] == oracle.SEP_LIST else [] for k in range(P)]
    off = np.zeros(P + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in lists])
    nodes = np.array([v for x in lists for v in x], dtype=np.int32)
    levels = [dict(level=int(r[0]), max_cand=0, edges_eligible=int(r[1]), tests_possible=0, tests_executed=int(r[2]),
                   tests_rechecked=0, deleted=int(r[3]), kernel_ms=0.0, test_kernel_ms=0.0, test_launches=0,
                   reserved=0, level_ms=0.0, tests_required=int(r[2])) for r in ref["levels"]]
    return dict(p=p, next_level=ref["next_level"], adj=ref["adj"], sep_level=ref["sep_level"], sep_kind=kind,
                sep_off=off, sep_nodes=nodes, levels=levels)


def _library_state(res):
    """An oracle resume dict from a library result stopped at a boundary."""
    lv = np.array([[x["level"], x["edges_eligible"], x["tests_required"], x["deleted"], 0] for x in res["levels"]],
                  dtype=np.int64)
    return dict(adj=res["adj"], sep_level=res["sep_level"], sep_kind=res["sep_kind"], sepsets=dict(res["sepsets"]),
                next_level=res["next_level"], levels=lv, total_tests=int(lv[:, 2].sum()))


@pytest.mark.parametrize("reverse", [True, False])
def test_resume_across_library_and_oracle(fpc, ctx, reverse):
    """FP64: a boundary state written by either side, continued by the
    other, ends in the oracle's uninterrupted result."""
    X = data(30, 17, 5.0, 1500)
    C = oracle.corr(X)
    Xd = dev(X)
    sched = fpc.FPC_REVERSE if reverse else fpc.FPC_FORWARD
    full = oracle.skeleton(C, 1500, alpha=0.01, reverse=reverse)
    for k in (1, 2):
        o_part = oracle.skeleton(C, 1500, alpha=0.01, reverse=reverse, stop_after_levels=k)
        got = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, schedule=sched, resume=_oracle_state(o_part))
        assert np.array_equal(got["adj"], full["adj"]) and got["sepsets"] == full["sepsets"]
        assert np.array_equal(got["sep_level"], full["sep_level"])
        g_part = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, schedule=sched, stop_after_levels=k)
        assert g_part["next_level"] == o_part["next_level"]
        back = oracle.skeleton(C, 1500, alpha=0.01, reverse=reverse, resume=_library_state(g_part))
        assert np.array_equal(back["adj"], full["adj"]) and back["sepsets"] == full["sepsets"]


def test_resume_errors(fpc, ctx):
    Xd = dev(data())
    part = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, stop_after_levels=1)
    with pytest.raises(fpc.FastPCError) as e:  # another p
        fpc.fpc_skeleton(ctx, Xd[:, :39], alpha=0.01, resume=part)
    assert e.value.code == fpc.FPC_EINVAL
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, Xd, alpha=0.01, resume=part, flags=fpc.FPC_FLAG_LOG_FEATURES)
    assert e.value.code == fpc.FPC_EINVAL
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, Xd, alpha=0.01, stop_after_levels=-1)
    assert e.value.code == fpc.FPC_EINVAL
    bad = dict(part)
    bad["next_level"] = 40
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_skeleton(ctx, Xd, alpha=0.01, resume=bad)
    # a complete run resumed is the same run
    full = fpc.fpc_skeleton(ctx, Xd, alpha=0.01)
    same(fpc.fpc_skeleton(ctx, Xd, alpha=0.01, resume=full), full, "complete")


def test_allocation_failure_hook(fpc):
    """FPC_FAIL_ALLOC=1: every device allocation the library attempts
    fails with FPC_ENOMEM before the runtime is called; without it the same
    context works."""
    Xd = dev(data(25, 18, 4.0, 800))
    with fpc.Context(0) as c:
        ref = fpc.fpc_skeleton(c, Xd, alpha=0.01)
        big = dev(data(120, 19, 4.0, 3000))
        os.environ["FPC_FAIL_ALLOC"] = "1"
        try:
            with pytest.raises(fpc.FastPCError) as e:  # a larger problem needs larger buffers
                fpc.fpc_skeleton(c, big, alpha=0.01)
            assert e.value.code == fpc.FPC_ENOMEM
            with pytest.raises(fpc.FastPCError) as e:
                fpc.Context(0)
            assert e.value.code == fpc.FPC_ENOMEM
        finally:
            del os.environ["FPC_FAIL_ALLOC"]
        got = fpc.fpc_skeleton(c, Xd, alpha=0.01)
        assert np.array_equal(got["adj"], ref["adj"]) and got["sepsets"] == ref["sepsets"]
        fpc.fpc_skeleton(c, big, alpha=0.01)
