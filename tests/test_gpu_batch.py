"""Many instances in one call (fpc_skeleton_batch), through the C ABI (GPU
only).

Every instance's result must equal that of fpc_skeleton on the instance
alone (skeleton, separating sets, level sequence), and the oracle's
skeleton at the sizes the oracle finishes quickly.  Resampled instances are
checked against the resampled rows materialised on the host.
"""
from __future__ import annotations

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


def _same(a, b, exact_sepsets=True):
    assert np.array_equal(a["adj"], b["adj"])
    assert np.array_equal(a["sep_level"], b["sep_level"])
    assert np.array_equal(a["sep_kind"], b["sep_kind"])
    if exact_sepsets:
        assert a["sepsets"] == b["sepsets"]
    la = [(x["level"], x["edges_eligible"], x["tests_possible"], x["deleted"]) for x in a["levels"]]
    lb = [(x["level"], x["edges_eligible"], x["tests_possible"], x["deleted"]) for x in b["levels"]]
    assert la == lb


def _mixed_instances(dtype, scale):
    base, boots, datas, cfg = semdata.batched_workload(n_boot=5, n_data=6, scale=scale, x_dtype=dtype)
    inst = [(base, None)] + [(base, r) for r in boots] + [(d, None) for d in datas]
    return inst, cfg


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("flags", [0, 4])
def test_batch_equals_single_runs(fpc, ctx, prec, flags):
    """Bootstraps of one data set and uneven independent data sets."""
    inst, cfg = _mixed_instances("f64" if prec == 0 else "f32", 0.06)
    _say(f"[batch] {len(inst)} instances, p={[x.shape[1] for x, _ in inst]} n={cfg['n']} prec={prec} flags={flags}")
    base_d = dev(inst[0][0])
    dinst = []
    for X, rows in inst:
        Xd = base_d if X is inst[0][0] else dev(X)
        dinst.append((Xd, None if rows is None else dev(rows)))
    got = fpc.fpc_skeleton_batch(ctx, dinst, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=prec,
                                 flags=flags)
    assert len(got) == len(inst)
    for k, (X, rows) in enumerate(inst):
        Xk = X if rows is None else X[rows]
        one = fpc.fpc_skeleton(ctx, dev(Xk), alpha=cfg["alpha"], max_level=cfg["max_level"], precision=prec)
        _same(got[k], one)
        if prec == 0 and k < 4:
            C = oracle.corr(Xk.astype(np.float64))
            ref = oracle.skeleton(C, Xk.shape[0], alpha=cfg["alpha"], max_level=cfg["max_level"])
            assert np.array_equal(got[k]["adj"], ref["adj"])
            assert got[k]["sepsets"] == ref["sepsets"]


def test_batch_of_one_and_uneven_levels(fpc, ctx):
    """A batch of one equals the single call; instances whose level
    sequences differ (a small dense graph next to a sparse larger one)."""
    X1, _, _ = semdata.workload("er_p20_n1000_d3", 3)
    sem2 = semdata.make_sem(60, 9, degree=6.0)
    X2 = semdata.sample(sem2, 1500, 9)
    X3 = semdata.sample(semdata.make_sem(7, 5, degree=4.0), 300, 5)
    one = fpc.fpc_skeleton(ctx, dev(X1), alpha=0.01)
    got = fpc.fpc_skeleton_batch(ctx, [(dev(X1), None)], alpha=0.01)
    _same(got[0], one)
    got = fpc.fpc_skeleton_batch(ctx, [(dev(X1), None), (dev(X2), None), (dev(X3), None)], alpha=0.01)
    for k, X in enumerate((X1, X2, X3)):
        _same(got[k], fpc.fpc_skeleton(ctx, dev(X), alpha=0.01))
        C = oracle.corr(X)
        ref = oracle.skeleton(C, X.shape[0], alpha=0.01)
        assert np.array_equal(got[k]["adj"], ref["adj"]) and got[k]["sepsets"] == ref["sepsets"]


def test_batch_errors(fpc, ctx):
    X = dev(semdata.sample(semdata.make_sem(10, 1), 200, 1))
    bad_rows = torch.tensor([0, 1, 500] + [2] * 197, dtype=torch.int32, device="cuda")
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_skeleton_batch(ctx, [(X, None), (X, bad_rows)], alpha=0.01)
    with pytest.raises(fpc.FastPCError):  # n <= p + 1
        fpc.fpc_skeleton_batch(ctx, [(X, None), (X[:11], None)], alpha=0.01)
    with pytest.raises(fpc.FastPCError):  # feature logging is single-instance only
        fpc.fpc_skeleton_batch(ctx, [(X, None)], alpha=0.01, flags=fpc.FPC_FLAG_LOG_FEATURES)
    # the context still works after the errors
    got = fpc.fpc_skeleton_batch(ctx, [(X, None)], alpha=0.01)
    _same(got[0], fpc.fpc_skeleton(ctx, X, alpha=0.01))


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_data_errors(fpc, ctx, prec):
    """The instances' correlations and first levels are queued together:
    non-finite data, a constant column and a bad resample row still give
    their errors (the first instance in order with one), and the context
    then runs a clean batch."""
    _say(f"[batch errors] prec={prec}")
    X = semdata.sample(semdata.make_sem(12, 2), 300, 2)
    good = dev(X)
    nan = X.copy()
    nan[7, 3] = np.nan
    const = X.copy()
    const[:, 5] = 1.5
    cases = ((nan, fpc.FPC_ENONFINITE), (const, fpc.FPC_ESINGULAR))
    for bad, code in cases:
        with pytest.raises(fpc.FastPCError) as e:
            fpc.fpc_skeleton_batch(ctx, [(good, None), (dev(bad), None), (good, None)], alpha=0.01, precision=prec)
        assert e.value.code == code
    # the first failing instance gives the error
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton_batch(ctx, [(dev(const), None), (dev(nan), None)], alpha=0.01, precision=prec)
    assert e.value.code == fpc.FPC_ESINGULAR
    rows = torch.tensor([0, 1, 400] + [2] * 297, dtype=torch.int32, device="cuda")
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton_batch(ctx, [(good, None), (good, rows)], alpha=0.01, precision=prec)
    assert e.value.code == fpc.FPC_EINVAL
    got = fpc.fpc_skeleton_batch(ctx, [(good, None), (good, None)], alpha=0.01, precision=prec)
    one = fpc.fpc_skeleton(ctx, good, alpha=0.01, precision=prec)
    _same(got[0], one)
    _same(got[1], one)


def test_batch_full_size_sampled(fpc, ctx):
    """64 bootstrap resamples of a 500-variable data set and 16 data sets
    with p uniform in [50, 2000] (n = 5000, mixed form, max_level 4) in one
    call; a sample of the instances against single runs."""
    base, boots, datas, cfg = semdata.batched_workload()
    _say(f"[batch full] 64 + 16 instances, p={[d.shape[1] for d in datas]}")
    base_d = dev(base)
    inst = [(base_d, dev(r)) for r in boots] + [(dev(d), None) for d in datas]
    got = fpc.fpc_skeleton_batch(ctx, inst, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1)
    assert len(got) == 80
    for k in (0, 37, 63, 64, 70, 79):
        X, rows = inst[k]
        Xk = X if rows is None else X[rows.long()]
        one = fpc.fpc_skeleton(ctx, Xk, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1)
        _say(f"  instance {k}: p={one['p']} edges={int(one['adj'].sum()) // 2}")
        _same(got[k], one)
