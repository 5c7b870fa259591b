"""Full-size parity: the benchmark workload (p = 1000, n = 10000, X in
FP32, max_level = 5) in the launch configuration bench.py times, against
the oracle's stored results (tests/golden/make_goldens.py) and against
per-test oracle calls on sampled outputs.  GPU only."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import semdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens  # noqa: E402

NAME, SEED = "er_p1000_n10000_d4", 0


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_04626_amd as fpc

    X, sem, cfg = semdata.workload(NAME, SEED)
    gold = make_goldens.load(NAME, SEED)
    ctx = fpc.Context(0)
    Xd = torch.from_numpy(X).cuda()
    yield fpc, ctx, X, Xd, cfg, gold
    ctx.close()


def test_golden_matches_workload(setup):
    fpc, ctx, X, Xd, cfg, gold = setup
    assert gold["p"] == cfg["p"] and gold["n"] == cfg["n"] and gold["max_level"] == cfg["max_level"]
    assert gold["min_margin"] > 1e-9  # no near-tie in the oracle's decisions


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_fullsize_skeleton_bit_exact(setup, prec, flags):
    fpc, ctx, X, Xd, cfg, gold = setup
    print(f"[fullsize] {NAME} seed={SEED} precision={prec} flags={flags}", flush=True)
    got = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=prec,
                           flags=flags)
    assert np.array_equal(got["adj"], gold["adj"])
    assert np.array_equal(got["sep_level"], gold["sep_level"])
    assert np.array_equal(got["sep_kind"], gold["sep_kind"])
    if prec == 0:
        assert got["sepsets"] == gold["sepsets"]
    else:
        # every GPU separating set re-tests as independent in the oracle
        C = oracle.corr(X.astype(np.float64))
        q = gold["q"]
        bad = [(k, K) for k, K in got["sepsets"].items() if not oracle.ci_test(C, cfg["n"], *k, K, q)[0]]
        assert not bad, bad[:5]
        same = sum(got["sepsets"][k] == gold["sepsets"].get(k) for k in got["sepsets"])
        print(f"  mixed sepsets identical to the oracle's: {same}/{len(got['sepsets'])}", flush=True)
    lv = {x["level"]: x for x in got["levels"]}
    for row in gold["levels"]:
        l, elig, tests, dels = int(row[0]), int(row[1]), int(row[2]), int(row[3])
        assert lv[l]["deleted"] == dels and lv[l]["edges_eligible"] == elig
        assert lv[l]["tests_executed"] >= tests


def test_fullsize_first_level_sampled(setup):
    """r of sampled pairs at l = p-2 against the oracle's explicit inverse."""
    fpc, ctx, X, Xd, cfg, gold = setup
    C = oracle.corr(X.astype(np.float64))
    Om = oracle.inverse(C)
    r, ind = fpc.fpc_first_level(ctx, torch.from_numpy(C).cuda(), cfg["n"], gold["q"])
    r = r.cpu().numpy()
    rng = np.random.default_rng(0)
    p = cfg["p"]
    for _ in range(2000):
        i, j = rng.choice(p, 2, replace=False)
        ref = -Om[i, j] / np.sqrt(Om[i, i] * Om[j, j])
        assert abs(r[i, j] - ref) < 1e-10


def test_fullsize_corr(setup):
    fpc, ctx, X, Xd, cfg, gold = setup
    C = oracle.corr(X.astype(np.float64))
    c64 = fpc.fpc_corr(ctx, Xd, fpc.FPC_CORR_FP64).cpu().numpy()
    c32 = fpc.fpc_corr(ctx, Xd, fpc.FPC_CORR_BF16X3).cpu().numpy().astype(np.float64)
    e64, e32 = np.abs(c64 - C).max(), np.abs(c32 - C).max()
    print(f"  corr max err fp64 {e64:.2e} bf16x3 {e32:.2e}", flush=True)
    assert e64 < 1e-12 and e32 < 5e-6
