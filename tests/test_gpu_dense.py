"""Dense small graphs: FP32 tests with FP64 re-runs near the threshold
must give the oracle's skeleton bit-exact, and both forms its separating
sets and test count, against the oracle's stored results
(tests/golden/make_goldens.py).  GPU only.

* er_p95_n5000_d12 (expected degree 12, n = 5000, max_level 6): C has a
  condition number of about 2e7; after the first level only levels 6 and 0
  run (level 6 leaves lists too short for 5..1);
* er_p95_n20000_d8_paper (degree 8, the paper's weight law, n = 20000,
  max_level 6): the levels after the first run 6, 5, 4, 3, 2, 1, 0."""
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

SEED = 0


@pytest.fixture(scope="module", params=["er_p95_n5000_d12", "er_p95_n20000_d8_paper"])
def setup(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_04626_amd as fpc

    name = request.param
    X, sem, cfg = semdata.workload(name, SEED)
    gold = make_goldens.load(name, SEED)
    ctx = fpc.Context(0)
    yield fpc, ctx, X, torch.from_numpy(X).cuda(), cfg, gold, name
    ctx.close()


@pytest.mark.parametrize("flags", [0, 4])
@pytest.mark.parametrize("prec", [0, 1])
def test_dense_skeleton_bit_exact(setup, prec, flags):
    fpc, ctx, X, Xd, cfg, gold, name = setup
    print(f"[dense] {name} seed={SEED} precision={prec} flags={flags}", flush=True)
    assert gold["p"] == cfg["p"] and gold["max_level"] == cfg["max_level"] and gold["min_margin"] > 1e-9
    got = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=prec, flags=flags)
    assert np.array_equal(got["adj"], gold["adj"])
    assert np.array_equal(got["sep_level"], gold["sep_level"])
    assert np.array_equal(got["sep_kind"], gold["sep_kind"])
    assert got["total_required"] == gold["total_tests"]
    assert dict(got["sepsets"]) == gold["sepsets"]
    if prec == 1:
        C = oracle.corr(X)
        bad = [(k, K) for k, K in got["sepsets"].items() if not oracle.ci_test(C, cfg["n"], *k, K, gold["q"])[0]]
        assert not bad, bad[:5]
        print(f"  re-run in FP64: {sum(x['tests_rechecked'] for x in got['levels'])} of "
              f"{got['total_tests']} tests; corr max abs err {got['corr_max_abs_err']:.2e}", flush=True)
    assert [x["level"] for x in got["levels"]] == [int(r[0]) for r in gold["levels"]]
    lv = {x["level"]: x for x in got["levels"]}
    for row in gold["levels"]:
        l, elig, dels = int(row[0]), int(row[1]), int(row[3])
        assert lv[l]["deleted"] == dels and lv[l]["edges_eligible"] == elig
