"""Full-size parity: the benchmark workload (p = 1000, n = 10000, X in
FP32, max_level = 5) in the launch configuration bench.py times, against
the oracle's stored results (tests/golden/make_goldens.py) and against
per-test oracle calls on sampled outputs.  GPU only."""
from __future__ import annotations

import math
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


@pytest.mark.parametrize("flags,tau,c32", [(0, 1e-4, 2), (1, 1e-4, 2), (0, -1.0, 2), (0, 1e-4, 1), (0, 1e-4, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_fullsize_skeleton_bit_exact(setup, prec, flags, tau, c32):
    fpc, ctx, X, Xd, cfg, gold = setup
    if prec == 0 and (tau != 1e-4 or c32 != 2):
        pytest.skip("FP64 form: no FP32 matrix and no trigger")
    print(f"[fullsize] {NAME} seed={SEED} precision={prec} flags={flags} tau={tau} c32={c32}", flush=True)
    got = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=prec,
                           flags=flags, ill_cond_tau=tau, c32_method=c32)
    assert np.array_equal(got["adj"], gold["adj"])
    assert np.array_equal(got["sep_level"], gold["sep_level"])
    assert np.array_equal(got["sep_kind"], gold["sep_kind"])
    # the lexicographically first separating set of every deleted edge: the
    # FP32 kernels decide only outside their error band and the FP64 re-run
    # decides inside it, so the mixed form finds the oracle's sets too
    assert dict(got["sepsets"]) == gold["sepsets"]
    if prec == 1:
        # and each re-tests as independent in the oracle
        C = oracle.corr(X.astype(np.float64))
        q = gold["q"]
        bad = [(k, K) for k, K in got["sepsets"].items() if not oracle.ci_test(C, cfg["n"], *k, K, q)[0]]
        assert not bad, bad[:5]
    lv = {x["level"]: x for x in got["levels"]}
    for row in gold["levels"]:
        l, elig, tests, dels = int(row[0]), int(row[1]), int(row[2]), int(row[3])
        assert lv[l]["deleted"] == dels and lv[l]["edges_eligible"] == elig
        assert lv[l]["tests_required"] == tests  # the oracle's count, level by level
        assert lv[l]["tests_executed"] >= tests
    assert got["total_required"] == gold["total_tests"]


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
    c6 = fpc.fpc_corr(ctx, Xd, fpc.FPC_CORR_BF16X6).cpu().numpy().astype(np.float64)
    cr = fpc.fpc_corr(ctx, Xd, fpc.FPC_CORR_FP32).cpu().numpy().astype(np.float64)
    e64, e32, e6, er = (np.abs(c - C).max() for c in (c64, c32, c6, cr))
    print(f"  corr max err fp64 {e64:.2e} bf16x3 {e32:.2e} bf16x6 {e6:.2e} fp32 {er:.2e}", flush=True)
    assert e64 < 1e-12 and e32 < 5e-6 and e6 < 1e-7 and er < 6e-8


def test_fullsize_level5_z_sampled(setup):
    """z of the dominant level (l = 5, the mixed form's FP32 triple kernel on
    its bf16x6 matrix, in the launch shapes the benchmark uses) against the
    oracle's FP64 tests, rank by rank, on sampled edges of the graph the first
    level leaves: the longest candidate list and a random sample, each on its
    first ranks, a middle run and its last ranks.  Tests decided in FP32 take
    the oracle's decision (default ill-conditioning threshold) and, under the
    strict threshold, have z within 1e-4; the rest go to the FP64 re-run."""
    fpc, ctx, X, Xd, cfg, gold = setup
    C = oracle.corr(X.astype(np.float64))
    p, n, q, l = cfg["p"], cfg["n"], gold["q"], cfg["max_level"]
    # the graph after the first level: every pair the oracle did not delete there
    first = gold["sep_level"] == p - 2
    adj1 = np.ones((p, p), np.uint8)
    iu, ju = np.triu_indices(p, 1)
    adj1[iu[first], ju[first]] = 0
    adj1[ju[first], iu[first]] = 0
    np.fill_diagonal(adj1, 0)
    ei, ej, off, nodes = fpc.fpc_candidates(adj1)  # only to choose which edges to sample
    m = np.diff(off)
    rng = np.random.default_rng(1)
    picks = [int(np.argmax(m))] + [int(k) for k in rng.choice(np.nonzero(m >= l)[0], 11, replace=False)]
    res = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=fpc.FPC_PREC_MIXED)
    c_err = res["corr_max_abs_err"]
    C32 = fpc.fpc_corr(ctx, Xd, fpc.FPC_CORR_BF16X6)
    nu = np.sqrt(n - l - 3)
    worst = 0.0
    rerun = total = 0
    for k in picks:
        i, j = int(ei[k]), int(ej[k])
        cand = oracle.candidates(adj1, i, j)
        assert cand == nodes[off[k]:off[k + 1]].tolist()
        N = math.comb(len(cand), l)
        spans = [(0, min(N, 20000))]
        if N > 60000:
            spans += [(N // 2, N // 2 + 5003), (N - 7001, N)]
        print(f"[fullsize-z] edge ({i},{j}) m={len(cand)} N={N}", flush=True)
        for lo, hi in spans:
            _, z_o = oracle.edge_series(C, n, i, j, cand, l, lo, hi)
            indep_o = z_o <= q
            _, dec = fpc.fpc_level_series(ctx, C32, n, l, i, j, cand, lo, hi, q, band_z=1e-3, c_err=c_err)
            dec = dec.cpu().numpy()
            assert not np.any((dec == 1) & ~indep_o) and not np.any((dec == 0) & indep_o)
            r, dec = fpc.fpc_level_series(ctx, C32, n, l, i, j, cand, lo, hi, q, band_z=1e-3, c_err=c_err,
                                          ill_cond_tau=-1.0)
            r, dec = r.cpu().numpy(), dec.cpu().numpy()
            z = nu * np.abs(np.arctanh(r))
            ok = ~np.isnan(z_o) & ~np.isnan(z) & (dec != 2)
            err = np.abs(z[ok] - z_o[ok]) / np.maximum(1.0, np.abs(z_o[ok]))
            worst = max(worst, float(err.max()))
            assert not np.any((dec == 1) & ~indep_o) and not np.any((dec == 0) & indep_o)
            rerun += int((dec == 2).sum())
            total += len(dec)
    print(f"  worst z error of the FP32 kernel (bf16x6 matrix, c_err {c_err:.2e}, strict threshold): "
          f"{worst:.3e}; left to FP64: {rerun} of {total}", flush=True)
    assert worst <= 1e-4
