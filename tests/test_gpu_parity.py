"""HIP path vs the FP64 CPU oracle, through the C ABI (GPU only).

Sizes are chosen so the oracle finishes in seconds while the HIP kernels
see several tiles and ragged tails.  Tolerances: z within 1e-6 relative
in FP64 and 1e-4 in FP32 (mixed absolute/relative for z near 0); the
skeleton bit-exact; separating sets identical in FP64 (both sides take
the lexicographically first one) and re-testing as separating in the
oracle for the mixed path.
"""
from __future__ import annotations

import math
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


# ------------------------------------------------------------------ correlation
@pytest.mark.parametrize("p,n,dtype", [(20, 1000, np.float64), (95, 5000, np.float64), (130, 777, np.float32),
                                       (257, 3001, np.float32)])
def test_corr_fp64_matches_oracle(fpc, ctx, p, n, dtype):
    _say(f"[corr fp64] p={p} n={n} {dtype.__name__}")
    sem = semdata.make_sem(p, 5, degree=3.0)
    X = semdata.sample(sem, n, 5, dtype=dtype)
    ref = oracle.corr(X.astype(np.float64))
    got = fpc.fpc_corr(ctx, dev(X), fpc.FPC_CORR_FP64).cpu().numpy()
    assert np.all(np.diag(got) == 1.0)
    err = np.abs(got - ref).max()
    _say(f"  max |C_gpu - C_oracle| = {err:.3e}")
    assert err < 1e-12


# entry error bounds: the two-way split drops lo.lo (biased for strongly
# correlated columns), the three-way split keeps every product above 2^-24,
# leaving the FP32 sums; FP32 rounding of the FP64 matrix is half an ulp
CORR_TOL = {1: 5e-6, 2: 1e-7, 3: 6e-8}


@pytest.mark.parametrize("method", [1, 2, 3], ids=["bf16x3", "bf16x6", "fp32"])
@pytest.mark.parametrize("p,n", [(20, 1000), (130, 777), (257, 3001), (1000, 10000)])
def test_corr_fp32_forms_error(fpc, ctx, p, n, method):
    _say(f"[corr fp32 forms] p={p} n={n} method={method}")
    sem = semdata.make_sem(p, 6, degree=4.0)
    X = semdata.sample(sem, n, 6, dtype=np.float32)
    ref = oracle.corr(X.astype(np.float64))
    got = fpc.fpc_corr(ctx, dev(X), method).cpu().numpy().astype(np.float64)
    assert np.all(np.diag(got) == 1.0)
    err = np.abs(got - ref).max()
    _say(f"  max |C - C_oracle| = {err:.3e}")
    assert err < CORR_TOL[method]


def test_corr_rejects_nonfinite_and_constant(fpc, ctx):
    X = np.random.default_rng(0).standard_normal((100, 5))
    Y = X.copy()
    Y[7, 3] = np.nan
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_corr(ctx, dev(Y))
    assert e.value.code == fpc.FPC_ENONFINITE
    Y = X.copy()
    Y[:, 2] = 4.0
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_corr(ctx, dev(Y))
    assert e.value.code == fpc.FPC_ESINGULAR


# ------------------------------------------------------------------ first level
# p = 33, 64, 65, 97: one to three panels, the last ragged or full, so the
# prologue's second inverse and the look-ahead's partial block both occur
@pytest.mark.parametrize("p,n", [(3, 50), (20, 1000), (33, 500), (64, 800), (65, 800), (95, 5000), (97, 1000),
                                 (150, 2000), (333, 4000)])
def test_first_level_matches_oracle_inverse(fpc, ctx, p, n):
    _say(f"[first level] p={p} n={n}")
    sem = semdata.make_sem(p, 7, degree=4.0)
    X = semdata.sample(sem, n, 7)
    C = oracle.corr(X)
    Om = oracle.inverse(C)
    d = np.sqrt(np.diag(Om))
    r_ref = -Om / np.outer(d, d)
    q = oracle.quantile(0.01)
    r, ind = fpc.fpc_first_level(ctx, dev(C), n, q)
    r = r.cpu().numpy()
    ind = ind.cpu().numpy()
    off = ~np.eye(p, dtype=bool)
    err = np.abs(r - r_ref)[off].max()
    _say(f"  max |r_gpu - r_oracle| = {err:.3e}")
    assert err < 1e-10
    res = oracle.skeleton(C, n, q=q, max_level=0)
    iu, ju = np.triu_indices(p, 1)
    want = res["sep_level"] == p - 2
    assert np.array_equal(ind[iu, ju].astype(bool), want)


def test_first_level_rejects_indefinite(fpc, ctx):
    C = np.eye(4)
    C[0, 1] = C[1, 0] = 0.9
    C[1, 2] = C[2, 1] = 0.9
    C[0, 2] = C[2, 0] = -0.9
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_first_level(ctx, dev(C), 100, 2.5)
    assert e.value.code == fpc.FPC_ESINGULAR


# ------------------------------------------------------------------ index-matrix batches
def _rows(rng, p, l, b):
    return np.stack([rng.permutation(p)[: l + 2] for _ in range(b)]).astype(np.int32)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 5, 8, 12, 16, 17, 24, 40])
def test_ci_batch_fp64_z_within_1e6(fpc, ctx, l):
    _say(f"[ci_batch fp64] l={l}")
    p, n = 60, 3000
    sem = semdata.make_sem(p, 8, degree=4.0)
    C = oracle.corr(semdata.sample(sem, n, 8))
    rng = np.random.default_rng(l)
    B = _rows(rng, p, l, 300)
    q = oracle.quantile(0.01)
    z, ind = fpc.fpc_ci_batch(ctx, dev(C), n, dev(B), q)
    z = z.cpu().numpy()
    ind = ind.cpu().numpy()
    for k in range(B.shape[0]):
        i, j, *K = B[k].tolist()
        indep, zr, st = oracle.ci_test(C, n, i, j, K, q)
        assert st == 0
        assert abs(z[k] - zr) <= 1e-6 * max(abs(zr), 1e-3), (k, z[k], zr)
        assert bool(ind[k]) == indep


@pytest.mark.parametrize("l", [0, 1, 3, 5, 8, 16, 20])
def test_ci_batch_fp32_z_within_1e4(fpc, ctx, l):
    _say(f"[ci_batch fp32] l={l}")
    p, n = 60, 3000
    sem = semdata.make_sem(p, 9, degree=3.0)
    C = oracle.corr(semdata.sample(sem, n, 9))
    rng = np.random.default_rng(100 + l)
    B = _rows(rng, p, l, 300)
    q = oracle.quantile(0.01)
    z, _ = fpc.fpc_ci_batch(ctx, dev(C.astype(np.float32)), n, dev(B), q)
    z = z.cpu().numpy()
    worst = 0.0
    for k in range(B.shape[0]):
        i, j, *K = B[k].tolist()
        _, zr, st = oracle.ci_test(C, n, i, j, K, q)
        worst = max(worst, abs(z[k] - zr) / max(abs(zr), 1.0))
    _say(f"  worst mixed error {worst:.2e}")
    assert worst <= 1e-4


def test_ci_batch_degenerate_rows(fpc, ctx):
    C = np.eye(5)
    C[0, 2] = C[2, 0] = 1.0  # identical variables 0 and 2
    B = np.array([[1, 3, 0, 2]], np.int32)
    z, ind = fpc.fpc_ci_batch(ctx, dev(C), 100, dev(B), 2.5)
    assert math.isnan(float(z[0])) and int(ind[0]) == 0


# ------------------------------------------------------------------ skeleton
def _compare_fp64(fpc, got, ref, p):
    assert np.array_equal(got["adj"], ref["adj"])
    assert np.array_equal(got["sep_level"], ref["sep_level"])
    assert np.array_equal(got["sep_kind"], ref["sep_kind"])
    assert got["sepsets"] == ref["sepsets"]


def _retest_sepsets(fpc, got, C, n, q):
    """Every GPU separating set re-tests as independent in the oracle."""
    p = got["p"]
    bad = []
    for (i, j), K in got["sepsets"].items():
        indep, z, st = oracle.ci_test(C, n, i, j, K, q)
        if not indep:
            bad.append((i, j, K, z))
    assert not bad, bad[:5]


@pytest.mark.parametrize("seed", range(10))
def test_skeleton_fp64_cfg1_bit_exact(fpc, ctx, seed):
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", seed)
    _say(f"[skeleton fp64] er_p20_n1000_d3 seed={seed}")
    C = oracle.corr(X)
    ref = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"])
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=cfg["alpha"])
    _compare_fp64(fpc, got, ref, cfg["p"])
    assert got["total_tests"] >= ref["total_tests"]
    # tests the method needs (first hit per edge in lexicographic order) = the oracle's count
    assert got["total_required"] == ref["total_tests"]


@pytest.mark.parametrize("seed", range(5))
def test_skeleton_mixed_cfg1_bit_exact(fpc, ctx, seed):
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", seed)
    _say(f"[skeleton mixed] er_p20_n1000_d3 seed={seed}")
    C = oracle.corr(X)
    ref = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"])
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=cfg["alpha"], precision=fpc.FPC_PREC_MIXED)
    # FP32 decisions outside the error band, FP64 re-runs inside it: the
    # oracle's skeleton, lexicographically first sets and required count
    _compare_fp64(fpc, got, ref, cfg["p"])
    assert got["total_required"] == ref["total_tests"]
    _retest_sepsets(fpc, got, C, cfg["n"], ref["q"])


@pytest.mark.parametrize("seed", range(4))
def test_skeleton_forward_matches_oracle(fpc, ctx, seed):
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", seed)
    _say(f"[skeleton forward] seed={seed}")
    C = oracle.corr(X)
    ref = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"], reverse=False)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=cfg["alpha"], schedule=fpc.FPC_FORWARD)
    _compare_fp64(fpc, got, ref, cfg["p"])


@pytest.mark.parametrize("p,n,deg,L,prec,graph", [(57, 2000, 5.0, -1, 0, "er"), (90, 3000, 5.0, -1, 1, "er"),
                                                  (150, 4000, 4.0, 3, 1, "ba"), (95, 10000, 0.0, -1, 0, "paper")])
def test_skeleton_forward_mid_sizes(fpc, ctx, p, n, deg, L, prec, graph):
    """Algorithm 1 beyond p = 20: levels 0, 1, ... on mid-size ER, a
    scale-free graph and the paper-shape graph, against the oracle's
    forward run (FP64 sepsets equal; mixed skeletons equal)."""
    _say(f"[skeleton forward mid] p={p} n={n} deg={deg} L={L} prec={prec} graph={graph}")
    if graph == "paper":
        X, sem, cfg = semdata.workload("paper_p95_n10000", 0)
        alpha = cfg["alpha"]
    else:
        sem = semdata.make_sem(p, 31, graph=graph, degree=deg)
        X = semdata.sample(sem, n, 31)
        alpha = 0.01
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=alpha, max_level=L, reverse=False)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=alpha, max_level=L, precision=prec, schedule=fpc.FPC_FORWARD)
    assert np.array_equal(got["adj"], ref["adj"])
    assert np.array_equal(got["sep_level"], ref["sep_level"])
    if prec == 0:
        assert got["sepsets"] == ref["sepsets"]
        assert got["total_required"] == ref["total_tests"]
    assert [x["level"] for x in got["levels"]] == [int(r[0]) for r in ref["levels"]]


def test_lists_of_1024_or_more_are_reported(fpc, ctx):
    """The forward schedule on p = 1030 independent variables starts at
    level 0 on the complete graph, whose lists hold p - 2 = 1028
    candidates: FPC_ETOOLARGE.  The reverse schedule on the same data
    works (its first level uses the inverse)."""
    X = np.random.default_rng(8).standard_normal((1100, 1030)).astype(np.float32)
    Xd = dev(X)
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, Xd, alpha=0.01, schedule=fpc.FPC_FORWARD)
    assert e.value.code == fpc.FPC_ETOOLARGE
    got = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, max_level=2)
    assert got["levels"][0]["level"] == 1028


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("p,n,deg,L,prec", [(57, 2000, 5.0, 4, 0), (57, 2000, 5.0, 4, 1),
                                             (130, 3000, 4.0, 3, 0), (130, 3000, 4.0, 3, 1),
                                             (90, 3000, 5.0, 6, 0), (90, 3000, 5.0, 6, 1),
                                             (40, 800, 6.0, -1, 0), (40, 800, 6.0, -1, 1)])
def test_skeleton_mid_sizes(fpc, ctx, p, n, deg, L, prec, flags):
    _say(f"[skeleton mid] p={p} n={n} deg={deg} L={L} prec={prec} flags={flags}")
    sem = semdata.make_sem(p, 11, degree=deg)
    X = semdata.sample(sem, n, 11)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=0.01, max_level=L)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=0.01, max_level=L, precision=prec, flags=flags)
    assert np.array_equal(got["adj"], ref["adj"])
    assert np.array_equal(got["sep_level"], ref["sep_level"])
    assert got["sepsets"] == ref["sepsets"]
    assert got["total_required"] == ref["total_tests"]
    if prec == 1:
        _retest_sepsets(fpc, got, C, n, ref["q"])
    _say(f"  tests gpu={got['total_tests']} required={got['total_required']} oracle={ref['total_tests']}")


@pytest.mark.parametrize("prec", [0, 1])
def test_skeleton_graph_mode_matches_eager(fpc, ctx, prec):
    """FPC_FLAG_GRAPH: each level's launches captured in one HIP graph; three
    runs in a row, eager runs between them, all equal to the eager result
    and to the oracle's skeleton."""
    p, n = 90, 3000
    _say(f"[graph mode] p={p} n={n} prec={prec}")
    sem = semdata.make_sem(p, 41, degree=5.0)
    X = semdata.sample(sem, n, 41)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=0.01, max_level=6)
    Xd = dev(X)
    for rep in range(3):
        eager = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, max_level=6, precision=prec)
        got = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, max_level=6, precision=prec, flags=fpc.FPC_FLAG_GRAPH)
        assert np.array_equal(got["adj"], ref["adj"]) and np.array_equal(eager["adj"], ref["adj"])
        assert np.array_equal(got["sep_level"], ref["sep_level"])
        assert got["sepsets"] == eager["sepsets"]
        assert got["sepsets"] == ref["sepsets"]
    if prec == 1:
        _retest_sepsets(fpc, got, C, n, ref["q"])


@pytest.mark.parametrize("p,n,deg,L,seed,prec", [(60, 1500, 8.0, -1, 5, 0), (60, 1500, 8.0, -1, 5, 1),
                                                 (40, 800, 6.0, -1, 11, 1), (90, 3000, 5.0, 6, 41, 1),
                                                 (90, 3000, 5.0, 6, 11, 1)])
def test_skeleton_small_levels_back_to_back(fpc, ctx, p, n, deg, L, seed, prec):
    """Small levels are queued back to back (up to eight, fewer after a run
    cut short by a deletion) and kept up to the first one that deletes an
    edge; a test budget makes every level run on its own.  Both runs give
    the oracle's sequence of levels (level, deletions, tests required),
    skeleton and separating sets."""
    _say(f"[small levels] p={p} n={n} deg={deg} L={L} seed={seed} prec={prec}")
    sem = semdata.make_sem(p, seed, degree=deg)
    X = semdata.sample(sem, n, seed)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=0.01, max_level=L)
    want = [(int(r[0]), int(r[3]), int(r[2])) for r in ref["levels"]]
    # the case has a subset level that deletes nothing with a level after it
    assert any(w[1] == 0 for w in want[1:-1])
    Xd = dev(X)
    queued = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, max_level=L, precision=prec)
    single = fpc.fpc_skeleton(ctx, Xd, alpha=0.01, max_level=L, precision=prec, max_tests=1 << 62)
    for got in (queued, single):
        assert [(x["level"], x["deleted"], x["tests_required"]) for x in got["levels"]] == want
        assert np.array_equal(got["adj"], ref["adj"])
        assert np.array_equal(got["sep_level"], ref["sep_level"])
        assert got["sepsets"] == ref["sepsets"]
    for x, y in zip(queued["levels"], single["levels"]):
        assert (x["tests_possible"], x["edges_eligible"], x["max_cand"]) == \
               (y["tests_possible"], y["edges_eligible"], y["max_cand"])
    # every subset level keeps its own launch count and device time
    assert all(x["test_launches"] >= 1 and x["kernel_ms"] > 0.0 for x in queued["levels"][1:])


# ------------------------------------------------------------------ edge cases
def test_skeleton_smallest_graphs(fpc, ctx):
    rng = np.random.default_rng(3)
    for p in (2, 3, 4):
        X = rng.standard_normal((50, p))
        X[:, 0] += 0.9 * X[:, p - 1]
        C = oracle.corr(X)
        for sched, rev in ((fpc.FPC_REVERSE, True), (fpc.FPC_FORWARD, False)):
            ref = oracle.skeleton(C, 50, alpha=0.05, reverse=rev)
            got = fpc.fpc_skeleton(ctx, dev(X), alpha=0.05, schedule=sched)
            _compare_fp64(fpc, got, ref, p)


def test_skeleton_extreme_thresholds(fpc, ctx):
    p = 10
    X, _, _ = semdata.workload("er_p20_n1000_d3", 1, p=p)
    got = fpc.fpc_skeleton(ctx, dev(X), q_override=float("inf"))
    assert got["adj"].sum() == 0 and got["total_tests"] == p * (p - 1) // 2
    got = fpc.fpc_skeleton(ctx, dev(X), q_override=0.0)
    assert got["adj"].sum() == p * (p - 1)
    assert got["total_tests"] == (p * (p - 1) // 2) * 2 ** (p - 2)


def test_skeleton_errors(fpc, ctx):
    rng = np.random.default_rng(4)
    X = rng.standard_normal((30, 6))
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(X[:7]))  # n <= p + 1
    assert e.value.code == fpc.FPC_EINVAL
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(X), alpha=1.5)
    assert e.value.code == fpc.FPC_EINVAL
    Y = X.copy()
    Y[3, 3] = np.inf
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(Y))
    assert e.value.code == fpc.FPC_ENONFINITE
    Y = X.copy()
    Y[:, 4] = Y[:, 1]  # duplicate column: C singular
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(Y))
    assert e.value.code == fpc.FPC_ESINGULAR
    # the mixed form queues its FP32 matrix behind the first level: the same
    # errors, and a failed call leaves the context usable
    ref = fpc.fpc_skeleton(ctx, dev(X), precision=fpc.FPC_PREC_MIXED)
    Y = X.copy()
    Y[3, 3] = np.inf
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(Y), precision=fpc.FPC_PREC_MIXED)
    assert e.value.code == fpc.FPC_ENONFINITE
    Y = X.copy()
    Y[:, 4] = Y[:, 1]
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(Y), precision=fpc.FPC_PREC_MIXED)
    assert e.value.code == fpc.FPC_ESINGULAR
    again = fpc.fpc_skeleton(ctx, dev(X), precision=fpc.FPC_PREC_MIXED)
    assert np.array_equal(again["adj"], ref["adj"]) and again["sepsets"] == ref["sepsets"]
    assert again["corr_max_abs_err"] == ref["corr_max_abs_err"]
    Xb, _, _ = semdata.workload("er_p20_n1000_d3", 0)
    with pytest.raises(fpc.FastPCError) as e:
        fpc.fpc_skeleton(ctx, dev(Xb), max_tests=500)
    assert e.value.code == fpc.FPC_EBUDGET


def test_skeleton_host_input_and_determinism(fpc, ctx):
    X, _, cfg = semdata.workload("er_p20_n1000_d3", 3)
    a = fpc.fpc_skeleton(ctx, X)  # host pointer
    b = fpc.fpc_skeleton(ctx, dev(X))
    assert np.array_equal(a["adj"], b["adj"]) and a["sepsets"] == b["sepsets"]
    assert [x["tests_executed"] for x in a["levels"][:1]] == [x["tests_executed"] for x in b["levels"][:1]]


@pytest.mark.parametrize("seed", range(4))
def test_cpdag_from_gpu_skeleton_matches_oracle(fpc, ctx, seed):
    """Phase II on the GPU run's skeleton and separating sets equals the
    oracle's Phase II on its own run."""
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", seed)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"])
    want = oracle.orient(ref["adj"], lambda i, j: oracle.sepset_of(ref, i, j))
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=cfg["alpha"])
    assert np.array_equal(fpc.fpc_orient(got), want)
