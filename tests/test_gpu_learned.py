"""Candidate-ranking MLP and the learned candidate order, through the C ABI
(GPU only).

The network's passes are checked against the oracle's FP64 network run on
the same bf16-rounded weights (the kernels round W1, W2, W3 to bf16 and
accumulate in FP32, so the FP32 error bound over 64-term sums sets the
tolerance).  The learned order must leave the skeleton unchanged (stable
schedule: deleting an edge depends on whether some subset of its
candidates separates it, not on the order they are tried in), and every
separating set it records must re-test as independent in the oracle.
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


def _params(seed):
    rng = np.random.default_rng(seed)
    sizes = [3 * 64, 64, 64 * 64, 64, 64, 1]
    scales = [0.8, 0.1, 0.18, 0.1, 0.25, 0.1]
    return np.concatenate([rng.standard_normal(s) * c for s, c in zip(sizes, scales)]).astype(np.float32)


def _bf16_weights(params):
    """The parameters as the passes see them: weight matrices rounded to
    bf16 (round to nearest even), biases kept in FP32."""
    q = params.astype(np.float64).copy()
    nW1, nb1, nW2, nb2, nW3 = 192, 64, 4096, 64, 64
    o2 = nW1 + nb1
    o3 = o2 + nW2 + nb2
    for a, b in ((0, nW1), (o2, o2 + nW2), (o3, o3 + nW3)):
        q[a:b] = torch.from_numpy(params[a:b].copy()).to(torch.bfloat16).to(torch.float64).numpy()
    return q


def _features(rng, n):
    X = np.empty((n, 3), np.float32)
    X[:, 0] = rng.uniform(0.0, 1.0, n)
    X[:, 1] = X[:, 0] * rng.uniform(0.0, 1.0, n)
    X[:, 2] = rng.integers(0, 40, n) / 99.0
    return X


@pytest.mark.parametrize("n", [1, 31, 1000, 70001])
def test_mlp_forward_matches_oracle(fpc, ctx, n):
    _say(f"[mlp forward] n={n}")
    params = _params(n)
    rng = np.random.default_rng(n + 1)
    X = _features(rng, n)
    model = fpc.fpc_mlp_init(ctx, params)
    np.testing.assert_array_equal(fpc.fpc_mlp_get(ctx, model), params)
    got = fpc.fpc_mlp_forward(ctx, dev(X), model).cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(_bf16_weights(params), X.astype(np.float64))
    scale = 1.0 + np.abs(ref).max()
    assert np.abs(got - ref).max() <= 2e-5 * scale


@pytest.mark.parametrize("n", [1, 32, 1000, 40003])
def test_mlp_grad_matches_oracle(fpc, ctx, n):
    _say(f"[mlp grad] n={n}")
    params = _params(100 + n)
    rng = np.random.default_rng(n + 2)
    X = _features(rng, n)
    y = (rng.random(n) < 0.3).astype(np.float32)
    model = fpc.fpc_mlp_init(ctx, params)
    g, loss = fpc.fpc_mlp_grad(ctx, dev(X), dev(y), model)
    q = _bf16_weights(params)
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    ref = oracle.mlp_grad(q, X64, y64)
    assert abs(loss - oracle.mlp_loss(q, X64, y64)) <= 1e-5 * (1 + abs(loss))
    # per block of parameters, relative to the block's largest entry
    bounds = [0, 192, 256, 4352, 4416, 4480, 4481]
    for a, b in zip(bounds[:-1], bounds[1:]):
        err = np.abs(g[a:b] - ref[a:b]).max()
        assert err <= 1e-4 * (np.abs(ref[a:b]).max() + 1e-6), (a, b, err)


def test_mlp_first_adam_step_is_signed(fpc, ctx):
    """Adam's bias-corrected first step moves every parameter by lr against
    the sign of its gradient (m_hat = g, v_hat = g^2)."""
    params = _params(7)
    rng = np.random.default_rng(8)
    X = _features(rng, 5000)
    y = (rng.random(5000) < 0.25).astype(np.float32)
    model = fpc.fpc_mlp_init(ctx, params)
    lr = 1e-3
    loss = fpc.fpc_mlp_train_step(ctx, dev(X), dev(y), model, lr)
    q = _bf16_weights(params)
    assert abs(loss - oracle.mlp_loss(q, X.astype(np.float64), y.astype(np.float64))) <= 1e-5 * (1 + loss)
    g = oracle.mlp_grad(q, X.astype(np.float64), y.astype(np.float64))
    new = fpc.fpc_mlp_get(ctx, model).astype(np.float64)
    step = new - params.astype(np.float64)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    np.testing.assert_allclose(step[big], -lr * np.sign(g[big]), rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(step) <= lr * (1 + 1e-3) + 1e-7)


def test_mlp_training_lowers_the_loss(fpc, ctx):
    """A separable toy problem: label = feature 0 above 0.5."""
    rng = np.random.default_rng(9)
    X = _features(rng, 20000)
    y = (X[:, 0] > 0.5).astype(np.float32)
    model = fpc.fpc_mlp_init(ctx, _params(9))
    Xd, yd = dev(X), dev(y)
    first = fpc.fpc_mlp_train_step(ctx, Xd, yd, model, 3e-3)
    for _ in range(300):
        last = fpc.fpc_mlp_train_step(ctx, Xd, yd, model, 3e-3)
    assert last < 0.5 * first
    z = fpc.fpc_mlp_forward(ctx, Xd, model).cpu().numpy()
    assert ((z > 0) == (y > 0.5)).mean() > 0.97


def test_mlp_rejects_bad_arguments(fpc, ctx):
    model = fpc.fpc_mlp_init(ctx, _params(1))
    X = dev(np.zeros((4, 3), np.float32))
    y = dev(np.zeros(4, np.float32))
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_mlp_train_step(ctx, X, y, model, 0.0)
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_mlp_grad(ctx, X[:0], y[:0], model)
    assert fpc.fpc_mlp_forward(ctx, X[:0], model).numel() == 0


def test_mlp_forward_hand_computed_network(fpc, ctx):
    """The sparse network of the oracle's hand-computed pin (weights exact
    in bf16): the library's forward pass gives -4.325 and 3.725."""
    p = np.zeros(fpc.fpc_mlp_params(), np.float32)
    oW1, ob1, oW2, ob2, oW3, ob3 = 0, 192, 256, 4352, 4416, 4480
    p[oW1 + 2], p[ob1 + 2], p[oW2 + 2 * 64 + 5], p[ob2 + 5], p[oW3 + 5] = 2.0, -0.5, 3.0, 0.25, -1.5
    p[oW1 + 64 + 7], p[oW2 + 7 * 64 + 9], p[oW3 + 9], p[ob3] = -1.0, 4.0, 2.0, 0.1
    model = fpc.fpc_mlp_init(ctx, p)
    z = fpc.fpc_mlp_forward(ctx, dev(np.array([[0.7, 0.3, 0.9], [0.1, -0.5, 0.0]], np.float32)), model)
    np.testing.assert_allclose(z.cpu().numpy(), [-4.325, 3.725], rtol=0, atol=2e-6)


def test_mlp_init_rejects_non_finite_parameters(fpc, ctx):
    model = fpc.fpc_mlp_init(ctx, _params(2))
    before = fpc.fpc_mlp_get(ctx, model)
    for bad in (np.nan, np.inf, -np.inf):
        p = _params(3)
        p[100] = bad
        with pytest.raises(fpc.FastPCError) as e:
            fpc.fpc_mlp_init(ctx, p, model)
        assert e.value.code == fpc.FPC_EINVAL
    assert np.array_equal(fpc.fpc_mlp_get(ctx, model), before)  # left untouched


def _nan_scoring(fpc, ctx):
    """Finite parameters whose output is inf - inf = NaN for every input:
    two first-layer units of bias 3e38 feed two second-layer units that
    overflow to +inf, weighted +1 and -1 at the output."""
    p = np.zeros(fpc.fpc_mlp_params(), np.float32)
    ob1, oW2, oW3 = 192, 256, 256 + 4096 + 64
    p[ob1 + 0] = p[ob1 + 1] = 3e38
    for i in (0, 1):
        for j in (0, 1):
            p[oW2 + 64 * i + j] = 1.0
    p[oW3 + 0], p[oW3 + 1] = 1.0, -1.0
    return fpc.fpc_mlp_init(ctx, p)


def test_learned_order_with_nan_scores_keeps_the_skeleton(fpc, ctx):
    """Scores that are all NaN rank as equal (-inf), so each list is kept
    as a permutation (here the identity): the skeleton and separating sets
    are the lexicographic ones."""
    model = _nan_scoring(fpc, ctx)
    z = fpc.fpc_mlp_forward(ctx, dev(_features(np.random.default_rng(4), 64)), model).cpu().numpy()
    assert np.isnan(z).all()
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", 1)
    sem2 = semdata.make_sem(60, 9, degree=5.0)
    for Xk, L in ((X, -1), (semdata.sample(sem2, 2000, 9), 4)):
        C = oracle.corr(Xk)
        ref = oracle.skeleton(C, Xk.shape[0], alpha=0.01, max_level=L)
        for prec in (0, 1):
            got = fpc.fpc_skeleton(ctx, dev(Xk), alpha=0.01, max_level=L, precision=prec, order_model=model)
            assert np.array_equal(got["adj"], ref["adj"])
            assert got["sepsets"] == ref["sepsets"]


# ------------------------------------------------------------------ learned order
def _trained_like(fpc, ctx, seed):
    """A model whose score grows with the first-level partial correlation
    (a hand-set network, no training needed): the order it induces is far
    from the id order."""
    p = np.zeros(fpc.fpc_mlp_params(), np.float32)
    p[64 * 1 + 0] = 4.0          # W1[1][0]: feature 1 -> unit 0
    p[192 + 64 + 0 * 64 + 0] = 1.0  # W2[0][0]
    p[192 + 64 + 4096 + 64 + 0] = 1.0  # W3[0]
    rng = np.random.default_rng(seed)
    p[:192] += (0.05 * rng.standard_normal(192)).astype(np.float32)
    return fpc.fpc_mlp_init(ctx, p)


def _retest(got, C, n, q):
    bad = []
    for (i, j), K in got["sepsets"].items():
        indep, z, st = oracle.ci_test(C, n, i, j, K, q)
        if not indep or len(K) != got["sep_level"][oracle.pair_index(i, j, got["p"])]:
            bad.append((i, j, K, z))
    assert not bad, bad[:5]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_learned_order_keeps_the_skeleton_cfg_small(fpc, ctx, seed, prec):
    X, sem, cfg = semdata.workload("er_p20_n1000_d3", seed)
    _say(f"[learned] er_p20_n1000_d3 seed={seed} prec={prec}")
    C = oracle.corr(X)
    ref = oracle.skeleton(C, cfg["n"], alpha=cfg["alpha"])
    model = _trained_like(fpc, ctx, seed)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=cfg["alpha"], precision=prec, order_model=model)
    assert np.array_equal(got["adj"], ref["adj"])
    assert np.array_equal(got["sep_level"], ref["sep_level"])
    _retest(got, C, cfg["n"], ref["q"])


@pytest.mark.parametrize("p,n,deg,L,prec,graph", [(57, 2000, 5.0, 4, 0, "er"), (130, 3000, 4.0, 3, 1, "er"),
                                                  (90, 3000, 5.0, 6, 1, "er"), (150, 4000, 4.0, 3, 1, "ba"),
                                                  (40, 800, 6.0, -1, 0, "er")])
def test_learned_order_keeps_the_skeleton_mid(fpc, ctx, p, n, deg, L, prec, graph):
    _say(f"[learned mid] p={p} n={n} deg={deg} L={L} prec={prec} graph={graph}")
    sem = semdata.make_sem(p, 21, graph=graph, degree=deg)
    X = semdata.sample(sem, n, 21)
    C = oracle.corr(X)
    ref = oracle.skeleton(C, n, alpha=0.01, max_level=L)
    lex = fpc.fpc_skeleton(ctx, dev(X), alpha=0.01, max_level=L, precision=prec)
    model = _trained_like(fpc, ctx, 21)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=0.01, max_level=L, precision=prec, order_model=model)
    assert np.array_equal(got["adj"], ref["adj"])
    assert np.array_equal(got["sep_level"], ref["sep_level"])
    _retest(got, C, n, ref["q"])
    # same number of tests for edges that survive; the order only moves
    # where each deleted edge's search stops
    for a, b in zip(lex["levels"], got["levels"]):
        assert a["level"] == b["level"] and a["deleted"] == b["deleted"]
    _say(f"  tests lex={lex['total_tests']} learned={got['total_tests']}")


def test_learned_order_full_size(fpc, ctx):
    """The 1000-variable, n = 10000 workload: learned order vs lexicographic
    (both mixed precision) give the same skeleton; sampled separating sets
    re-test as independent in the oracle."""
    X, sem, cfg = semdata.workload("er_p1000_n10000_d4", 0)
    _say("[learned full] er_p1000_n10000_d4")
    Xd = dev(X)
    lex = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1)
    model = _trained_like(fpc, ctx, 0)
    got = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1,
                           order_model=model)
    assert np.array_equal(got["adj"], lex["adj"])
    assert np.array_equal(got["sep_level"], lex["sep_level"])
    C = oracle.corr(X)
    keys = sorted(k for k in got["sepsets"] if got["sep_level"][oracle.pair_index(*k, cfg["p"])] >= 1)
    rng = np.random.default_rng(0)
    pick = [keys[t] for t in rng.choice(len(keys), min(300, len(keys)), replace=False)]
    sub = {"p": cfg["p"], "sep_level": got["sep_level"], "sepsets": {k: got["sepsets"][k] for k in pick}}
    _retest(sub, C, cfg["n"], got["q"])


def _graph_at_level(res, l):
    """The graph a level l (after the first) started from: the final graph
    plus every pair deleted at a level at or below l (the reverse schedule
    runs levels in decreasing order after the first level; deletions apply
    at the end of their level)."""
    p = res["p"]
    A = res["adj"].copy()
    iu, ju = np.triu_indices(p, 1)
    back = (res["sep_kind"] == 1) & (res["sep_level"] >= 0) & (res["sep_level"] <= l)
    A[iu[back], ju[back]] = 1
    A[ju[back], iu[back]] = 1
    return A


@pytest.mark.parametrize("prec", [0, 1])
def test_feature_log_rows(fpc, ctx, prec):
    """FPC_FLAG_LOG_FEATURES: one group serial per edge deleted after the
    first level, in execution order and pair order within a level; its rows
    are the candidates adj n path of the graph the level started from, in id
    order, with features max(|C_ik|, |C_jk|), max(|R_ik|, |R_jk|) (R the
    first-level partial correlations) and deg(k)/(p-1), labelled 1 exactly
    on the recorded separating set.  All three features are recomputed from
    the oracle's correlation matrix and inverse."""
    p, n = 90, 3000
    _say(f"[feature log] p={p} n={n} prec={prec}")
    sem = semdata.make_sem(p, 31, degree=5.0)
    X = semdata.sample(sem, n, 31)
    got = fpc.fpc_skeleton(ctx, dev(X), alpha=0.01, max_level=6, precision=prec,
                           flags=fpc.FPC_FLAG_LOG_FEATURES)
    log = got["log"]
    assert log is not None
    C = oracle.corr(X)
    Om = oracle.inverse(C)
    d = np.sqrt(np.diag(Om))
    R = -Om / np.outer(d, d)
    # expected groups: per executed level after the first, deleted pairs in pair order
    iu, ju = np.triu_indices(p, 1)
    order = []
    for lv in got["levels"][1:]:
        l = lv["level"]
        ks = np.nonzero((got["sep_kind"] == 1) & (got["sep_level"] == l))[0]
        order += [(l, int(iu[k]), int(ju[k])) for k in ks]
    grp = log["group"]
    assert np.all(np.diff(grp) >= 0)  # groups are contiguous and in serial order
    assert len(order) > 0 and grp.max() < len(order)
    lo = np.searchsorted(grp, np.arange(len(order)), side="left")
    hi = np.searchsorted(grp, np.arange(len(order)), side="right")
    graphs = {}
    tol = 1e-5 if prec == 0 else 5e-5
    for g, (l, i, j) in enumerate(order):
        rows = slice(lo[g], hi[g])
        assert np.all(log["level"][rows] == l)
        if l not in graphs:
            graphs[l] = _graph_at_level(got, l)
        A = graphs[l]
        cand = oracle.candidates(A, i, j)
        assert hi[g] - lo[g] == len(cand), (l, i, j)  # an edge with no candidates has no rows
        if not cand:
            continue
        S = set(fpc.sepset_of(got, i, j))
        assert [k for k, y in zip(cand, log["y"][rows]) if y] == sorted(S)
        x = log["x"][rows].astype(np.float64)
        ck = np.maximum(np.abs(C[i, cand]), np.abs(C[j, cand]))
        rk = np.maximum(np.abs(R[i, cand]), np.abs(R[j, cand]))
        dk = A[cand].sum(axis=1) / (p - 1)
        assert np.abs(x[:, 0] - ck).max() <= tol, (l, i, j)
        assert np.abs(x[:, 1] - rk).max() <= tol, (l, i, j)
        assert np.abs(x[:, 2] - dk).max() <= 1e-6, (l, i, j)
    # the log does not depend on the order the level used
    model = _trained_like(fpc, ctx, 3)
    got2 = fpc.fpc_skeleton(ctx, dev(X), alpha=0.01, max_level=6, precision=prec,
                            flags=fpc.FPC_FLAG_LOG_FEATURES, order_model=model)
    assert np.array_equal(got2["log"]["x"], log["x"])
    assert np.array_equal(got2["log"]["group"], log["group"])


def test_trained_ranker_gain_on_held_out_scale_free_graphs(fpc, ctx):
    """What the trained network gains over the lexicographic order, on
    held-out seeds of the scale-free workload it was trained for (BA DAG,
    p = 1000, n = 10000, max_level = 3): the same skeleton, fewer tests.
    Any order can only save tests on the edges a level deletes (a kept
    edge runs all its subsets), about 5% of this workload's tests.  The
    count compared is the tests the order requires (each deleted edge up to
    its first separating set): the tests executed also include the ranks
    past a hit that waves ran before they saw it, which depends on timing."""
    from paper_2109_04626_amd.learned import DEFAULT_MODEL

    model = fpc.fpc_mlp_init(ctx, np.load(DEFAULT_MODEL))
    tl = tb = 0
    for seed in (2000, 2001, 2002):
        X, sem, cfg = semdata.workload("ba_p1000_n10000_m2", seed)
        _say(f"[ranker gain] ba_p1000_n10000_m2 seed={seed}")
        Xd = dev(X)
        a = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1)
        b = fpc.fpc_skeleton(ctx, Xd, alpha=cfg["alpha"], max_level=cfg["max_level"], precision=1,
                             order_model=model)
        assert np.array_equal(a["adj"], b["adj"]) and np.array_equal(a["sep_level"], b["sep_level"])
        tl += sum(x["tests_required"] for x in a["levels"][1:])
        tb += sum(x["tests_required"] for x in b["levels"][1:])
    _say(f"  tests lex={tl} learned={tb} ratio={tb / tl:.4f}")
    assert tb < 0.995 * tl
