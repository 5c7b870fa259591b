"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (closed forms, textbook definitions, library routines,
brute force, invariants).  CPU only."""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
import pytest
import scipy.special

import oracle
import semdata
from tests import graphtools as gt

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------- quantile
def test_ppnd16_matches_library_ndtri():
    ps = np.concatenate([np.linspace(1e-300, 1e-10, 7), np.linspace(1e-9, 1 - 1e-9, 4001),
                         1 - np.logspace(-16, -9, 9)])
    for p in ps:
        ref = scipy.special.ndtri(p)
        got = oracle.ppnd16(p)
        assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)), (p, got, ref)


def test_quantile_matches_high_precision_values():
    """Phi^{-1}(1 - alpha/2) against 50-digit values (golden file)."""
    for line in open(os.path.join(HERE, "golden", "normal_quantiles.txt")):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        alpha, ref = float(line[0]), float(line[1])
        assert oracle.quantile(alpha) == pytest.approx(ref, rel=5e-16, abs=0), alpha


def test_paper_printed_threshold_pins_n_minus_l_minus_3():
    """Power experiment: alpha = 1e-3, N = 1e5, |K| = 1 gives the printed
    threshold 0.01040577 (Sec. 6, power-loss experiment); |K| = 0 would
    give 0.01040572, so the value also fixes the N - |K| - 3 dof."""
    gold = _golden("paper_threshold.txt")
    q = oracle.quantile(gold["alpha"])
    thr = q / math.sqrt(gold["N"] - gold["K"] - 3)
    assert round(thr, 8) == gold["threshold"]
    assert round(q / math.sqrt(gold["N"] - 0 - 3), 8) != gold["threshold"]


def _golden(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split("=")
            out[k.strip()] = float(v) if "." in v or "e" in v else int(v)
    return out


# ------------------------------------------------------------ correlation
def test_corr_matches_numpy_corrcoef():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 7)) @ rng.standard_normal((7, 7)) + 5.0
    C = oracle.corr(X)
    np.testing.assert_allclose(C, np.corrcoef(X, rowvar=False), rtol=0, atol=1e-13)
    assert np.all(np.diag(C) == 1.0)
    assert np.array_equal(C, C.T)


# -------------------------------------------------------- partial correlation
def _residual_pcor(X, i, j, K):
    """Textbook definition: correlation of the residuals of X_i and X_j
    after least-squares regression on [1, X_K]."""
    n = X.shape[0]
    Z = np.column_stack([np.ones(n)] + [X[:, k] for k in K])
    ri = X[:, i] - Z @ np.linalg.lstsq(Z, X[:, i], rcond=None)[0]
    rj = X[:, j] - Z @ np.linalg.lstsq(Z, X[:, j], rcond=None)[0]
    return float(ri @ rj / math.sqrt((ri @ ri) * (rj @ rj)))


def test_pcor_equals_residual_correlation_on_data():
    rng = np.random.default_rng(2)
    p, n = 9, 500
    X = rng.standard_normal((n, p)) @ rng.standard_normal((p, p))
    C = oracle.corr(X)
    for l in range(0, p - 1):
        for _ in range(3):
            i, j, *K = rng.permutation(p)[: l + 2]
            r, st = oracle.pcor(C, i, j, K)
            assert st == 0
            assert r == pytest.approx(_residual_pcor(X, i, j, K), abs=1e-11)


def test_pcor_closed_forms_l0_l1():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 5)) @ rng.standard_normal((5, 5))
    C = oracle.corr(X)
    r0, _ = oracle.pcor(C, 0, 1, [])
    assert r0 == C[0, 1]
    r1, _ = oracle.pcor(C, 0, 1, [2])
    ref = (C[0, 1] - C[0, 2] * C[1, 2]) / math.sqrt((1 - C[0, 2] ** 2) * (1 - C[1, 2] ** 2))
    assert r1 == pytest.approx(ref, rel=1e-13)


def test_pcor_agrees_with_explicit_inverse_reference():
    rng = np.random.default_rng(4)
    p = 40
    A = rng.standard_normal((400, p)) @ rng.standard_normal((p, p))
    C = oracle.corr(A)
    for l in [0, 1, 2, 5, 10, 20, 38]:
        i, j, *K = rng.permutation(p)[: l + 2]
        r1, s1 = oracle.pcor(C, i, j, K)
        r2, s2 = oracle.pcor_inverse(C, i, j, K)
        assert s1 == s2 == 0
        assert r1 == pytest.approx(r2, abs=1e-10)
        # library inverse of the same (l+2) submatrix
        idx = [i, j] + list(K)
        P = np.linalg.inv(C[np.ix_(idx, idx)])
        assert r1 == pytest.approx(-P[0, 1] / math.sqrt(P[0, 0] * P[1, 1]), abs=1e-10)


def test_edge_series_follows_lexicographic_subsets_and_explicit_inverse():
    """Rank t of an edge's level-l tests conditions on the t-th l-subset of
    the list in lexicographic order of positions (itertools' order), and its
    r is the partial correlation of the explicit-inverse reference."""
    rng = np.random.default_rng(11)
    p = 14
    A = rng.standard_normal((300, p)) @ rng.standard_normal((p, p))
    C = oracle.corr(A)
    cand = [9, 2, 13, 5, 7, 11, 3, 8]  # any order: positions index the list
    for l in [0, 1, 2, 3, 5, 8]:
        combos = list(itertools.combinations(range(len(cand)), l))
        r, z = oracle.edge_series(C, 300, 0, 1, cand, l, 0, len(combos))
        assert len(r) == len(combos)
        for t, pos in enumerate(combos):
            K = [cand[a] for a in pos]
            ref, st = oracle.pcor_inverse(C, 0, 1, K)
            assert st == 0 and r[t] == pytest.approx(ref, abs=1e-12)
            P = np.linalg.inv(C[np.ix_([0, 1] + K, [0, 1] + K)])
            assert r[t] == pytest.approx(-P[0, 1] / math.sqrt(P[0, 0] * P[1, 1]), abs=1e-11)
            assert z[t] == pytest.approx(math.sqrt(300 - l - 3) * abs(math.atanh(ref)), rel=1e-12)
        # a window of the series equals that slice of the whole series
        if len(combos) > 4:
            r2, _ = oracle.edge_series(C, 300, 0, 1, cand, l, 2, len(combos) - 1)
            assert np.array_equal(r2, r[2:-1])
    with pytest.raises(oracle.OracleError):
        oracle.edge_series(C, 300, 0, 1, cand, 3, 0, 57)  # C(8,3) = 56 subsets


def test_edge_series_marks_degenerate_tests():
    C = np.eye(5)
    C[2, 3] = C[3, 2] = 1.0  # X2 == X3: any K holding both is singular
    r, z = oracle.edge_series(C, 100, 0, 1, [2, 3, 4], 2, 0, 3)
    # subsets (2,3), (2,4), (3,4)
    assert np.isnan(r[0]) and np.isnan(z[0])
    assert r[1] == 0.0 and r[2] == 0.0


def test_inverse_matches_library():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 30))
    A = A @ A.T + 30 * np.eye(30)
    np.testing.assert_allclose(oracle.inverse(A), np.linalg.inv(A), rtol=1e-12, atol=1e-14)


def test_pcor_degenerate_cases():
    C = np.eye(4)
    C[0, 2] = C[2, 0] = 1.0  # X0 == X2: H2 singular once both are in K
    C[1, 3] = C[3, 1] = 0.3
    _, st = oracle.pcor(C, 1, 3, [0, 2])
    assert st == 1
    # |r| >= 1 -> degenerate
    D = np.ones((2, 2))
    _, st = oracle.pcor(D, 0, 1, [])
    assert st == 1


def test_zstat_is_fisher_z():
    for r, n, l in [(0.1, 1000, 0), (-0.5, 500, 3), (0.026, 10000, 5)]:
        z = oracle.zstat(r, n, l)
        ref = math.sqrt(n - l - 3) * abs(0.5 * math.log((1 + r) / (1 - r)))
        assert z == pytest.approx(ref, rel=1e-14)


# ------------------------------------------------------------- candidates
def test_candidates_match_simple_path_enumeration():
    rng = np.random.default_rng(6)
    for trial in range(60):
        p = int(rng.integers(3, 9))
        und = np.triu(rng.random((p, p)) < rng.uniform(0.2, 0.8), 1)
        und = (und | und.T).astype(np.uint8)
        for i in range(p):
            for j in range(i + 1, p):
                if not und[i, j]:
                    continue
                assert oracle.candidates(und, i, j) == gt.brute_candidates(und, i, j), (trial, i, j)


def test_candidates_on_tree_are_empty_and_on_cycle_are_all():
    p = 6
    path = np.zeros((p, p), np.uint8)
    for a in range(p - 1):
        path[a, a + 1] = path[a + 1, a] = 1
    for a in range(p - 1):
        assert oracle.candidates(path, a, a + 1) == []
    cyc = path.copy()
    cyc[0, p - 1] = cyc[p - 1, 0] = 1
    assert oracle.candidates(cyc, 0, 1) == [2, p - 1]


# ------------------------------------------------ the paper's 4-node example
def _four_node_sem():
    """A DAG with exactly the independences the motivating example lists:
    X1 _|_ X3 | X2 and X3 _|_ X4 | X2 (and supersets): X3 -> X2 -> X1,
    X2 -> X4, X1 -> X4 (0-indexed 2->1->0, 1->3, 0->3)."""
    W = np.zeros((4, 4))
    W[2, 1], W[1, 0], W[1, 3], W[0, 3] = 0.8, 0.7, 0.6, 0.5
    return semdata.SEM(W=W, order=np.array([2, 1, 0, 3]))


@pytest.mark.parametrize("stable", [True, False])
def test_four_node_example_forward_count_is_17(stable):
    """Sec. 3.1: conventional PC performs 17 CI tests on the example."""
    sem = _four_node_sem()
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    res = oracle.skeleton(C, 10**9, alpha=0.01, reverse=False, stable=stable)
    assert res["total_tests"] == 17
    assert np.array_equal(res["adj"], semdata.true_skeleton(sem))
    # the stated independences, with the stated separating sets
    assert oracle.sepset_of(res, 0, 2) == [1]
    assert oracle.sepset_of(res, 2, 3) == [1]


def test_four_node_example_reverse_finds_supersets():
    """Sec. 3.1: reverse order deletes both pairs at stage 2 with the
    supersets {X2, X4} and {X1, X2}."""
    sem = _four_node_sem()
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    res = oracle.skeleton(C, 10**9, alpha=0.01)
    assert np.array_equal(res["adj"], semdata.true_skeleton(sem))
    assert oracle.sepset_of(res, 0, 2) == [1, 3]
    assert oracle.sepset_of(res, 2, 3) == [0, 1]
    assert res["levels"][0].tolist() == [2, 6, 6, 2, 0]


# --------------------------------------------------------- population mode
def _pop(seed, p, degree, graph="er"):
    sem = semdata.make_sem(p, seed, graph=graph, degree=degree)
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    return sem, C


@pytest.mark.parametrize("seed", range(12))
def test_population_recovers_true_skeleton_and_dseparating_sepsets(seed):
    """Oracle version: exact correlations, a nominal N large enough that
    the threshold is far above FP64 noise but far below every nonzero
    partial correlation's z."""
    rng = np.random.default_rng(seed)
    p = int(rng.integers(4, 9))
    sem, C = _pop(100 + seed, p, degree=float(rng.uniform(1.5, 4.0)))
    res = oracle.skeleton(C, 10**9, q=1e-2)
    assert np.array_equal(res["adj"], semdata.true_skeleton(sem))
    A = sem.W != 0
    for i in range(p):
        for j in range(i + 1, p):
            K = oracle.sepset_of(res, i, j)
            if K is None:
                continue
            assert gt.d_separated(A, i, j, K), (i, j, K)


def _dsep_replay(A, p):
    """Algorithm 2 (stable) driven by d-separation in the DAG instead of a
    statistical test: pure Python, brute-force candidates."""
    G = np.ones((p, p), np.uint8) - np.eye(p, dtype=np.uint8)
    seps = {}
    for l in range(p - 2, -1, -1):
        dels = []
        for i in range(p):
            for j in range(i + 1, p):
                if not G[i, j]:
                    continue
                cand = gt.brute_candidates(G, i, j)
                if len(cand) < l:
                    continue
                for S in itertools.combinations(cand, l):
                    if gt.d_separated(A, i, j, S):
                        seps[(i, j)] = (l, list(S))
                        dels.append((i, j))
                        break
        for i, j in dels:
            G[i, j] = G[j, i] = 0
    return G, seps


@pytest.mark.parametrize("seed", range(6))
def test_population_run_equals_dseparation_replay(seed):
    """Oracle version of Algorithm 2: with exact correlations the numeric
    run equals a replay that asks d-separation in the true DAG.  This also
    shows Prop. 2: adjacent pairs are never deleted (kept through stage
    0), non-adjacent ones are deleted at the first stage whose candidate
    subsets contain a separating set."""
    p = 7
    sem, C = _pop(200 + seed, p, degree=3.0)
    res = oracle.skeleton(C, 10**9, q=1e-2)
    A = sem.W != 0
    G, seps = _dsep_replay(A, p)
    assert np.array_equal(res["adj"], G)
    assert np.array_equal(G, semdata.true_skeleton(sem))
    for (i, j), (l, S) in seps.items():
        assert res["sep_level"][oracle.pair_index(i, j, p)] == l
        assert oracle.sepset_of(res, i, j) == S


def test_forward_and_reverse_agree_in_population():
    for seed in range(6):
        sem, C = _pop(300 + seed, 8, degree=3.0)
        a = oracle.skeleton(C, 10**9, q=1e-2)
        b = oracle.skeleton(C, 10**9, q=1e-2, reverse=False)
        assert np.array_equal(a["adj"], b["adj"])


def test_population_cfg1_shape_p20():
    sem, C = _pop(7, 20, degree=3.0)
    res = oracle.skeleton(C, 10**9, q=1e-2)
    assert np.array_equal(res["adj"], semdata.true_skeleton(sem))


# ------------------------------------------------------ first-level identity
def test_first_level_precision_matrix_identity_matches_per_test_cholesky():
    rng = np.random.default_rng(8)
    for p in (3, 6, 15, 30):
        X = rng.standard_normal((10 * p, p)) @ rng.standard_normal((p, p))
        C = oracle.corr(X)
        Om = np.linalg.inv(C)
        for i in range(p):
            for j in range(i + 1, p):
                K = [k for k in range(p) if k not in (i, j)]
                r, st = oracle.pcor(C, i, j, K)
                assert st == 0
                assert r == pytest.approx(-Om[i, j] / math.sqrt(Om[i, i] * Om[j, j]), abs=1e-10)


def test_first_level_decisions_match_explicit_cholesky_loop():
    """The stable run's first level (via Omega) deletes exactly the pairs
    whose per-test Cholesky z is <= q."""
    sem = semdata.make_sem(12, 9, degree=3.0)
    X = semdata.sample(sem, 400, 9)
    C = oracle.corr(X)
    q = oracle.quantile(0.01)
    res = oracle.skeleton(C, 400, q=q, max_level=0)
    p = 12
    first = {(i, j) for i in range(p) for j in range(i + 1, p)
             if oracle.sepset_of(res, i, j) is not None
             and res["sep_level"][oracle.pair_index(i, j, p)] == p - 2}
    want = set()
    for i in range(p):
        for j in range(i + 1, p):
            K = [k for k in range(p) if k not in (i, j)]
            ind, z, st = oracle.ci_test(C, 400, i, j, K, q)
            if ind:
                want.add((i, j))
    assert first == want


# -------------------------------------------------- extreme-threshold counts
def test_q_infinite_deletes_everything_at_first_level():
    sem = semdata.make_sem(15, 1, degree=3.0)
    C = oracle.corr(semdata.sample(sem, 300, 1))
    res = oracle.skeleton(C, 300, q=float("inf"))
    assert res["adj"].sum() == 0
    assert res["total_tests"] == 15 * 14 // 2
    assert np.all(res["sep_level"] == 13)


def test_ties_are_independent():
    """The test keeps H0 (independence) when |F_z| equals the threshold:
    with exactly uncorrelated variables and q = 0 every pair goes at the
    first stage."""
    res = oracle.skeleton(np.eye(6), 100, q=0.0)
    assert res["adj"].sum() == 0 and res["total_tests"] == 15
    fwd = oracle.skeleton(np.eye(6), 100, q=0.0, reverse=False)
    assert fwd["adj"].sum() == 0 and fwd["total_tests"] == 15


def test_q_zero_keeps_complete_graph_with_closed_form_count():
    p = 12
    sem = semdata.make_sem(p, 2, degree=3.0)
    C = oracle.corr(semdata.sample(sem, 300, 2))
    res = oracle.skeleton(C, 300, q=0.0)
    assert res["adj"].sum() == p * (p - 1)
    assert res["total_tests"] == (p * (p - 1) // 2) * 2 ** (p - 2)


# ------------------------------------------------------- search brute force
@pytest.mark.parametrize("seed,p,alpha,degree,n", [(400, 7, 0.05, 3.0, 150), (401, 7, 0.05, 3.0, 150),
                                                   (403, 9, 0.3, 3.0, 150), (1005, 6, 0.3, 1.0, 100),
                                                   (406, 8, 0.2, 1.5, 150)])
def test_search_brute_force_on_tiny_sample(seed, p, alpha, degree, n):
    """For each deleted pair, every lexicographically earlier l-subset of
    its candidates (in the graph frozen at that level) tests dependent and
    the recorded one tests independent; kept pairs test dependent on every
    subset at the last level (stage 0: K empty)."""
    sem = semdata.make_sem(p, seed, degree=degree)
    X = semdata.sample(sem, n, seed)
    C = oracle.corr(X)
    q = oracle.quantile(alpha)
    res = oracle.skeleton(C, n, q=q)
    # replay level by level
    G = np.ones((p, p), np.uint8) - np.eye(p, dtype=np.uint8)
    for l in range(p - 2, -1, -1):
        dels = []
        for i in range(p):
            for j in range(i + 1, p):
                if not G[i, j]:
                    continue
                cand = gt.brute_candidates(G, i, j)
                if len(cand) < l:
                    continue
                K = oracle.sepset_of(res, i, j)
                lvl = res["sep_level"][oracle.pair_index(i, j, p)]
                first = None
                for S in itertools.combinations(cand, l):
                    ind, _, _ = oracle.ci_test(C, n, i, j, list(S), q)
                    if ind:
                        first = list(S)
                        break
                if first is not None:
                    assert lvl == l and K == first
                    dels.append((i, j))
                else:
                    assert lvl != l
        for i, j in dels:
            G[i, j] = G[j, i] = 0
    assert np.array_equal(G, res["adj"])


# --------------------------------------------------------------- invariants
def test_relabelling_permutes_the_skeleton():
    p, n = 30, 2000
    sem = semdata.make_sem(p, 11, degree=3.0)
    X = semdata.sample(sem, n, 11)
    perm = np.random.default_rng(0).permutation(p)
    a = oracle.skeleton(oracle.corr(X), n, alpha=0.01)
    b = oracle.skeleton(oracle.corr(X[:, perm]), n, alpha=0.01)
    assert np.array_equal(a["adj"][np.ix_(perm, perm)], b["adj"])
    assert a["total_tests"] > 0


def test_stable_skeleton_independent_of_thread_count():
    sem = semdata.make_sem(20, 12, degree=3.0)
    X = semdata.sample(sem, 1000, 12)
    C = oracle.corr(X)
    a = oracle.skeleton(C, 1000, alpha=0.01, nthreads=1)
    b = oracle.skeleton(C, 1000, alpha=0.01, nthreads=4)
    assert np.array_equal(a["adj"], b["adj"])
    assert a["sepsets"] == b["sepsets"]
    assert a["total_tests"] == b["total_tests"]


@pytest.mark.parametrize("reverse,max_level", [(True, -1), (True, 3), (False, -1), (False, 2)])
def test_resume_from_every_level_boundary(reverse, max_level):
    """Stopping after k levels and continuing from the boundary state ends
    as the uninterrupted run (skeleton, separating sets, level rows, test
    count), for every k; the boundary's graph is a supergraph of the final
    one (the deleted set only grows)."""
    sem = semdata.make_sem(30, 14, degree=5.0)
    X = semdata.sample(sem, 1500, 14)
    C = oracle.corr(X)
    kw = dict(alpha=0.01, max_level=max_level, reverse=reverse)
    full = oracle.skeleton(C, 1500, **kw)
    assert full["next_level"] == -1
    nlev = len(full["levels"])
    assert nlev >= 3
    for k in range(1, nlev + 1):
        part = oracle.skeleton(C, 1500, stop_after_levels=k, **kw)
        assert len(part["levels"]) == k
        assert np.array_equal(part["levels"], full["levels"][:k])
        assert np.all(part["adj"] >= full["adj"])
        if k < nlev:
            assert part["next_level"] == int(full["levels"][k][0])
        else:
            assert part["next_level"] == -1
        res = oracle.skeleton(C, 1500, resume=part, **kw)
        assert np.array_equal(res["adj"], full["adj"])
        assert np.array_equal(res["sep_level"], full["sep_level"])
        assert np.array_equal(res["sep_kind"], full["sep_kind"])
        assert res["sepsets"] == full["sepsets"]
        assert np.array_equal(res["levels"], full["levels"])
        assert res["total_tests"] == full["total_tests"]
        # and in two more steps of one level each
        mid = oracle.skeleton(C, 1500, resume=part, stop_after_levels=1, **kw)
        if mid["next_level"] >= 0:
            assert int(mid["levels"][-1][0]) == int(full["levels"][k][0])
            res2 = oracle.skeleton(C, 1500, resume=mid, **kw)
            assert res2["sepsets"] == full["sepsets"] and np.array_equal(res2["levels"], full["levels"])


def test_resume_rejects_bad_states():
    C = np.eye(6)
    st = dict(adj=np.ones((6, 6), np.uint8), sep_level=np.full(15, -1, np.int32), sep_kind=np.zeros(15, np.int8),
              sepsets={}, next_level=7, levels=np.zeros((0, 5), np.int64), total_tests=0)
    with pytest.raises(oracle.OracleError):
        oracle.skeleton(C, 100, alpha=0.01, resume=st)  # next level beyond p - 3
    st["next_level"] = 2
    with pytest.raises(oracle.OracleError):
        oracle.skeleton(C, 100, alpha=0.01, resume=st, stable=False)  # stable schedule only


def test_max_level_cap_and_budget():
    sem = semdata.make_sem(40, 13, degree=4.0)
    X = semdata.sample(sem, 2000, 13)
    C = oracle.corr(X)
    res = oracle.skeleton(C, 2000, alpha=0.01, max_level=2)
    lv = [int(r[0]) for r in res["levels"]]
    assert lv[0] == 38 and all(l <= 2 for l in lv[1:])
    with pytest.raises(oracle.OracleError) as e:
        oracle.skeleton(C, 2000, alpha=0.01, max_tests=100)
    assert e.value.code == oracle.ORC_EBUDGET


def test_invalid_inputs():
    C = np.eye(5)
    with pytest.raises(oracle.OracleError):
        oracle.skeleton(C, 6, alpha=0.01)  # n <= p + 1
    S = np.ones((4, 4))
    with pytest.raises(oracle.OracleError) as e:
        oracle.skeleton(S, 100, alpha=0.01)  # singular
    assert e.value.code == oracle.ORC_ESINGULAR
    rng = np.random.default_rng(0)
    X = rng.standard_normal((40, 6))
    X[:, 4] = X[:, 1]  # duplicate column: 1 - R^2 of column 4 is 0
    with pytest.raises(oracle.OracleError) as e:
        oracle.skeleton(oracle.corr(X), 40, alpha=0.01)
    assert e.value.code == oracle.ORC_ESINGULAR
    X[:, 4] = X[:, 1] + 1e-3 * rng.standard_normal(40)  # nearly, not numerically, determined
    oracle.skeleton(oracle.corr(X), 40, alpha=0.01)


def test_batched_goldens_match_their_data_sets():
    """The stored oracle runs of three independent data sets of the
    many-instance workload are for those data sets (p, n, alpha, cap) and
    hold no near-tie that a rounding difference could flip."""
    sys_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    import sys

    if sys_path not in sys.path:
        sys.path.insert(0, sys_path)
    import make_goldens

    cfg = semdata.BATCHED
    for d in make_goldens.BATCHED_GOLDENS:
        g = make_goldens.load(f"batched_data{d}", 0)
        pd = int(np.random.default_rng([cfg["data_seed"] + d, 0xD1]).integers(cfg["p_lo"], cfg["p_hi"] + 1))
        assert g["p"] == pd and g["n"] == cfg["n"] and g["max_level"] == cfg["max_level"]
        assert g["alpha"] == cfg["alpha"] and g["min_margin"] > 1e-9
        assert int(g["levels"][0][0]) == pd - 2
