"""Phase II orientation: the library's host routine against the oracle's
plain implementation, and the oracle against the DAG itself in population
mode (Markov equivalence: same adjacencies and same unshielded colliders;
Prop. 3: forward and reverse runs give the same CPDAG).  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import semdata


def _csr(res):
    """Oracle skeleton result -> the library's (sep_off, sep_nodes) layout."""
    p = res["p"]
    P = p * (p - 1) // 2
    off = np.zeros(P + 1, np.int64)
    nodes = []
    iu, ju = np.triu_indices(p, 1)
    for k in range(P):
        if res["sep_kind"][k] == oracle.SEP_LIST:
            nodes.extend(res["sepsets"][(int(iu[k]), int(ju[k]))])
        off[k + 1] = len(nodes)
    return dict(p=p, adj=res["adj"], sep_level=res["sep_level"], sep_kind=res["sep_kind"], sep_off=off,
                sep_nodes=np.array(nodes, np.int32))


def _sepfun(res):
    return lambda i, j: oracle.sepset_of(res, i, j)


def test_collider_and_chain():
    # 0 -> 2 <- 1 : a v-structure; 3 -> 4 -> 5 : stays undirected
    W = np.zeros((6, 6))
    W[0, 2], W[1, 2], W[3, 4], W[4, 5] = 0.8, 0.7, 0.9, 0.6
    sem = semdata.SEM(W=W, order=np.arange(6))
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    res = oracle.skeleton(C, 10**9, q=1e-2)
    D = oracle.orient(res["adj"], _sepfun(res))
    assert D[0, 2] == 1 and D[2, 0] == 0 and D[1, 2] == 1 and D[2, 1] == 0
    assert D[3, 4] == D[4, 3] == D[4, 5] == D[5, 4] == 1


@pytest.mark.parametrize("seed", range(10))
def test_population_cpdag_has_the_dag_v_structures(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(5, 10))
    sem = semdata.make_sem(p, 500 + seed, degree=float(rng.uniform(2.0, 3.5)))
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    res = oracle.skeleton(C, 10**9, q=1e-2)
    D = oracle.orient(res["adj"], _sepfun(res))
    A = sem.W != 0
    # every arrowhead agrees with the DAG (soundness of the orientation)
    for a in range(p):
        for b in range(p):
            if D[a, b] and not D[b, a]:
                assert A[a, b], (a, b)
    # unshielded colliders of the CPDAG = those of the DAG
    got = set()
    for k in range(p):
        for i in range(p):
            for j in range(i + 1, p):
                if (D[i, k] and not D[k, i] and D[j, k] and not D[k, j] and not res["adj"][i, j]):
                    got.add((i, j, k))
    assert got == oracle.dag_v_structures(sem.W)


@pytest.mark.parametrize("seed", range(6))
def test_forward_and_reverse_give_the_same_cpdag(seed):
    """Prop. 3 (oracle version)."""
    sem = semdata.make_sem(8, 600 + seed, degree=3.0)
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    a = oracle.skeleton(C, 10**9, q=1e-2)
    b = oracle.skeleton(C, 10**9, q=1e-2, reverse=False)
    assert np.array_equal(oracle.orient(a["adj"], _sepfun(a)), oracle.orient(b["adj"], _sepfun(b)))


@pytest.mark.parametrize("seed,p,n,alpha", [(1, 12, 300, 0.05), (2, 15, 500, 0.2), (3, 20, 1000, 0.01),
                                            (4, 30, 800, 0.05), (5, 25, 200, 0.3)])
def test_library_orientation_matches_oracle(seed, p, n, alpha):
    import paper_2109_04626_amd as fpc

    sem = semdata.make_sem(p, 700 + seed, degree=3.0)
    X = semdata.sample(sem, n, 700 + seed)
    res = oracle.skeleton(oracle.corr(X), n, alpha=alpha)
    want = oracle.orient(res["adj"], _sepfun(res))
    got = fpc.fpc_orient(_csr(res))
    assert np.array_equal(got, want)


def _essential_graph(W):
    """Brute force over all orientations of the DAG's skeleton: keep the
    acyclic ones with the DAG's unshielded colliders (Markov equivalence
    theorem, Sec. 2.2); an edge is directed when every member agrees."""
    A = W != 0
    p = A.shape[0]
    edges = [(i, j) for i in range(p) for j in range(i + 1, p) if A[i, j] or A[j, i]]
    want = oracle.dag_v_structures(W)
    members = []
    for bits in range(1 << len(edges)):
        B = np.zeros((p, p))
        for t, (i, j) in enumerate(edges):
            if bits >> t & 1:
                B[i, j] = 1
            else:
                B[j, i] = 1
        # acyclic: repeatedly strip sources
        left, M = set(range(p)), B.copy()
        while True:
            src = [v for v in left if not M[list(left), v].any()]
            if not src:
                break
            for v in src:
                left.discard(v)
        if left:
            continue
        if oracle.dag_v_structures(B) == want:
            members.append(B)
    D = np.zeros((p, p), np.uint8)
    for i, j in edges:
        fwd = all(M[i, j] for M in members)
        bwd = all(M[j, i] for M in members)
        D[i, j] = 0 if bwd else 1
        D[j, i] = 0 if fwd else 1
    return D


@pytest.mark.parametrize("seed", range(12))
def test_population_cpdag_is_the_essential_graph(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(4, 7))
    sem = semdata.make_sem(p, 800 + seed, degree=float(rng.uniform(2.0, 3.5)))
    if int((sem.W != 0).sum()) > 11:
        pytest.skip("too many edges for brute force")
    C = oracle.cov_to_corr(semdata.population_cov(sem))
    res = oracle.skeleton(C, 10**9, q=1e-2)
    assert np.array_equal(oracle.orient(res["adj"], _sepfun(res)), _essential_graph(sem.W))
