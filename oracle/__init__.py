"""FP64 CPU oracle for the reverse-order pruning PC skeleton (test
infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The library under
``paper_2109_04626_amd/`` never loads it, and it shares no code with it.

The arithmetic lives in ``fastpc_oracle.c`` (plain C, FP64, OpenMP over
the edges of one level); this module is the ctypes marshalling around it
plus small pure-Python pieces (Phase II orientation, the MLP reference).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fastpc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_EINVAL, ORC_ESINGULAR, ORC_EBUDGET, ORC_ENOMEM = 0, 1, 2, 3, 4
_ERRNAMES = {1: "EINVAL", 2: "ESINGULAR", 3: "EBUDGET", 4: "ENOMEM"}

SEP_NONE, SEP_LIST, SEP_ALL_BUT = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {_ERRNAMES.get(code, code)}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()  # compiles when the library is missing or older than its source
        lib = ctypes.CDLL(_LIB)
        d, i, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        lib.orc_ppnd16.restype = d
        lib.orc_ppnd16.argtypes = [d]
        lib.orc_quantile.restype = d
        lib.orc_quantile.argtypes = [d]
        lib.orc_corr.restype = i
        lib.orc_corr.argtypes = [vp, i, i, vp]
        lib.orc_cov_to_corr.restype = i
        lib.orc_cov_to_corr.argtypes = [vp, i, vp]
        lib.orc_pcor.restype = i
        lib.orc_pcor.argtypes = [vp, i, i, i, vp, i, vp]
        lib.orc_pcor_inverse.restype = i
        lib.orc_pcor_inverse.argtypes = [vp, i, i, i, vp, i, vp]
        lib.orc_inverse.restype = i
        lib.orc_inverse.argtypes = [vp, i, vp]
        lib.orc_zstat.restype = d
        lib.orc_zstat.argtypes = [d, i, i]
        lib.orc_candidates.restype = i
        lib.orc_edge_series.restype = i
        lib.orc_edge_series.argtypes = [vp, i, i, i, i, vp, i, i, i64, i64, vp, vp]
        lib.orc_candidates.argtypes = [vp, i, i, i, vp]
        lib.orc_skeleton.restype = vp
        lib.orc_skeleton.argtypes = [vp, i, i, d, i, i, i, i64, i, i]
        lib.orc_skeleton_ex.restype = vp
        lib.orc_skeleton_ex.argtypes = [vp, i, i, d, i, i, i, i64, i, i, i, vp, vp, vp, vp, vp, i]
        lib.orc_result_next_level.restype = i
        lib.orc_result_next_level.argtypes = [vp]
        lib.orc_result_free.argtypes = [vp]
        lib.orc_result_status.restype = i
        lib.orc_result_status.argtypes = [vp]
        lib.orc_result_nlevels.restype = i
        lib.orc_result_nlevels.argtypes = [vp]
        lib.orc_result_total_tests.restype = i64
        lib.orc_result_total_tests.argtypes = [vp]
        lib.orc_result_min_margin.restype = d
        lib.orc_result_min_margin.argtypes = [vp]
        lib.orc_result_adj.argtypes = [vp, vp]
        lib.orc_result_sepsets.restype = i64
        lib.orc_result_sepsets.argtypes = [vp, vp, vp, vp, vp, i64]
        lib.orc_result_levels.argtypes = [vp, vp, vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- pieces
def ppnd16(p: float) -> float:
    """Phi^{-1}(p) by Wichura's AS 241."""
    return _L().orc_ppnd16(float(p))


def quantile(alpha: float) -> float:
    """Threshold Phi^{-1}(1 - alpha/2) of the two-sided Fisher-z test."""
    return _L().orc_quantile(float(alpha))


def corr(X: np.ndarray) -> np.ndarray:
    """Pearson correlation matrix of row-major data (n x p), FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, p = X.shape
    C = np.empty((p, p), dtype=np.float64)
    st = _L().orc_corr(_ptr(X), n, p, _ptr(C))
    if st:
        raise OracleError(st)
    return C


def cov_to_corr(S: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.float64)
    C = np.empty_like(S)
    _L().orc_cov_to_corr(_ptr(S), S.shape[0], _ptr(C))
    return C


def pcor(C: np.ndarray, i: int, j: int, K) -> tuple[float, int]:
    """(r, status) from H = H0 - H1 H2^{-1} H1^T; status 1 = degenerate."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    K = np.ascontiguousarray(np.asarray(K, dtype=np.int32).reshape(-1))
    r = np.zeros(1)
    st = _L().orc_pcor(_ptr(C), C.shape[0], int(i), int(j), _ptr(K), K.size, _ptr(r))
    return float(r[0]), int(st)


def pcor_inverse(C: np.ndarray, i: int, j: int, K) -> tuple[float, int]:
    """(r, status) from the explicit inverse of the (l+2)x(l+2) matrix."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    K = np.ascontiguousarray(np.asarray(K, dtype=np.int32).reshape(-1))
    r = np.zeros(1)
    st = _L().orc_pcor_inverse(_ptr(C), C.shape[0], int(i), int(j), _ptr(K), K.size, _ptr(r))
    return float(r[0]), int(st)


def inverse(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.empty_like(A)
    st = _L().orc_inverse(_ptr(A), A.shape[0], _ptr(out))
    if st:
        raise OracleError(st)
    return out


def zstat(r: float, n: int, l: int) -> float:
    """sqrt(n - l - 3) * |atanh r|."""
    return _L().orc_zstat(float(r), int(n), int(l))


def ci_test(C, n, i, j, K, q) -> tuple[bool, float, int]:
    """(independent, z, status) of one Fisher-z test; degenerate = dependent."""
    r, st = pcor(C, i, j, K)
    if st:
        return False, float("nan"), st
    z = zstat(r, n, len(K))
    return bool(z <= q), z, 0


def edge_series(C, n, i, j, cand, l, r0, r1):
    """(r, z) of the tests ranked r0..r1-1 of the pair (i, j) at level l:
    rank t conditions on the t-th l-subset (lexicographic over positions)
    of the list ``cand``; degenerate tests give NaN."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.int32).reshape(-1))
    r = np.empty(max(int(r1) - int(r0), 1), dtype=np.float64)
    z = np.empty_like(r)
    st = _L().orc_edge_series(_ptr(C), C.shape[0], int(n), int(i), int(j), _ptr(cand), cand.size, int(l), int(r0),
                              int(r1), _ptr(r), _ptr(z))
    if st:
        raise OracleError(ORC_EINVAL)
    k = max(int(r1) - int(r0), 0)
    return r[:k], z[:k]


def candidates(adj: np.ndarray, i: int, j: int) -> list[int]:
    """adj(G,i,j) n path(G,i,j), sorted."""
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    out = np.empty(adj.shape[0], dtype=np.int32)
    m = _L().orc_candidates(_ptr(adj), adj.shape[0], int(i), int(j), _ptr(out))
    return [int(v) for v in out[:m]]


def pair_index(i: int, j: int, p: int) -> int:
    """Row-major index of the unordered pair i<j in the upper triangle."""
    if i > j:
        i, j = j, i
    return i * p - i * (i + 1) // 2 + (j - i - 1)


# ---------------------------------------------------------------- Phase I
def skeleton(C: np.ndarray, n: int, alpha: float | None = None, q: float | None = None,
             max_level: int = -1, reverse: bool = True, stable: bool = True,
             max_tests: int = 0, nthreads: int = 0, verbose: bool = False,
             partial_ok: bool = False, stop_after_levels: int = 0, resume: dict | None = None) -> dict:
    """Phase I (Algorithm 2 if ``reverse`` else Algorithm 1), sampling
    version, on the correlation matrix ``C`` with sample size ``n``.

    Returns a dict with ``adj`` (p x p uint8), ``sep_level``/``sep_kind``
    (per pair i<j, row-major upper triangle), ``sepsets`` ({(i,j): list}
    for LIST kind; ALL_BUT kind means K = V \\ {i,j}), ``levels`` (rows of
    level, eligible edges, tests, deleted, degenerate), ``total_tests``,
    ``min_margin`` (min |z - q| over the tests) and ``q``.  With
    ``partial_ok`` a run stopped by ``max_tests`` returns its counts so far
    (``budget_stopped`` = True; the graph and separating sets are then
    incomplete).

    ``stop_after_levels`` > 0 returns at the level boundary after that many
    levels of this call (``next_level`` >= 0 if the run is not complete);
    ``resume`` continues from such a result (stable schedule): ``adj``,
    ``sep_level``, ``sep_kind``, ``sepsets``, ``next_level``, and its
    ``levels`` rows and ``total_tests``, which the result carries on.
    """
    C = np.ascontiguousarray(C, dtype=np.float64)
    p = C.shape[0]
    if q is None:
        if alpha is None:
            raise ValueError("alpha or q required")
        q = quantile(alpha)
    lib = _L()
    if resume is not None:
        P = p * (p - 1) // 2
        r_adj = np.ascontiguousarray(resume["adj"], dtype=np.uint8)
        r_lev = np.ascontiguousarray(resume["sep_level"], dtype=np.int32)
        r_kind = np.ascontiguousarray(resume["sep_kind"], dtype=np.int8)
        r_off = np.zeros(P + 1, np.int64)
        iu, ju = np.triu_indices(p, 1)
        lists = [resume["sepsets"][(int(iu[k]), int(ju[k]))] if r_kind[k] == SEP_LIST else [] for k in range(P)]
        r_off[1:] = np.cumsum([len(x) for x in lists])
        r_nodes = np.array([v for x in lists for v in x] or [0], dtype=np.int32)
        R = lib.orc_skeleton_ex(_ptr(C), p, int(n), float(q), int(max_level), int(reverse), int(stable),
                                int(max_tests), int(nthreads), int(verbose), int(stop_after_levels),
                                _ptr(r_adj), _ptr(r_lev), _ptr(r_kind), _ptr(r_off), _ptr(r_nodes),
                                int(resume["next_level"]))
    else:
        R = lib.orc_skeleton_ex(_ptr(C), p, int(n), float(q), int(max_level), int(reverse), int(stable),
                                int(max_tests), int(nthreads), int(verbose), int(stop_after_levels),
                                None, None, None, None, None, 0)
    if not R:
        raise MemoryError("oracle allocation failed")
    try:
        st = lib.orc_result_status(R)
        stopped = st == ORC_EBUDGET and partial_ok
        if st and not stopped:
            raise OracleError(st)
        adj = np.empty((p, p), dtype=np.uint8)
        lib.orc_result_adj(R, _ptr(adj))
        P = p * (p - 1) // 2
        lev = np.empty(P, dtype=np.int32)
        kind = np.empty(P, dtype=np.int8)
        off = np.empty(P + 1, dtype=np.int64)
        tot = lib.orc_result_sepsets(R, _ptr(lev), _ptr(kind), _ptr(off), None, 0)
        nodes = np.empty(max(tot, 1), dtype=np.int32)
        lib.orc_result_sepsets(R, None, None, None, _ptr(nodes), tot)
        nl = lib.orc_result_nlevels(R)
        rows = np.empty((nl, 5), dtype=np.int64)
        secs = np.empty(nl, dtype=np.float64)
        lib.orc_result_levels(R, _ptr(rows), _ptr(secs))
        sepsets = {}
        iu, ju = np.triu_indices(p, 1)
        for k in np.nonzero(kind == SEP_LIST)[0]:
            sepsets[(int(iu[k]), int(ju[k]))] = [int(v) for v in nodes[off[k]:off[k + 1]]]
        total = int(lib.orc_result_total_tests(R))
        if resume is not None:  # the levels of the run so far, then this call's
            rows = np.concatenate([np.asarray(resume["levels"], np.int64).reshape(-1, 5), rows])
            secs = np.concatenate([np.asarray(resume.get("level_seconds", np.zeros(len(resume["levels"])))), secs])
            total += int(resume["total_tests"])
        return dict(adj=adj, sep_level=lev, sep_kind=kind, sepsets=sepsets,
                    levels=rows, level_seconds=secs, total_tests=total,
                    min_margin=float(lib.orc_result_min_margin(R)), q=float(q), p=p, n=int(n),
                    budget_stopped=bool(stopped), next_level=int(lib.orc_result_next_level(R)))
    finally:
        lib.orc_result_free(R)


def sepset_of(res: dict, i: int, j: int):
    """The recorded separating set of pair (i, j), or None if kept."""
    if i > j:
        i, j = j, i
    p = res["p"]
    k = pair_index(i, j, p)
    kind = int(res["sep_kind"][k])
    if kind == SEP_NONE:
        return None
    if kind == SEP_ALL_BUT:
        return [v for v in range(p) if v != i and v != j]
    return list(res["sepsets"][(i, j)])


# ---------------------------------------------------------------- Phase II
def orient(adj: np.ndarray, sepset) -> np.ndarray:
    """Phase II of Algorithm 1 (reused by Algorithm 2): CPDAG marks from the
    skeleton ``adj`` and ``sepset(i, j)`` (the separating set of a deleted
    pair, or None).  D[a, b] = 1 when the edge a-b may point a -> b.

    Unshielded triples i - k - j with k not in S(i, j) become i -> k <- j,
    taken in lexicographic (i, j, k) order, skipping a triple that would
    reverse an arrow already placed; then R1-R4 (Phase II listing; R4 in
    Meek's form, the printed one being garbled) are applied in row-major
    sweeps over the undirected edges until a sweep changes nothing.
    Plain O(p^3)-per-sweep loops, for small graphs.
    """
    p = adj.shape[0]
    A = adj.astype(bool)
    D = A.astype(np.uint8).copy()

    def directed(a, b):
        return D[a, b] and not D[b, a]

    def undirected(a, b):
        return D[a, b] and D[b, a]

    for i in range(p):
        for j in range(i + 1, p):
            if A[i, j]:
                continue
            S = sepset(i, j)
            for k in range(p):
                if k in (i, j) or not (A[i, k] and A[j, k]):
                    continue
                if S is not None and k in S:
                    continue
                if not directed(k, i) and not directed(k, j):
                    D[k, i] = 0
                    D[k, j] = 0
    changed = True
    while changed:
        changed = False
        for a in range(p):
            for b in range(p):
                if a == b or not undirected(a, b):
                    continue
                hit = False
                for c in range(p):
                    if c in (a, b):
                        continue
                    if directed(c, a) and not A[c, b]:  # R1
                        hit = True
                    if directed(a, c) and directed(c, b):  # R2
                        hit = True
                for c in range(p):  # R3
                    for d in range(c + 1, p):
                        if len({a, b, c, d}) < 4:
                            continue
                        if (undirected(a, c) and directed(c, b) and undirected(a, d) and directed(d, b)
                                and not A[c, d]):
                            hit = True
                for c in range(p):  # R4
                    for d in range(p):
                        if len({a, b, c, d}) < 4:
                            continue
                        if (undirected(a, c) and not A[c, b] and directed(c, d) and directed(d, b)
                                and A[a, d]):
                            hit = True
                if hit:
                    D[b, a] = 0
                    changed = True
    return D


def dag_v_structures(W: np.ndarray):
    """Unshielded colliders i -> k <- j (i < j non-adjacent) of a DAG."""
    A = W != 0
    p = A.shape[0]
    out = set()
    for k in range(p):
        pa = np.nonzero(A[:, k])[0]
        for x in range(len(pa)):
            for y in range(x + 1, len(pa)):
                i, j = int(pa[x]), int(pa[y])
                if not A[i, j] and not A[j, i]:
                    out.add((min(i, j), max(i, j), k))
    return out


# ---------------------------------------------------------------- ranking MLP reference
MLP_IN, MLP_H = 3, 64


def mlp_unpack(params):
    """Split the flat parameter vector (W1[3][64], b1, W2[64][64], b2, W3, b3)."""
    params = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = params[o:o + MLP_IN * MLP_H].reshape(MLP_IN, MLP_H); o += MLP_IN * MLP_H
    b1 = params[o:o + MLP_H]; o += MLP_H
    W2 = params[o:o + MLP_H * MLP_H].reshape(MLP_H, MLP_H); o += MLP_H * MLP_H
    b2 = params[o:o + MLP_H]; o += MLP_H
    W3 = params[o:o + MLP_H]; o += MLP_H
    b3 = params[o]
    return W1, b1, W2, b2, W3, b3


def mlp_forward(params, X):
    """Logits of the 3 -> 64 -> 64 -> 1 ReLU network, FP64."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(params)
    h1 = np.maximum(np.asarray(X, np.float64) @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def mlp_loss(params, X, y):
    """Mean binary cross-entropy with logits."""
    z = mlp_forward(params, X)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z))) - y * z))


def mlp_grad(params, X, y):
    """Gradient of mlp_loss by the chain rule (backpropagation), FP64."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(params)
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    N = X.shape[0]
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3 + b3
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / N
    dW3 = h2.T @ dz
    db3 = dz.sum()
    da2 = np.outer(dz, W3) * (a2 > 0)
    dW2 = h1.T @ da2
    db2 = da2.sum(0)
    da1 = (da2 @ W2.T) * (a1 > 0)
    dW1 = X.T @ da1
    db1 = da1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])
