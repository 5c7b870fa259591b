"""Seeded synthetic inputs: random DAGs, linear-Gaussian SEM weights, data.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds input generation only -- graph topology, edge weights, samples drawn
from the structural equations, bootstrap resampling and the population
covariance of the SEM -- and none of the skeleton method's arithmetic
(no correlation matrix, no partial correlation, no test statistic).

Workload shapes follow the paper's simulation section (a fixed variable
order, a Bernoulli edge indicator per ordered pair, a random coefficient
per edge, independent N(0,1) noise) with the sizes and weight law of the
benchmark configurations:

* Erdos-Renyi DAG in a uniformly random topological order, each of the
  p(p-1)/2 ordered pairs an edge with probability d/(p-1), so the expected
  total degree of a node is d;
* Barabasi-Albert undirected graph (m=2, seed graph a triangle), oriented
  by a uniformly random topological order;
* weights w = s*u, u ~ U[0.5, 1.5], s = +-1 equiprobable (the paper's own
  law U([-0.8,-0.2] u [0.2,0.8]) is available as ``weight_law="paper"``);
* X_j = sum_{i in pa(j)} w_ij X_i + eps_j, eps ~ N(0,1), no rescaling.

Everything is driven by numpy's PCG64 generator seeded with the config
seed, so a seed fixes graph, weights and data on every platform.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "SEM",
    "er_dag",
    "ba_dag",
    "paper_dag",
    "draw_weights",
    "sample",
    "population_cov",
    "make_sem",
    "bootstrap_rows",
    "bootstrap_index",
    "true_skeleton",
    "batched_workload",
]


@dataclasses.dataclass
class SEM:
    """A linear-Gaussian structural equation model.

    ``W[i, j]`` is the coefficient of the edge i -> j (zero if absent);
    ``order`` is a topological order of the nodes.
    """

    W: np.ndarray
    order: np.ndarray

    @property
    def p(self) -> int:
        return self.W.shape[0]


def _topo_orient(und: np.ndarray, order: np.ndarray) -> np.ndarray:
    """Orient an undirected 0/1 adjacency by a topological order."""
    p = und.shape[0]
    pos = np.empty(p, dtype=np.int64)
    pos[order] = np.arange(p)
    i, j = np.nonzero(np.triu(und, 1))
    a = np.zeros((p, p), dtype=bool)
    fwd = pos[i] < pos[j]
    a[i[fwd], j[fwd]] = True
    a[j[~fwd], i[~fwd]] = True
    return a


def er_dag(p: int, degree: float, rng: np.random.Generator):
    """Erdos-Renyi DAG with expected total degree ``degree``.

    Returns (A, order) with A[i, j] = True for an edge i -> j.
    """
    order = rng.permutation(p)
    prob = 0.0 if p < 2 else min(1.0, degree / (p - 1))
    u = rng.random((p, p))
    und = np.triu(u < prob, 1)
    und = und | und.T
    return _topo_orient(und, order), order


def ba_dag(p: int, m: int, rng: np.random.Generator):
    """Barabasi-Albert graph (m edges per new node, seed triangle),
    oriented by a uniformly random topological order."""
    if p < 3:
        raise ValueError("BA graph needs p >= 3")
    und = np.zeros((p, p), dtype=bool)
    und[0, 1] = und[1, 0] = und[0, 2] = und[2, 0] = und[1, 2] = und[2, 1] = True
    # repeated-node list: each node appears once per incident edge
    targets = [0, 0, 1, 1, 2, 2]
    for v in range(3, p):
        chosen: set[int] = set()
        while len(chosen) < min(m, v):
            chosen.add(targets[int(rng.integers(len(targets)))])
        for t in sorted(chosen):
            und[v, t] = und[t, v] = True
            targets.extend((v, t))
    order = rng.permutation(p)
    return _topo_orient(und, order), order


def paper_dag(p: int, rng: np.random.Generator, avg_neighbors: float = 5.0,
              n_hubs: int = 2, hub_neighbors: int = 10):
    """The paper's simulation shape: a fixed order 0..p-1, Bernoulli edges
    giving ``avg_neighbors`` neighbours on average, plus ``n_hubs`` hubs
    with ``hub_neighbors`` neighbours each."""
    order = np.arange(p)
    prob = min(1.0, avg_neighbors / (p - 1))
    und = np.triu(rng.random((p, p)) < prob, 1)
    und = und | und.T
    hubs = rng.choice(p, size=min(n_hubs, p), replace=False)
    for h in hubs:
        others = np.setdiff1d(np.arange(p), [h])
        nb = rng.choice(others, size=min(hub_neighbors, p - 1), replace=False)
        und[h, :] = False
        und[:, h] = False
        und[h, nb] = und[nb, h] = True
    return _topo_orient(und, order), order


def draw_weights(A: np.ndarray, rng: np.random.Generator,
                 weight_law: str = "baseline") -> np.ndarray:
    """Edge coefficients for the 0/1 DAG ``A``."""
    p = A.shape[0]
    if weight_law == "baseline":
        mag = rng.uniform(0.5, 1.5, size=(p, p))
    elif weight_law == "paper":
        mag = rng.uniform(0.2, 0.8, size=(p, p))
    else:
        raise ValueError(weight_law)
    sign = np.where(rng.random((p, p)) < 0.5, -1.0, 1.0)
    return np.where(A, sign * mag, 0.0)


def make_sem(p: int, seed: int, graph: str = "er", degree: float = 3.0,
             weight_law: str = "baseline", ba_m: int = 2) -> SEM:
    """Graph + weights for one seeded configuration."""
    rng = np.random.default_rng(seed)
    if graph == "er":
        A, order = er_dag(p, degree, rng)
    elif graph == "ba":
        A, order = ba_dag(p, ba_m, rng)
    elif graph == "paper":
        A, order = paper_dag(p, rng)
    else:
        raise ValueError(graph)
    W = draw_weights(A, rng, weight_law)
    return SEM(W=W, order=np.asarray(order))


def sample(sem: SEM, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n samples (rows) from the SEM, row-major n x p.

    Nodes are filled in topological order; the noise stream is seeded
    independently of the graph stream so that changing n keeps the graph.
    """
    rng = np.random.default_rng([seed, 0x5EED])
    p = sem.p
    X = np.zeros((n, p), dtype=np.float64)
    eps = rng.standard_normal((n, p))
    for j in sem.order:
        pa = np.nonzero(sem.W[:, j])[0]
        X[:, j] = eps[:, j]
        if pa.size:
            X[:, j] += X[:, pa] @ sem.W[pa, j]
    return np.ascontiguousarray(X.astype(dtype))


def population_cov(sem: SEM) -> np.ndarray:
    """Exact covariance of the SEM: X = E (I - W)^{-1} with Cov(E) = I."""
    p = sem.p
    M = np.linalg.inv(np.eye(p) - sem.W)
    return M.T @ M


def bootstrap_index(n: int, seed: int) -> np.ndarray:
    """Row indices of a bootstrap resample: n draws with replacement."""
    rng = np.random.default_rng([seed, 0xB007])
    return rng.integers(0, n, size=n).astype(np.int32)


def bootstrap_rows(X: np.ndarray, seed: int) -> np.ndarray:
    """Rows drawn with replacement (same n)."""
    return np.ascontiguousarray(X[bootstrap_index(X.shape[0], seed)])


def true_skeleton(sem: SEM) -> np.ndarray:
    """Undirected 0/1 adjacency of the DAG."""
    a = sem.W != 0
    return (a | a.T).astype(np.uint8)


# ---------------------------------------------------------------- workloads
# Named synthetic workloads (shapes of the benchmark configurations).
WORKLOADS = {
    # plain method, FP64, all levels
    "er_p20_n1000_d3": dict(p=20, n=1000, graph="er", degree=3.0, x_dtype="f64", alpha=0.01, max_level=-1),
    # dense small graph, FP32 tests with FP64 recheck
    "er_p95_n5000_d12": dict(p=95, n=5000, graph="er", degree=12.0, x_dtype="f64", alpha=0.01, max_level=6),
    # dense p = 95 graph whose level sequence after the first runs 6, 5, 4, 3, 2, 1, 0 (the paper's
    # weight law keeps the variances bounded, so true edges survive level 6)
    "er_p95_n20000_d8_paper": dict(p=95, n=20000, graph="er", degree=8.0, x_dtype="f64", alpha=0.01, max_level=6,
                                   weight_law="paper"),
    # sparse large graph, X in FP32
    "er_p1000_n10000_d4": dict(p=1000, n=10000, graph="er", degree=4.0, x_dtype="f32", alpha=0.01, max_level=5),
    # scale-free graph
    "ba_p1000_n10000_m2": dict(p=1000, n=10000, graph="ba", degree=0.0, x_dtype="f32", alpha=0.01, max_level=3),
    # the paper's simulation shape (5 neighbours on average, two hubs of 10,
    # its weight law, alpha 1e-3); n is not stated there
    "paper_p95_n10000": dict(p=95, n=10000, graph="paper", degree=0.0, x_dtype="f64", alpha=0.001, max_level=6,
                             weight_law="paper"),
}


def workload(name: str, seed: int, **over):
    """(X, sem, cfg) for a named workload; ``over`` overrides cfg keys."""
    cfg = dict(WORKLOADS[name])
    cfg.update(over)
    sem = make_sem(cfg["p"], seed, graph=cfg["graph"], degree=cfg["degree"],
                   weight_law=cfg.get("weight_law", "baseline"))
    X = sample(sem, cfg["n"], seed, dtype=np.float32 if cfg["x_dtype"] == "f32" else np.float64)
    return X, sem, cfg


# Many instances in one call: bootstrap resamples of one data set plus
# independent data sets of uneven size (ER DAGs, expected degree 6, n=5000).
BATCHED = dict(n=5000, degree=6.0, x_dtype="f32", alpha=0.01, max_level=4, base_p=500, n_boot=64, n_data=16,
               p_lo=50, p_hi=2000, base_seed=3000, boot_seed=3001, data_seed=3100)


def batched_workload(n_boot: int | None = None, n_data: int | None = None, scale: float = 1.0, **over):
    """(base X, bootstrap row-index arrays, [independent X], cfg).

    The base data set has ``base_p`` variables (seed ``base_seed``); resample
    b uses seed ``boot_seed + b``; data set d has p uniform in
    [p_lo, p_hi] (drawn from seed ``data_seed + d``) and seed
    ``data_seed + d``.  ``scale`` shrinks every p (and n) for small tests.
    """
    cfg = dict(BATCHED)
    cfg.update(over)
    nb = cfg["n_boot"] if n_boot is None else n_boot
    nd = cfg["n_data"] if n_data is None else n_data
    dt = np.float32 if cfg["x_dtype"] == "f32" else np.float64
    n = max(8, int(round(cfg["n"] * scale)))
    bp = max(4, int(round(cfg["base_p"] * scale)))
    base = sample(make_sem(bp, cfg["base_seed"], degree=cfg["degree"]), n, cfg["base_seed"], dtype=dt)
    boots = [bootstrap_index(n, cfg["boot_seed"] + b) for b in range(nb)]
    datas = []
    for d in range(nd):
        seed = cfg["data_seed"] + d
        pd = int(np.random.default_rng([seed, 0xD1]).integers(cfg["p_lo"], cfg["p_hi"] + 1))
        pd = max(4, min(n - 3, int(round(pd * scale))))
        datas.append(sample(make_sem(pd, seed, degree=cfg["degree"]), n, seed, dtype=dt))
    cfg["n"] = n
    cfg["base_p"] = bp
    return base, boots, datas, cfg
