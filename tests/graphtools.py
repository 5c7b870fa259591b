"""Brute-force graph helpers for tiny graphs (test side only).

Written from the definitions in the paper's preliminaries: a path is a
sequence of distinct adjacent nodes; d-separation blocks a path when a
chain or fork has its middle node in Z, or a collider has neither itself
nor any descendant in Z; X_i and X_j are d-separated by Z when every path
between them is blocked.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_simple_paths(und: np.ndarray, i: int, j: int):
    """Every simple path from i to j in the undirected 0/1 graph ``und``."""
    p = und.shape[0]
    out = []
    stack = [(i, [i])]
    while stack:
        u, path = stack.pop()
        if u == j:
            out.append(path)
            continue
        for v in range(p):
            if und[u, v] and v not in path:
                stack.append((v, path + [v]))
    return out


def brute_candidates(und: np.ndarray, i: int, j: int) -> list[int]:
    """adj(G,i,j) n path(G,i,j): neighbours of i or j (not i, j) that lie
    on some simple path between i and j."""
    p = und.shape[0]
    on_path = set()
    for path in all_simple_paths(und, i, j):
        on_path.update(path[1:-1])
    nb = {k for k in range(p) if k not in (i, j) and (und[i, k] or und[j, k])}
    return sorted(nb & on_path)


def descendants(A: np.ndarray, k: int) -> set[int]:
    """Descendants of k in the DAG A (A[u, v] = edge u -> v), k excluded."""
    out, stack = set(), [k]
    while stack:
        u = stack.pop()
        for v in np.nonzero(A[u])[0]:
            v = int(v)
            if v not in out:
                out.add(v)
                stack.append(v)
    return out


def d_separated(A: np.ndarray, i: int, j: int, Z) -> bool:
    """Brute force over all simple paths of the DAG's skeleton."""
    Z = set(int(z) for z in Z)
    und = (A | A.T).astype(bool)
    for path in all_simple_paths(und, i, j):
        blocked = False
        for a, m, b in zip(path, path[1:], path[2:]):
            collider = A[a, m] and A[b, m]
            if collider:
                if m not in Z and not (descendants(A, m) & Z):
                    blocked = True
                    break
            elif m in Z:
                blocked = True
                break
        if not blocked:
            return False
    return True


def lex_subsets(items, l):
    return list(itertools.combinations(items, l))
