"""C-ABI library: loads, exports every declared symbol, and its host-only
logic (quantile, candidate sets) agrees with the oracle.  CPU only: no
call here touches a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastpc.h")
LIB = os.path.join(ROOT, "paper_2109_04626_amd", "libfastpc.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python paper_2109_04626_amd/build.py)"
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_binding_lists_the_same_names():
    import paper_2109_04626_amd as fpc

    assert sorted(fpc.EXPORTED) == _declared()
    for name in fpc.EXPORTED:
        assert hasattr(fpc, name), name


def test_quantile_matches_oracle_as241():
    import paper_2109_04626_amd as fpc

    for a in [0.5, 0.2, 0.05, 0.01, 1e-3, 1e-4, 1e-6, 1e-9, 1e-15, 1e-100]:
        assert fpc.fpc_quantile(a) == pytest.approx(oracle.quantile(a), rel=8e-16, abs=0)
    assert np.isnan(fpc.fpc_quantile(0.0)) and np.isnan(fpc.fpc_quantile(1.0))


def _random_graph(rng, p, dens):
    u = np.triu(rng.random((p, p)) < dens, 1)
    return (u | u.T).astype(np.uint8)


@pytest.mark.parametrize("p,dens", [(5, 0.5), (8, 0.4), (12, 0.25), (30, 0.1), (60, 0.06), (200, 0.02), (530, 0.006)])
def test_candidate_sets_match_oracle_bfs(p, dens):
    import paper_2109_04626_amd as fpc

    rng = np.random.default_rng(p)
    for _ in range(4):
        adj = _random_graph(rng, p, dens)
        ei, ej, off, nodes = fpc.fpc_candidates(adj)
        iu, ju = np.nonzero(np.triu(adj, 1))
        assert np.array_equal(ei, iu) and np.array_equal(ej, ju)
        for e in range(len(ei)):
            got = nodes[off[e]:off[e + 1]].tolist()
            assert got == oracle.candidates(adj, int(ei[e]), int(ej[e])), (e, ei[e], ej[e])


def test_candidate_sets_take_any_nonzero_entry_as_an_edge():
    import paper_2109_04626_amd as fpc

    rng = np.random.default_rng(7)
    p = 37  # rows of eight entries plus a ragged tail
    adj = _random_graph(rng, p, 0.2)
    w = np.triu(rng.choice(np.array([1, 2, 3, 128, 255], np.uint8), size=(p, p)), 1)
    heavy = (adj * (w + w.T)).astype(np.uint8)
    ref = fpc.fpc_candidates(adj)
    got = fpc.fpc_candidates(heavy)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("p,dens", [(777, 0.008), (1003, 0.004)])
def test_candidate_sets_of_large_graphs(p, dens):
    """Graphs of 512 nodes or more take the row-parallel adjacency build:
    edge order as numpy lists it, any nonzero byte an edge, and sampled sets
    equal to the oracle's breadth-first search."""
    import paper_2109_04626_amd as fpc

    rng = np.random.default_rng(p)
    adj = _random_graph(rng, p, dens)
    w = np.triu(rng.choice(np.array([1, 2, 3, 128, 255], np.uint8), size=(p, p)), 1)
    heavy = (adj * (w + w.T)).astype(np.uint8)
    ei, ej, off, nodes = fpc.fpc_candidates(heavy)
    iu, ju = np.nonzero(np.triu(adj, 1))
    assert np.array_equal(ei, iu) and np.array_equal(ej, ju)
    for e in rng.choice(len(ei), size=min(150, len(ei)), replace=False):
        got = nodes[off[e]:off[e + 1]].tolist()
        assert got == oracle.candidates(adj, int(ei[e]), int(ej[e])), (e, ei[e], ej[e])


def test_candidate_sets_on_complete_and_empty_graphs():
    import paper_2109_04626_amd as fpc

    p = 7
    full = (np.ones((p, p)) - np.eye(p)).astype(np.uint8)
    ei, ej, off, nodes = fpc.fpc_candidates(full)
    assert len(ei) == p * (p - 1) // 2
    assert np.all(np.diff(off) == p - 2)
    ei, ej, off, nodes = fpc.fpc_candidates(np.zeros((p, p), np.uint8))
    assert len(ei) == 0 and off.tolist() == [0]


def test_candidate_sets_reject_asymmetric_input():
    import paper_2109_04626_amd as fpc

    a = np.zeros((3, 3), np.uint8)
    a[0, 1] = 1
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_candidates(a)
