"""z-statistics of the level kernels against the oracle, test by test.

fpc_level_series runs, for one edge and a range of ranks, the same kernels
(per-test Cholesky, shared-prefix pair and triple kernels, both pair-decode
paths of the triple kernel) that a skeleton level runs, and returns every
rank's r and decision.  Each is compared with the oracle's test of the same
conditioning set (the rank-t lexicographic l-subset of the list):

* FP64 kernels: z within 1e-6 relative (absolute for |z| < 1), degenerate
  tests agree, decisions equal z <= q away from exact ties;
* FP32 kernels (on the mixed form's bf16x6 matrix): every test the FP32
  kernel decides itself -- outside the error band of the threshold and not
  ill-conditioned -- takes the oracle's decision; the others go to the FP64
  re-run (whose arithmetic is the FP64 kernels' above).  With the strict
  ill-conditioning threshold (ill_cond_tau < 0) every z decided in FP32 is
  within 1e-4 relative (absolute for |z| < 1); with the default threshold
  the rare ill-conditioned tests decided in FP32 stay within 1e-3.

GPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import semdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_SAMPLES = 10000
Q = oracle.quantile(0.01)
TOL64, TOL32 = 1e-6, 1e-4


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_04626_amd as fpc

    # a dense ER SEM: neighbourhoods overlap, so subsets of a pair's
    # candidates both separate it and leave it dependent
    sem = semdata.make_sem(90, 7, graph="er", degree=8.0)
    X = semdata.sample(sem, N_SAMPLES, 7)
    C = oracle.corr(X)
    und = semdata.true_skeleton(sem)
    moral = und.copy()
    A = sem.W != 0
    for v in range(sem.p):
        pa = np.nonzero(A[:, v])[0]
        for a in pa:
            moral[a, pa] = 1
    np.fill_diagonal(moral, 0)
    ctx = fpc.Context(0)
    C64 = torch.from_numpy(C).cuda()
    C32 = fpc.fpc_corr(ctx, torch.from_numpy(X).cuda(), fpc.FPC_CORR_BF16X6)
    c_err = float(np.abs(C32.cpu().numpy().astype(np.float64) - C).max())
    print(f"[series] bf16x6 matrix entry error {c_err:.2e}", flush=True)
    yield fpc, ctx, C, C64, C32, c_err, moral
    ctx.close()


def pick_edge(C, moral, m, seed):
    """A non-adjacent pair with common moral neighbours, and a list of m
    candidates: the union of their moral neighbourhoods, then random
    nodes, in a shuffled order."""
    rng = np.random.default_rng(seed)
    p = C.shape[0]
    best = None
    for _ in range(200):
        i, j = sorted(rng.choice(p, 2, replace=False))
        if moral[i, j]:
            continue
        common = np.nonzero(moral[i] & moral[j])[0]
        if best is None or len(common) > best[2]:
            best = (int(i), int(j), len(common))
    i, j, _ = best
    nb = [int(v) for v in np.nonzero(moral[i] | moral[j])[0] if v not in (i, j)]
    rest = [v for v in rng.permutation(p).tolist() if v not in nb and v not in (i, j)]
    cand = (nb + rest)[:m]
    rng.shuffle(cand)
    return i, j, cand


def ranges(N, width):
    """Rank windows: the first ranks, a middle run and the ragged tail."""
    if N <= 3 * width:
        return [(0, N)]
    mid = N // 2 - 17
    return [(0, width), (mid, mid + width // 3 + 5), (N - width // 2 - 3, N)]


def compare(fpc, ctx, C, Cd, c_err, l, i, j, cand, lo, hi, kernel, rpw, table, fp32, tag, tau=1e-4):
    r, dec = fpc.fpc_level_series(ctx, Cd, N_SAMPLES, l, i, j, cand, lo, hi, Q, kernel=kernel, ranks_per_wave=rpw,
                                  pair_table=table, band_z=1e-3, c_err=c_err, ill_cond_tau=tau)
    r = r.cpu().numpy()
    dec = dec.cpu().numpy()
    r_o, z_o = oracle.edge_series(C, N_SAMPLES, i, j, cand, l, lo, hi)
    nu = math.sqrt(N_SAMPLES - l - 3)
    with np.errstate(invalid="ignore"):
        z = nu * np.abs(np.arctanh(r))
    deg_o = np.isnan(z_o)
    if not fp32:
        assert np.array_equal(np.isnan(z), deg_o), f"{tag}: degenerate tests differ"
    ok = ~deg_o & ~np.isnan(z)
    if fp32:
        ok &= dec != 2  # decided in FP32; the rest is re-run in FP64
    tol = (TOL32 if tau < 0 else 10 * TOL32) if fp32 else TOL64
    err = np.abs(z[ok] - z_o[ok]) / np.maximum(1.0, np.abs(z_o[ok]))
    worst = float(err.max()) if err.size else 0.0
    assert worst <= tol, f"{tag}: z error {worst:.3e} > {tol:g} at rank {lo + int(np.nonzero(ok)[0][err.argmax()])}"
    indep_o = z_o <= Q
    if fp32:
        # decisions the FP32 kernel takes itself must be the oracle's
        assert not np.any((dec == 1) & ~indep_o), f"{tag}: FP32 independent, oracle dependent"
        assert not np.any((dec == 0) & indep_o), f"{tag}: FP32 dependent, oracle independent"
        assert np.all(dec[deg_o] != 1), f"{tag}: degenerate test decided independent"
    else:
        clear = np.abs(z_o - Q) > 1e-9
        want = np.where(deg_o, 0, indep_o.astype(np.uint8))
        assert np.array_equal(dec[clear | deg_o], want[clear | deg_o]), f"{tag}: FP64 decisions differ"
        assert set(np.unique(dec)) <= {0, 1}
    return worst, int((dec == 1).sum()), int((dec == 2).sum()), len(dec)


# (l, m): lists long enough for several prefixes, tails and both pair paths
CASES = [(2, 40), (3, 40), (4, 36), (5, 30), (6, 26), (7, 22), (8, 20)]


@pytest.mark.parametrize("l,m", CASES)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_level_kernels_z_match_oracle(env, l, m, fp32):
    fpc, ctx, C, C64, C32, c_err, moral = env
    Cd, ce = (C32, c_err) if fp32 else (C64, 0.0)
    i, j, cand = pick_edge(C, moral, m, seed=100 + l)
    N = math.comb(m, l)
    kernels = [(fpc.FPC_KERNEL_AUTO, 0, -1), (fpc.FPC_KERNEL_PER_TEST, 0, -1), (fpc.FPC_KERNEL_PAIR, 0, -1),
               (fpc.FPC_KERNEL_PAIR, 100, -1), (fpc.FPC_KERNEL_GLOBAL, 64, -1)]
    if l >= 3:
        # pair table for every pair, none (arithmetic decode), and part of them;
        # short, ragged work items (100 ranks per wave)
        kernels += [(fpc.FPC_KERNEL_TRIPLE, 0, -1), (fpc.FPC_KERNEL_TRIPLE, 0, 0), (fpc.FPC_KERNEL_TRIPLE, 100, 37),
                    (fpc.FPC_KERNEL_TRIPLE, 64, 0)]
    print(f"[series] l={l} m={m} edge=({i},{j}) N={N} fp32={fp32}", flush=True)
    stats = []
    taus = [1e-4, -1.0] if fp32 else [1e-4]
    for kernel, rpw, table in kernels:
        for lo, hi in ranges(N, 30000):
            for tau in taus:
                tag = f"l={l} kernel={kernel} rpw={rpw} table={table} ranks=[{lo},{hi}) tau={tau}"
                stats.append((tau,) + compare(fpc, ctx, C, Cd, ce, l, i, j, cand, lo, hi, kernel, rpw, table, fp32,
                                              tag, tau))
    for tau in taus:
        st = [x for x in stats if x[0] == tau]
        print(f"  tau={tau}: worst z error {max(x[1] for x in st):.2e}, independent {sum(x[2] for x in st)}, "
              f"left to FP64 {sum(x[3] for x in st)} of {sum(x[4] for x in st)}", flush=True)
    assert sum(x[2] for x in stats) > 0  # the windows hold tests on both sides of the threshold


def test_level_series_kernels_agree_bitwise_in_fp64(env):
    """The per-test and shared-prefix kernels factor the same matrix in a
    different order: their FP64 r agree to rounding, and each kernel is
    deterministic run to run."""
    fpc, ctx, C, C64, C32, c_err, moral = env
    i, j, cand = pick_edge(C, moral, 24, seed=5)
    l = 5
    N = math.comb(24, l)
    a, _ = fpc.fpc_level_series(ctx, C64, N_SAMPLES, l, i, j, cand, 0, N, Q, kernel=fpc.FPC_KERNEL_TRIPLE)
    b, _ = fpc.fpc_level_series(ctx, C64, N_SAMPLES, l, i, j, cand, 0, N, Q, kernel=fpc.FPC_KERNEL_TRIPLE,
                                ranks_per_wave=64, pair_table=0)
    c, _ = fpc.fpc_level_series(ctx, C64, N_SAMPLES, l, i, j, cand, 0, N, Q, kernel=fpc.FPC_KERNEL_PER_TEST)
    a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    assert np.array_equal(a, b)  # same arithmetic whatever the cut and decode path
    assert np.max(np.abs(a - c)) < 1e-12


def test_level_series_rejects_bad_arguments(env):
    fpc, ctx, C, C64, C32, c_err, moral = env
    cand = [3, 4, 5, 6]
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_level_series(ctx, C64, N_SAMPLES, 2, 0, 1, cand, 0, 7, Q)  # C(4,2) = 6 ranks
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_level_series(ctx, C64, N_SAMPLES, 2, 0, 1, [3, 3, 5, 6], 0, 6, Q)  # repeated candidate
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_level_series(ctx, C64, N_SAMPLES, 2, 0, 1, [0, 3, 5, 6], 0, 6, Q)  # i among the candidates
    with pytest.raises(fpc.FastPCError):
        fpc.fpc_level_series(ctx, C64, N_SAMPLES, 2, 0, 1, cand, 0, 6, Q, kernel=fpc.FPC_KERNEL_TRIPLE)  # l < 3
