"""fpc_first_level_noalloc: the first reverse level with the library's static
workspace, against fpc_first_level (the allocating entry point), through the
C ABI: two calls in a row, the second on a smaller matrix, then a matrix
beyond the workspace.  GPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import semdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _corr(p, n, seed):
    sem = semdata.make_sem(p, seed, degree=4.0)
    X = semdata.sample(sem, n, seed)
    return oracle.corr(X)


def test_first_level_noalloc_matches_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_04626_amd as fpc

    with fpc.Context(0) as ctx:
        q = fpc.fpc_quantile(0.01)
        # the largest size the workspace holds, then a smaller one: the second
        # call must not see the first call's contents (flag, buffers)
        for p, n, seed in [(fpc.FPC_NOALLOC_MAX_P, 4000, 3), (131, 1500, 4)]:
            print(f"[noalloc] p={p} n={n} seed={seed}", flush=True)
            C = torch.from_numpy(_corr(p, n, seed)).cuda()
            r_ref, ind_ref = fpc.fpc_first_level(ctx, C, n, q)
            r = torch.full((p, p), float("nan"), dtype=torch.float64, device="cuda")
            ind = torch.full((p, p), 7, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            fpc.fpc_first_level_noalloc(ctx, C, n, q, r, ind)
            # same kernels, same arithmetic: identical results
            assert torch.equal(r, r_ref)
            assert torch.equal(ind, ind_ref)
            assert 0 < int(ind.sum()) < p * (p - 1)  # both decisions occur
        # a correlation matrix that is not positive definite: reported, and the
        # flag does not stick to the next call
        Cs = np.eye(4)
        Cs[0, 1] = Cs[1, 0] = 0.9
        Cs[1, 2] = Cs[2, 1] = 0.9
        Cs[0, 2] = Cs[2, 0] = -0.9
        r = torch.empty((4, 4), dtype=torch.float64, device="cuda")
        ind = torch.empty((4, 4), dtype=torch.uint8, device="cuda")
        with pytest.raises(fpc.FastPCError) as e:
            fpc.fpc_first_level_noalloc(ctx, torch.from_numpy(Cs).cuda(), 100, 2.5, r, ind)
        assert e.value.code == fpc.FPC_ESINGULAR
        r = torch.empty((40, 40), dtype=torch.float64, device="cuda")
        ind = torch.empty((40, 40), dtype=torch.uint8, device="cuda")
        C = torch.from_numpy(_corr(40, 500, 6)).cuda()
        fpc.fpc_first_level_noalloc(ctx, C, 500, q, r, ind)
        r_ref, ind_ref = fpc.fpc_first_level(ctx, C, 500, q)
        assert torch.equal(r, r_ref) and torch.equal(ind, ind_ref)
        # beyond the static workspace: a clear error, nothing written
        p = fpc.FPC_NOALLOC_MAX_P + 1
        C = torch.from_numpy(_corr(p, 2000, 7)).cuda()
        r = torch.zeros((p, p), dtype=torch.float64, device="cuda")
        ind = torch.zeros((p, p), dtype=torch.uint8, device="cuda")
        with pytest.raises(fpc.FastPCError) as e:
            fpc.fpc_first_level_noalloc(ctx, C, 2000, q, r, ind)
        assert e.value.code == fpc.FPC_ESCRATCH
        assert "static workspace" in str(e.value)
        assert float(r.abs().sum()) == 0.0 and int(ind.sum()) == 0
