"""Slab-recursive PLUQ (Section 4.1, row-major pivot search by halves of
the rows) against the oracle's row-major-order PLUQ, element by element:
L\\U, P, Q, rank and both rank profiles; shapes across several 32-row leaf
slabs with ragged tails, ranks 0 to full, both arithmetic paths; at 8192
the generic input gives the same bits as ffp_pluq (both are then the LU
without pivoting) and the rank-4096 input passes the full-size checks.
"""
import sys

import numpy as np
import pytest

import checks
import workloads as wl

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


CASES = [(1, 1, 1), (5, 9, 3), (32, 32, 32), (33, 40, 20), (64, 64, 0), (100, 70, 70), (130, 200, 90),
         (257, 190, 150), (300, 300, 300), (520, 450, 333)]


@pytest.mark.parametrize("p", [2, 3, 251, 65521, 131071, 8388593, 94906249])
def test_pluq_slab_parity(lib, orc, p):
    import torch
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8, int8_limbs
    rng = np.random.default_rng(p + 23)
    paths = [PATH_FP64] + ([PATH_INT8] if int8_limbs(p) > 0 else [])
    for path in paths:
        for (m, n, r) in CASES:
            r = min(r, m, n)
            A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40))) if (m + n) % 2 else wl.uniform(m, n, p, int(
                rng.integers(1 << 40)))
            want = orc.pluq_rowmajor(A, p)
            note("slab", p, path, m, n, r)
            Ad = dev(A)
            res = lib.pluq_slab(Ad, p, path=path)
            torch.cuda.synchronize()
            assert res.rank == want.rank
            assert np.array_equal(res.P.cpu().numpy(), want.P), (p, path, m, n)
            assert np.array_equal(res.Q.cpu().numpy(), want.Q), (p, path, m, n)
            assert np.array_equal(Ad.cpu().numpy(), want.LU), (p, path, m, n)
            assert np.array_equal(res.rrp.cpu().numpy(), want.rrp)
            assert np.array_equal(res.crp.cpu().numpy(), want.crp)


def test_pluq_slab_special(lib, orc):
    import torch
    p = 65521
    for A in (np.zeros((70, 50), np.int32), np.eye(90, 80, dtype=np.int32),
              np.eye(64, dtype=np.int32)[np.random.default_rng(3).permutation(64)]):
        note("slab special", A.shape)
        want = orc.pluq_rowmajor(A, p)
        Ad = dev(A)
        res = lib.pluq_slab(Ad, p)
        torch.cuda.synchronize()
        assert res.rank == want.rank
        assert np.array_equal(Ad.cpu().numpy(), want.LU)
        assert np.array_equal(res.P.cpu().numpy(), want.P) and np.array_equal(res.Q.cpu().numpy(), want.Q)
    E = torch.zeros((0, 5), dtype=torch.int32, device="cuda")
    assert lib.pluq_slab(E, p).rank == 0


def test_pluq_slab_8192(lib, orc):
    import torch
    p = 131071
    A = wl.make("pluq8192_p131071")
    Ad = dev(A)
    ref = Ad.clone()
    note("slab 8192 uniform")
    r0 = lib.pluq(ref, p)
    res = lib.pluq_slab(Ad, p)
    torch.cuda.synchronize()
    assert res.rank == r0.rank
    assert torch.equal(Ad, ref) and torch.equal(res.P, r0.P) and torch.equal(res.Q, r0.Q)
    del Ad, ref
    B = wl.make("pluq8192_r4096_p131071")
    Bd = dev(B)
    note("slab 8192 rank 4096")
    res = lib.pluq_slab(Bd, p)
    torch.cuda.synchronize()
    r = res.rank
    assert r == 4096
    LU, P, Q = Bd.cpu().numpy(), res.P.cpu().numpy(), res.Q.cpu().numpy()
    assert checks.is_perm(P, 8192) and checks.is_perm(Q, 8192)
    assert checks.structure_ok(LU, r, p) is None
    assert checks.reconstruct_ok(B, LU, P, Q, r, p, exact_limit=0)
    assert checks.reveals_rank_profile_matrix(LU, P, Q, r)
    assert (np.diff(P[:r]) > 0).all() and (np.diff(P[r:]) > 0).all() and (np.diff(Q[r:]) > 0).all()
    assert np.array_equal(res.rrp.cpu().numpy(), P[:r])
