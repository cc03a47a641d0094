"""GPU parity at the full workload sizes, through properties that hold at any
size (the oracle would need minutes per run there):

  A == P L U Q (Freivalds, 4 vectors), triangular structure, the pivots are
  the rank profile matrix (Bruhat-type criterion), the pivot order is the
  quadrant order computed by the oracle's index-only ORDER, the rank is the
  constructed one; and sampled rows of the n^3 product recomputed by the
  oracle.  Given P and Q, L and U are unique, so this pins every output bit.
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


def _factor(lib, A, p, path):
    import torch
    Ad = torch.from_numpy(A).cuda()
    res = lib.pluq(Ad, p, path=path)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), res.P.cpu().numpy(), res.Q.cpu().numpy(), res.rank, res


def test_pluq_8192_uniform(lib, orc):
    A = wl.make("pluq8192_p131071")
    p = 131071
    note("pluq 8192 uniform p=131071")
    LU, P, Q, r, res = _factor(lib, A, p, 0)
    assert r == 8192 or r == 8191   # full rank with overwhelming probability
    err = checks.full_check(A, LU, P, Q, r, p, orc.order, exact_limit=0)
    assert err is None, err
    assert np.array_equal(res.rrp.cpu().numpy(), np.sort(P[:r]))


def test_pluq_8192_rank_4096(lib, orc):
    A = wl.make("pluq8192_r4096_p131071")
    p = 131071
    note("pluq 8192 rank 4096 p=131071")
    LU, P, Q, r, res = _factor(lib, A, p, 0)
    assert r == 4096
    err = checks.full_check(A, LU, P, Q, r, p, orc.order, exact_limit=0)
    assert err is None, err
    assert np.array_equal(res.crp.cpu().numpy(), np.sort(Q[:r]))


def test_fgemm_8192_sampled_rows(lib, orc):
    import torch
    p = 131071
    n = 8192
    X = wl.uniform(n, n, p, 102)
    Y = wl.uniform(n, n, p, 103)
    from paper_1402_3501_amd import PATH_FP64
    Z = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    note("fgemm 8192^3")
    lib.fgemm(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), Z, p, path=PATH_FP64)
    got = Z.cpu().numpy()
    rows = np.random.default_rng(1).choice(n, 12, replace=False)
    want = orc.fgemm(X[rows], Y, np.zeros((len(rows), n), np.int32), p, 1, 0)
    assert np.array_equal(got[rows], want)


@pytest.mark.parametrize("side,uplo", [(0, 0), (1, 1)])
def test_ftrsm_8192_sampled(lib, orc, side, uplo):
    """The solves of the 8192 factorisation at full size, both paths (AUTO and
    FP64, bit-identical): a left lower and a right upper 8192-triangle with
    2048 right-hand sides; sampled columns (left) or rows (right) of the
    solution recomputed by the oracle from the same triangle and the same
    sampled right-hand sides (each depends on nothing else)."""
    import torch
    from paper_1402_3501_amd import PATH_AUTO, PATH_FP64
    p = 131071
    d, nv = 8192, 2048
    T = wl.uniform(d, d, p, 301)
    T[np.arange(d), np.arange(d)] = np.maximum(T[np.arange(d), np.arange(d)], 1)
    B = wl.uniform(d, nv, p, 302) if side == 0 else wl.uniform(nv, d, p, 302)
    Td = torch.from_numpy(T).cuda()
    outs = []
    for path in (PATH_AUTO, PATH_FP64):
        note(f"ftrsm {d} side={side} uplo={uplo} path={path}")
        Bd = torch.from_numpy(B).cuda()
        lib.ftrsm(side, uplo, 0, 1, Td, Bd, p, 1, path=path)
        torch.cuda.synchronize()
        outs.append(Bd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    idx = np.random.default_rng(side).choice(nv, 3, replace=False)
    if side == 0:
        want = orc.ftrsm(side, uplo, 0, 1, T, np.ascontiguousarray(B[:, idx]), p, 1)
        assert np.array_equal(outs[0][:, idx], want)
    else:
        want = orc.ftrsm(side, uplo, 0, 1, T, np.ascontiguousarray(B[idx, :]), p, 1)
        assert np.array_equal(outs[0][idx, :], want)
