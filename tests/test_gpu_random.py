"""Seeded random campaign: PLUQ, fgemm and the batched call on random shapes,
primes, input structures (uniform, low rank, sparse, zero rows and columns,
entries in {0, 1, 2}) and every path a prime allows, each output compared
with the oracle's element by element."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

PRIMES = [2, 3, 5, 251, 257, 32749, 65521, 131071, 1048573, 8388593, 94906249]


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _paths(p):
    from paper_1402_3501_amd import PATH_AUTO, PATH_FP64, PATH_INT8, int8_limbs
    return [PATH_AUTO, PATH_FP64] + ([PATH_INT8] if int8_limbs(p) > 0 else [])


def _matrix(rng, p, m, n):
    kind = int(rng.integers(0, 5))
    if kind == 0:
        return rng.integers(0, p, (m, n)).astype(np.int32)
    if kind == 1:
        r = int(rng.integers(0, min(m, n) + 1))
        return wl.lowrank(m, n, r, p, int(rng.integers(1, 1 << 30))) if r > 0 else np.zeros((m, n), np.int32)
    if kind == 2:
        return (rng.integers(0, p, (m, n)) * (rng.random((m, n)) < 0.05)).astype(np.int32)
    if kind == 3:
        A = rng.integers(0, p, (m, n)).astype(np.int32)
        A[rng.random(m) < 0.3, :] = 0
        A[:, rng.random(n) < 0.3] = 0
        return A
    return rng.integers(0, min(p, 3), (m, n)).astype(np.int32)


@pytest.mark.parametrize("seed", [1, 2])
def test_random_pluq_and_fgemm(lib, orc, seed):
    import torch
    rng = np.random.default_rng(1000 + seed)
    for case in range(40):
        p = int(rng.choice(PRIMES))
        m, n = int(rng.integers(1, 700)), int(rng.integers(1, 700))
        A = _matrix(rng, p, m, n)
        want = orc.pluq(A, p, selfcheck=False)
        for path in _paths(p):
            note("random pluq", seed, case, p, path, m, n)
            Ad = torch.from_numpy(A).cuda()
            res = lib.pluq(Ad, p, path=path)
            assert res.rank == want.rank, (seed, case)
            assert np.array_equal(Ad.cpu().numpy(), want.LU), (seed, case, path)
            assert np.array_equal(res.P.cpu().numpy(), want.P) and np.array_equal(res.Q.cpu().numpy(), want.Q)
        mm, nn, kk = int(rng.integers(1, 600)), int(rng.integers(1, 600)), int(rng.integers(1, 3000))
        ta, tb = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        X = rng.integers(0, p, (kk, mm) if ta else (mm, kk)).astype(np.int32)
        Y = rng.integers(0, p, (nn, kk) if tb else (kk, nn)).astype(np.int32)
        Z = rng.integers(0, p, (mm, nn)).astype(np.int32)
        al, be = int(rng.integers(0, p)), int(rng.integers(0, p))
        wz = orc.fgemm(X, Y, Z, p, al, be, bool(ta), bool(tb))
        for path in _paths(p):
            note("random fgemm", seed, case, p, path, mm, nn, kk, ta, tb)
            Zd = torch.from_numpy(Z).cuda()
            lib.fgemm(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), Zd, p, al, be, bool(ta), bool(tb),
                      path=path)
            assert np.array_equal(Zd.cpu().numpy(), wz), (seed, case, path)


def test_random_batches(lib, orc):
    import torch
    rng = np.random.default_rng(77)
    for case in range(8):
        p = int(rng.choice(PRIMES))
        cnt = int(rng.integers(1, 40))
        bm = rng.integers(0, 300, cnt).astype(np.int32)
        bn = rng.integers(0, 300, cnt).astype(np.int32)
        mats = [_matrix(rng, p, int(bm[i]), int(bn[i])) if bm[i] * bn[i] else np.zeros((bm[i], bn[i]), np.int32)
                for i in range(cnt)]
        off = np.concatenate([[0], np.cumsum(bm.astype(np.int64) * bn)[:-1]]).astype(np.int64)
        Ab = np.concatenate([x.ravel() for x in mats] + [np.zeros(1, np.int32)]).astype(np.int32)
        note("random batch", case, p, cnt)
        Abd = torch.from_numpy(Ab).cuda()
        rb = lib.pluq_batched(torch.from_numpy(bm).cuda(), torch.from_numpy(bn).cuda(), Abd,
                              torch.from_numpy(off).cuda(), p)
        LU, P, Q, rk = Abd.cpu().numpy(), rb.P.cpu().numpy(), rb.Q.cpu().numpy(), rb.rank.cpu().numpy()
        po = np.concatenate([[0], np.cumsum(bm)[:-1]]).astype(np.int64)
        qo = np.concatenate([[0], np.cumsum(bn)[:-1]]).astype(np.int64)
        for i in range(cnt):
            mi, ni = int(bm[i]), int(bn[i])
            want = orc.pluq(Ab[off[i]:off[i] + mi * ni].reshape(mi, ni), p, selfcheck=False)
            assert rk[i] == want.rank, (case, i)
            assert np.array_equal(LU[off[i]:off[i] + mi * ni].reshape(mi, ni), want.LU), (case, i)
            assert np.array_equal(P[po[i]:po[i] + mi], want.P) and np.array_equal(Q[qo[i]:qo[i] + ni], want.Q)
