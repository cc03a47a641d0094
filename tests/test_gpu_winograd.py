"""Strassen-Winograd layer over fgemm: bit-exact against the oracle's plain
product (the definition of C <- alpha op(A) op(B) + beta C mod p), on both
arithmetic paths, for forced numbers of levels on shapes that reach the
1 x 1 base, odd dimensions at every level (peeling), transposed operands and
general alpha / beta; at 8192 and 16384 the Winograd product equals the plain
one bit for bit (the plain one is pinned against the oracle by sampled rows
in the full-size tests) and sampled rows equal the oracle's.
"""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


SHAPES = [(2, 2, 2), (3, 5, 7), (8, 8, 8), (33, 17, 65), (130, 70, 101), (257, 300, 129), (512, 384, 640)]


@pytest.mark.parametrize("p", [2, 251, 65521, 131071, 8388593, 94906249])
def test_winograd_parity(lib, orc, p):
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8, int8_limbs
    rng = np.random.default_rng(p + 99)
    paths = [PATH_FP64] + ([PATH_INT8] if int8_limbs(p) > 0 else [])
    for path in paths:
        for (m, n, k) in SHAPES:
            big = m * n * k > 2 ** 24
            for levels in ((1, 2) if big else (1, 2, 3, 6 if min(m, n, k) < 64 else 4)):
                for ta, tb in ([(0, 0)] if big else [(0, 0), (1, 1)] if levels < 3 else [(0, 0), (1, 0), (0, 1)]):
                    A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
                    B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
                    C = rng.integers(0, p, (m, n)).astype(np.int32)
                    alpha, beta = [(1, 0), (p - 1, 1), (int(rng.integers(0, p)), int(rng.integers(0, p)))][
                        (m + levels + ta) % 3]
                    note("wino", p, path, m, n, k, levels, ta, tb, alpha, beta)
                    want = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
                    Cd = dev(C)
                    lib.fgemm_wino(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=path, levels=levels)
                    assert np.array_equal(host(Cd), want), (p, path, m, n, k, levels, ta, tb, alpha, beta)


def test_winograd_worst_case_magnitudes(lib, orc):
    """All entries p - 1 (the largest centred magnitudes) with a long inner
    dimension: the additions reduce, so the block products stay exact."""
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8
    for p, path in [(94906249, PATH_FP64), (8388593, PATH_INT8), (8388593, PATH_FP64)]:
        m, n, k = 96, 80, 1200
        A = np.full((m, k), p - 1, np.int32)
        B = np.full((k, n), p - 1, np.int32)
        A[::3, ::2] = 1
        C = np.zeros((m, n), np.int32)
        note("wino worst", p, path)
        want = orc.fgemm(A, B, C, p)
        Cd = dev(C)
        lib.fgemm_wino(dev(A), dev(B), Cd, p, path=path, levels=3)
        assert np.array_equal(host(Cd), want)


@pytest.mark.parametrize("n,p", [(8192, 131071), (16384, 8388593)])
def test_winograd_full_size_equals_plain(lib, orc, n, p):
    import torch
    from paper_1402_3501_amd import PATH_AUTO, WINO_AUTO
    X = wl.uniform(n, n, p, 401)
    Y = wl.uniform(n, n, p, 402)
    Xd, Yd = dev(X), dev(Y)
    plain = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    lib.fgemm(Xd, Yd, plain, p, path=PATH_AUTO)
    for levels in (1, 2, WINO_AUTO):
        note("wino full", n, p, levels)
        Z = torch.zeros((n, n), dtype=torch.int32, device="cuda")
        lib.fgemm_wino(Xd, Yd, Z, p, path=PATH_AUTO, levels=levels)
        torch.cuda.synchronize()
        assert torch.equal(Z, plain), levels
        del Z
    rows = np.random.default_rng(n).choice(n, 3, replace=False)
    got = plain[torch.from_numpy(rows).cuda()].cpu().numpy()
    for t, i in enumerate(rows):
        want = orc.fgemm(X[i:i + 1], Y, np.zeros((1, n), np.int32), p)
        assert np.array_equal(got[t:t + 1], want), i
