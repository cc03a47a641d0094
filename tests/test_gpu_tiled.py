"""Tile-iterative LU (right-looking, Crout, left-looking; Section 3.1,
Table 1) on the GPU against the oracle: on inputs of generic rank profile
the result is the unique LU without pivoting, equal element by element to
the oracle's PLUQ (whose P and Q are then the identity); on inputs that are
not generic the reported first zero pivot equals the first vanishing leading
principal minor, computed from the oracle's pivots.  Tiles that do and do
not divide the size, rectangular shapes, both arithmetic paths; at 8192 the
three variants equal ffp_pluq bit for bit.
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


def first_zero_pivot(orc, A, p):
    """1 + the index of the first vanishing leading principal minor (0 if none):
    the leading s x s block is nonsingular iff s pivots of R_A lie in it."""
    r, rows, cols = orc.pivots(A, p)
    K = min(A.shape)
    for s in range(1, K + 1):
        if int(np.sum((rows < s) & (cols < s))) < s:
            return s
    return 0


SHAPES = [(64, 64, 16), (130, 130, 64), (200, 200, 64), (257, 257, 100), (300, 180, 64), (180, 300, 48),
          (512, 512, 128), (700, 650, 256)]


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_lu_tiled_parity(lib, orc, variant):
    import torch
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8
    rng = np.random.default_rng(variant + 40)
    for p in (131071, 8388593, 94906249):
        for path in ([PATH_FP64, PATH_INT8] if p < 16711421 else [PATH_FP64]):
            for (m, n, k) in SHAPES:
                A = wl.uniform(m, n, p, int(rng.integers(1 << 40)))
                want = orc.pluq(A, p)
                fz = first_zero_pivot(orc, A, p)
                note("lu_tiled", variant, p, path, m, n, k, fz)
                Ad = dev(A)
                info = lib.lu_tiled(Ad, p, variant, k, path=path)
                torch.cuda.synchronize()
                assert int(info.cpu()[0]) == fz
                if fz == 0:
                    assert np.array_equal(want.P, np.arange(m)) and np.array_equal(want.Q, np.arange(n))
                    assert np.array_equal(Ad.cpu().numpy(), want.LU), (variant, p, path, m, n, k)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_lu_tiled_zero_pivot(lib, orc, variant):
    """Inputs that are not of generic rank profile: uniform mod 3 and mod 251
    (a leading minor vanishes with probability about 1/p per order) report
    the first vanishing leading principal minor; a planted zero leading
    entry stops at index 0."""
    import torch
    seen = 0
    for p, n in ((3, 200), (251, 1000), (251, 700)):
        for seed in (1, 2):
            A = wl.uniform(n, n, p, 500 + seed)
            fz = first_zero_pivot(orc, A, p)
            seen += fz > 0
            note("lu_tiled zero pivot", variant, p, n, seed, fz)
            info = lib.lu_tiled(dev(A), p, variant, 64)
            torch.cuda.synchronize()
            assert int(info.cpu()[0]) == fz, (p, n, seed, fz)
    assert seen >= 2
    B = wl.uniform(200, 200, 65521, 9)
    B[0, 0] = 0
    info = lib.lu_tiled(dev(B), 65521, variant, 64)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 1


def test_lu_tiled_8192_equals_pluq(lib):
    import torch
    p = 131071
    A = dev(wl.make("pluq8192_p131071"))
    ref = A.clone()
    res = lib.pluq(ref, p)
    assert res.rank == 8192
    for variant in (0, 1, 2):
        for k in (512, 1024):
            note("lu_tiled 8192", variant, k)
            B = A.clone()
            info = lib.lu_tiled(B, p, variant, k)
            torch.cuda.synchronize()
            assert int(info.cpu()[0]) == 0
            assert torch.equal(B, ref), (variant, k)
            del B
