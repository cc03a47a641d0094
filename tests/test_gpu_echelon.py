"""Echelon forms, nullspaces and linear solves from the GPU PLUQ, element by
element against the oracle's Gauss-Jordan (which never uses a PLUQ):
reduced row echelon form = oracle RREF; reduced column echelon form =
transposed oracle RREF of A^T; right nullspace = oracle nullspace; left
nullspace = transposed oracle nullspace of A^T; solutions and consistency
flags = oracle solve.  Shapes span several tiles of the triangular solves
with ragged tails, ranks from 0 to full, on both arithmetic paths.
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


CASES = [(1, 1, 1), (5, 7, 3), (40, 33, 0), (64, 64, 64), (130, 70, 55), (200, 260, 199), (333, 290, 290),
         (600, 450, 300)]


@pytest.mark.parametrize("p", [2, 251, 65521, 131071, 8388593])
def test_echelon_nullspace_solve(lib, orc, p):
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8, int8_limbs
    rng = np.random.default_rng(p + 5)
    paths = [PATH_FP64] + ([PATH_INT8] if int8_limbs(p) > 0 else [])
    for path in paths:
        for (m, n, r) in CASES:
            r = min(r, m, n)
            A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
            note("echelon", p, path, m, n, r)
            Ad = dev(A)
            res = lib.pluq(Ad, p, path=path)
            assert res.rank == r
            rk, R, pc = orc.rref(A, p)
            E = host(lib.echelon(res, p, form=0, path=path))
            assert np.array_equal(E, R), ("rref", p, path, m, n, r)
            rkt, Rt, _ = orc.rref(A.T, p)
            C = host(lib.echelon(res, p, form=1, path=path))
            assert np.array_equal(C, Rt.T), ("cref", p, path, m, n, r)
            N = host(lib.nullspace(res, p, side=0, path=path))
            assert np.array_equal(N, orc.nullspace(A, p)), ("right nullspace", p, path, m, n, r)
            NL = host(lib.nullspace(res, p, side=1, path=path))
            assert np.array_equal(NL, orc.nullspace(A.T, p).T), ("left nullspace", p, path, m, n, r)
            Y = rng.integers(0, p, (n, 3)).astype(np.int32)
            B = np.concatenate([orc.fgemm(A, Y, np.zeros((m, 3), np.int32), p),
                                rng.integers(0, p, (m, 2)).astype(np.int32)], 1)
            Xw, okw, _ = orc.solve(A, B, p)
            X, ok = lib.solve(res, dev(B), p, path=path)
            assert np.array_equal(host(ok).astype(bool), okw), ("consistent", p, path, m, n, r)
            assert np.array_equal(host(X), Xw), ("solve", p, path, m, n, r)


def test_echelon_generic_large(lib, orc):
    """A 1500 x 1200 matrix of rank 1100 (the factorisation takes its
    general recursion, the solves their recursive path)."""
    p = 131071
    A = wl.lowrank(1500, 1200, 1100, p, 77)
    Ad = dev(A)
    res = lib.pluq(Ad, p)
    note("echelon large")
    rk, R, pc = orc.rref(A, p)
    assert np.array_equal(host(lib.echelon(res, p, form=0)), R)
    assert np.array_equal(host(lib.nullspace(res, p, side=0)), orc.nullspace(A, p))
