"""Pins of the oracle's echelon forms, nullspace and solver against what the
mathematics fixes (no use of the oracle's PLUQ, and no retyped formula):

* the reduced row echelon form R of A is the only matrix that (i) has its
  pivot columns ascending with R[:, pivcols] = I, (ii) has the leading entry
  of row t in column pivcols[t], and (iii) spans the row space of A with the
  same rank: A = A[:, pivcols] R, checked with Python big integers;
* a nullspace basis that is the identity on the non-pivot rows is unique:
  A N = 0 and N[free] = I;
* the solution that is zero off the pivot columns is unique: A x = b and
  x[free] = 0; a column of B is inconsistent exactly when appending it
  raises the rank (ranks by minor enumeration on small inputs);
* exhaustive small cases over F_2 and F_3 against a brute-force search of
  the row space.
"""
import itertools

import numpy as np
import pytest

import workloads as wl

PRIMES = [2, 3, 5, 251, 65521, 131071, 8388593]


def _mul(A, B, p):
    return (A.astype(object).dot(B.astype(object))) % p


def _rref_characterised(A, R, pc, r, p):
    m, n = A.shape
    assert R.shape == (r, n) and len(pc) == r
    assert all(pc[i] < pc[i + 1] for i in range(r - 1))
    assert np.array_equal(R[:, pc], np.eye(r, dtype=np.int32))
    for t in range(r):
        nz = np.nonzero(R[t])[0]
        assert nz[0] == pc[t]
    assert np.array_equal(_mul(A[:, pc], R, p), A.astype(object) % p)


@pytest.mark.parametrize("p", PRIMES)
def test_rref_characterisation_random(orc, p):
    rng = np.random.default_rng(p)
    for t in range(12):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        r = int(rng.integers(0, min(m, n) + 1))
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        rk, R, pc = orc.rref(A, p)
        assert rk == r
        _rref_characterised(A, R, pc, rk, p)
        # the pivot columns are the column rank profile (leftmost independent columns)
        r2, _, cols = orc.pivots(A, p)
        assert np.array_equal(np.sort(cols), pc)


def _row_space(A, p):
    m, n = A.shape
    vecs = set()
    for coef in itertools.product(range(p), repeat=m):
        v = tuple((np.array(coef, np.int64).dot(A.astype(np.int64)) % p).tolist())
        vecs.add(v)
    return vecs


@pytest.mark.parametrize("p,m,n", [(2, 3, 3), (2, 2, 4), (3, 2, 3)])
def test_rref_exhaustive_row_space(orc, p, m, n):
    """Every matrix over a tiny field: the RREF rows span exactly the row
    space of A (brute force over all combinations), and the RREF is the
    reduced echelon matrix of that space."""
    for flat in itertools.product(range(p), repeat=m * n):
        A = np.array(flat, np.int32).reshape(m, n)
        r, R, pc = orc.rref(A, p)
        assert _row_space(A, p) == (_row_space(R, p) if r else {tuple([0] * n)})
        if r:
            _rref_characterised(A, R, pc, r, p)


@pytest.mark.parametrize("p", PRIMES)
def test_nullspace(orc, p):
    rng = np.random.default_rng(p + 1)
    for t in range(10):
        m, n = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        r = int(rng.integers(0, min(m, n) + 1))
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        N = orc.nullspace(A, p)
        assert N.shape == (n, n - r)
        assert not _mul(A, N, p).any()
        _, _, pc = orc.rref(A, p)
        free = [j for j in range(n) if j not in set(pc.tolist())]
        assert np.array_equal(N[free], np.eye(n - r, dtype=np.int32))


def test_nullspace_special_cases(orc):
    p = 65521
    assert orc.nullspace(np.eye(4, dtype=np.int32), p).shape == (4, 0)
    Z = np.zeros((3, 5), np.int32)
    assert np.array_equal(orc.nullspace(Z, p), np.eye(5, dtype=np.int32))


@pytest.mark.parametrize("p", PRIMES)
def test_solve(orc, p):
    rng = np.random.default_rng(p + 2)
    for t in range(10):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        r = int(rng.integers(0, min(m, n) + 1))
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        # consistent right-hand sides (A times something) and random ones
        Y = rng.integers(0, p, (n, 3)).astype(np.int32)
        B = np.concatenate([np.array(_mul(A, Y, p), np.int32), rng.integers(0, p, (m, 2)).astype(np.int32)], 1)
        X, ok, rk = orc.solve(A, B, p)
        assert rk == r
        _, _, pc = orc.rref(A, p)
        free = [j for j in range(n) if j not in set(pc.tolist())]
        for j in range(B.shape[1]):
            aug = np.concatenate([A, B[:, j:j + 1]], 1)
            r_aug = orc.pivots(aug, p)[0]
            assert ok[j] == (r_aug == r), (j, r_aug, r)
            if ok[j]:
                assert np.array_equal(_mul(A, X[:, j:j + 1], p).astype(np.int64), B[:, j:j + 1].astype(np.int64))
                assert not X[free, j].any()
            else:
                assert not X[:, j].any()
        assert ok[:3].all()
