"""Pins of the oracle's row-major-order PLUQ (the output of the slab
algorithms of Section 4.1): pivots equal the rank profile matrix by minor
enumeration (exhaustive over tiny fields), pivot rows ascend, A == PLUQ
exactly, triangular structure, and the pivot pairs agree as a set with the
four-quadrant PLUQ (computed through ORDER and pass 2, a different route).
"""
import numpy as np
import pytest

import checks
import workloads as wl
from test_oracle_pins import _all_matrices, _rank_profile_matrix


@pytest.mark.parametrize("p,m,n", [(2, 3, 3), (2, 3, 4), (2, 4, 3), (3, 3, 3)])
def test_rowmajor_exhaustive(orc, p, m, n):
    Ms = _all_matrices(p, m, n)
    R, rank = _rank_profile_matrix(Ms, p)
    for t in range(Ms.shape[0]):
        A = Ms[t].astype(np.int32)
        f = orc.pluq_rowmajor(A, p)
        assert f.rank == rank[t]
        got = np.zeros((m, n), np.int64)
        got[f.P[:f.rank], f.Q[:f.rank]] = 1
        assert np.array_equal(got, R[t])
        assert (np.diff(f.P[:f.rank]) > 0).all()
        assert checks.structure_ok(f.LU, f.rank, p) is None
        assert checks.reconstruct_ok(A, f.LU, f.P, f.Q, f.rank, p)


@pytest.mark.parametrize("p", [2, 3, 251, 65521, 131071, 8388593])
def test_rowmajor_random(orc, p):
    rng = np.random.default_rng(p + 11)
    for _ in range(8):
        m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        r = int(rng.integers(0, min(m, n) + 1))
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        f = orc.pluq_rowmajor(A, p)
        g = orc.pluq(A, p)
        assert f.rank == g.rank == r
        assert set(zip(f.P[:r].tolist(), f.Q[:r].tolist())) == set(zip(g.P[:r].tolist(), g.Q[:r].tolist()))
        assert np.array_equal(f.rrp, g.rrp) and np.array_equal(f.crp, g.crp)
        assert np.array_equal(f.P[:r], f.rrp)
        assert (np.diff(f.P[r:]) > 0).all() and (np.diff(f.Q[r:]) > 0).all()
        assert checks.structure_ok(f.LU, r, p) is None
        assert checks.reconstruct_ok(A, f.LU, f.P, f.Q, r, p)
        assert checks.reveals_rank_profile_matrix(f.LU, f.P, f.Q, r)
