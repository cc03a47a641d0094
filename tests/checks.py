"""Host-side checks of a PLUQ result that hold at any size.

Used on GPU outputs too large for the oracle to recompute, and pinned on small
inputs against the oracle and brute force.  Together they determine the
canonical factorisation uniquely:

  * structure: P, Q permutations; L unit lower trapezoidal (implicit unit
    diagonal), U upper trapezoidal with nonzero diagonal; zero block [r:, r:];
  * A == P L U Q (mod p): exactly for small sizes, otherwise by Freivalds'
    test with several random vectors (false-accept probability <= p^-k);
  * the pivot set is the rank profile matrix R_A: a PLUQ decomposition reveals
    R_A exactly when P [L 0] P^T is lower triangular and Q^T [U; 0] Q is upper
    triangular (each nonzero L[i, t] sits in an original row after the pivot
    row of column t; each nonzero U[t, j] in an original column after the
    pivot column of row t);
  * the pivot order and the order of the non-pivots follow the four-quadrant
    recursion (the index-only ORDER of the oracle), non-pivots ascending.
Given P and Q, the L and U factors are unique, so these checks pin every
output bit.
"""
from __future__ import annotations

import numpy as np


def is_perm(v: np.ndarray, n: int) -> bool:
    v = np.asarray(v)
    return v.shape == (n,) and np.array_equal(np.sort(v), np.arange(n))


def structure_ok(LU: np.ndarray, r: int, p: int) -> str | None:
    m, n = LU.shape
    if not (0 <= r <= min(m, n)):
        return "rank out of range"
    if (LU < 0).any() or (LU >= p).any():
        return "entry outside [0, p)"
    if r and (np.diagonal(LU)[:r] == 0).any():
        return "zero on the diagonal of U"
    if (LU[r:, r:] != 0).any():
        return "nonzero Schur block"
    return None


def _matvec_mod(A: np.ndarray, x: np.ndarray, p: int, rows_per_chunk: int = 2048) -> np.ndarray:
    """A @ x mod p without int64 overflow (A, x residues < 2^31)."""
    out = np.empty(A.shape[0], np.int64)
    # split x into 16-bit halves so that each partial dot product fits in int64
    # for up to 2^15 columns: 2^31 * 2^16 * 2^15 = 2^62
    xl = (x & 0xFFFF).astype(np.int64)
    xh = (x >> 16).astype(np.int64)
    for s in range(0, A.shape[0], rows_per_chunk):
        blk = A[s:s + rows_per_chunk].astype(np.int64)
        lo = (blk @ xl) % p
        hi = (blk @ xh) % p
        out[s:s + rows_per_chunk] = (lo + hi * (65536 % p)) % p
    return out


def reconstruct_ok(A: np.ndarray, LU: np.ndarray, P, Q, r: int, p: int,
                   exact_limit: int = 600, vectors: int = 4, seed: int = 12345) -> bool:
    """A[P[i], Q[j]] == sum_t L[i, t] U[t, j] (mod p)."""
    m, n = A.shape
    P = np.asarray(P, np.int64)
    Q = np.asarray(Q, np.int64)
    if max(m, n) <= exact_limit:
        L = np.tril(LU[:, :r].astype(object), -1)
        for t in range(r):
            L[t, t] = 1
        U = np.triu(LU[:r, :].astype(object))
        prod = (L.dot(U) % p) if r else np.zeros((m, n), dtype=object)
        return bool(np.array_equal(prod.astype(np.int64), A[P][:, Q].astype(np.int64)))
    rng = np.random.default_rng(seed)
    for _ in range(vectors):
        w = rng.integers(0, p, n, dtype=np.int64)
        # lhs = (P^T A Q^T) w  ==  (A wq)[P] with wq[Q[j]] = w[j]
        wq = np.empty(n, np.int64)
        wq[Q] = w
        lhs = _matvec_mod(A, wq, p)[P]
        # rhs = L (U w)
        Uw = np.zeros(r, np.int64)
        if r:
            Ut = np.triu(LU[:r, :])
            Uw = _matvec_mod(Ut, w, p)
            Lr = np.tril(LU[:, :r], -1)
            rhs = _matvec_mod(Lr, Uw, p)
            rhs[:r] = (rhs[:r] + Uw) % p
        else:
            rhs = np.zeros(m, np.int64)
        if not np.array_equal(lhs, rhs):
            return False
    return True


def reveals_rank_profile_matrix(LU: np.ndarray, P, Q, r: int) -> bool:
    """P [L 0] P^T lower triangular and Q^T [U; 0] Q upper triangular."""
    P = np.asarray(P, np.int64)
    Q = np.asarray(Q, np.int64)
    m, n = LU.shape
    if r == 0:
        return True
    Lp = np.tril(LU[:, :r], -1)          # i > t
    ii, tt = np.nonzero(Lp)
    if (P[ii] <= P[tt]).any():
        return False
    Up = np.triu(LU[:r, :], 1)           # j > t
    tt, jj = np.nonzero(Up)
    if (Q[jj] <= Q[tt]).any():
        return False
    return True


def canonical_order_ok(P, Q, r: int, order_fn) -> bool:
    """Pivots in ORDER, non-pivot rows / columns ascending.

    ``order_fn(m, n, rows, cols)`` returns the ordered pivot pairs."""
    P = np.asarray(P, np.int64)
    Q = np.asarray(Q, np.int64)
    m, n = len(P), len(Q)
    orow, ocol = order_fn(m, n, P[:r].astype(np.int32), Q[:r].astype(np.int32))
    if len(orow) != r or not np.array_equal(orow, P[:r]) or not np.array_equal(ocol, Q[:r]):
        return False
    return bool((np.diff(P[r:]) > 0).all() and (np.diff(Q[r:]) > 0).all())


def full_check(A, LU, P, Q, r, p, order_fn, **kw) -> str | None:
    """None when every property holds, else the name of the first failure."""
    m, n = A.shape
    if not is_perm(P, m) or not is_perm(Q, n):
        return "P or Q not a permutation"
    s = structure_ok(LU, r, p)
    if s:
        return s
    if not reconstruct_ok(A, LU, P, Q, r, p, **kw):
        return "A != PLUQ"
    if not reveals_rank_profile_matrix(LU, P, Q, r):
        return "pivots are not the rank profile matrix"
    if not canonical_order_ok(P, Q, r, order_fn):
        return "pivot order not canonical"
    return None
