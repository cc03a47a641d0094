"""Direct block implementation of the four-quadrant tile recursion, for tests.

A deliberately naive, pure NumPy (int64) rendering of the tiled recursive
PLUQ of Section 4.1 ("Tiled recursive elimination"): split rows and columns
in halves, factor the top-left tile, update the three other tiles, factor
the top-right and bottom-left remainders (independent of each other when the
top-left tile is rank deficient), update and factor the bottom-right
remainder, and restore the echelon layout with order-preserving rotations.
The block equations are derived from A = P L U Q (they are spelled out in
the project design notes); the base cases are a single row (first nonzero)
and a single column (first nonzero).

It is used only on small inputs, as an independent check of the oracle's
pivot order (pass 1 + ORDER + pass 2 computes the same result by a different
route) and, in the property checks, of large GPU outputs.
"""
from __future__ import annotations

import numpy as np


def _inv(a: int, p: int) -> int:
    return pow(int(a), p - 2, p)


def _lower_unit_solve(L: np.ndarray, B: np.ndarray, p: int) -> np.ndarray:
    """X with L X = B, L unit lower triangular (forward substitution)."""
    X = B.copy() % p
    for i in range(L.shape[0]):
        for t in range(i):
            X[i] = (X[i] - L[i, t] * X[t]) % p
    return X


def _upper_right_solve(B: np.ndarray, U: np.ndarray, p: int) -> np.ndarray:
    """X with X U = B, U upper triangular with nonzero diagonal."""
    X = B.copy() % p
    for j in range(U.shape[0]):
        for t in range(j):
            X[:, j] = (X[:, j] - X[:, t] * U[t, j]) % p
        X[:, j] = (X[:, j] * _inv(U[j, j], p)) % p
    return X


def _rec(W: np.ndarray, p: int):
    """Factor the view W in place; return (P, Q, r) local to W."""
    m, n = W.shape
    if m == 0 or n == 0:
        return np.arange(m), np.arange(n), 0
    if m == 1:
        nz = np.flatnonzero(W[0])
        if len(nz) == 0:
            return np.arange(1), np.arange(n), 0
        j = nz[0]
        Q = np.concatenate([[j], np.delete(np.arange(n), j)])
        W[0] = W[0, Q]
        return np.arange(1), Q, 1
    if n == 1:
        nz = np.flatnonzero(W[:, 0])
        if len(nz) == 0:
            return np.arange(m), np.arange(1), 0
        i = nz[0]
        P = np.concatenate([[i], np.delete(np.arange(m), i)])
        W[:, 0] = W[P, 0]
        W[1:, 0] = (W[1:, 0] * _inv(W[0, 0], p)) % p
        return P, np.arange(1), 1
    m1, n1 = m // 2, n // 2
    P1, Q1, r1 = _rec(W[:m1, :n1], p)
    W[:m1, n1:] = W[:m1, n1:][P1]
    W[m1:, :n1] = W[m1:, :n1][:, Q1]
    L1 = np.tril(W[:r1, :r1], -1) + np.eye(r1, dtype=np.int64)
    U1 = np.triu(W[:r1, :r1])
    W[:r1, n1:] = _lower_unit_solve(L1, W[:r1, n1:], p)               # D
    W[m1:, :r1] = _upper_right_solve(W[m1:, :r1], U1, p)              # E
    D, E = W[:r1, n1:], W[m1:, :r1]
    W[r1:m1, n1:] = (W[r1:m1, n1:] - W[r1:m1, :r1] @ D) % p           # F
    W[m1:, r1:n1] = (W[m1:, r1:n1] - E @ W[:r1, r1:n1]) % p           # G
    W[m1:, n1:] = (W[m1:, n1:] - E @ D) % p                           # H
    P2, Q2, r2 = _rec(W[r1:m1, n1:], p)
    P3, Q3, r3 = _rec(W[m1:, r1:n1], p)
    W[r1:m1, :r1] = W[r1:m1, :r1][P2]
    W[:r1, r1:n1] = W[:r1, r1:n1][:, Q3]
    W[m1:, :r1] = W[m1:, :r1][P3]
    W[m1:, n1:] = W[m1:, n1:][P3]
    W[:r1, n1:] = W[:r1, n1:][:, Q2]
    W[m1:, n1:] = W[m1:, n1:][:, Q2]
    U2 = np.triu(W[r1:r1 + r2, n1:n1 + r2])
    V2 = W[r1:r1 + r2, n1 + r2:]
    L3 = np.tril(W[m1:m1 + r3, r1:r1 + r3], -1) + np.eye(r3, dtype=np.int64)
    M3 = W[m1 + r3:, r1:r1 + r3]
    W[m1:, n1:n1 + r2] = _upper_right_solve(W[m1:, n1:n1 + r2], U2, p)     # [I; K]
    I_, K = W[m1:m1 + r3, n1:n1 + r2], W[m1 + r3:, n1:n1 + r2]
    W[m1:m1 + r3, n1 + r2:] = _lower_unit_solve(
        L3, (W[m1:m1 + r3, n1 + r2:] - I_ @ V2) % p, p)                   # O
    O = W[m1:m1 + r3, n1 + r2:]
    W[m1 + r3:, n1 + r2:] = (W[m1 + r3:, n1 + r2:] - K @ V2 - M3 @ O) % p  # R
    P4, Q4, r4 = _rec(W[m1 + r3:, n1 + r2:], p)
    W[m1 + r3:, :n1 + r2] = W[m1 + r3:, :n1 + r2][P4]
    W[:m1 + r3, n1 + r2:] = W[:m1 + r3, n1 + r2:][:, Q4]
    # index bookkeeping: position -> local original index
    P = np.arange(m)
    P[:m1] = P[:m1][P1]
    P[r1:m1] = P[r1:m1][P2]
    P[m1:] = P[m1:][P3]
    P[m1 + r3:] = P[m1 + r3:][P4]
    Q = np.arange(n)
    Q[:n1] = Q[:n1][Q1]
    Q[n1:] = Q[n1:][Q2]
    Q[r1:n1] = Q[r1:n1][Q3]
    Q[n1 + r2:] = Q[n1 + r2:][Q4]
    # final rotations: rows [a f f' g R r'] -> [a f g R f' r'],
    # columns [a g g' f R c'] -> [a f g R g' c']
    a, f, fp = np.arange(0, r1), np.arange(r1, r1 + r2), np.arange(r1 + r2, m1)
    g, R, rest = np.arange(m1, m1 + r3), np.arange(m1 + r3, m1 + r3 + r4), np.arange(m1 + r3 + r4, m)
    rsel = np.concatenate([a, f, g, R, fp, rest]).astype(np.int64)
    ca, cg, cgp = np.arange(0, r1), np.arange(r1, r1 + r3), np.arange(r1 + r3, n1)
    cf, cR, crest = np.arange(n1, n1 + r2), np.arange(n1 + r2, n1 + r2 + r4), np.arange(n1 + r2 + r4, n)
    csel = np.concatenate([ca, cf, cg, cR, cgp, crest]).astype(np.int64)
    W[:, :] = W[rsel][:, csel]
    return P[rsel], Q[csel], r1 + r2 + r3 + r4


def pluq(A: np.ndarray, p: int):
    """Returns (LU, P, Q, r) in the same layout as the oracle."""
    W = np.array(A, dtype=np.int64) % p
    P, Q, r = _rec(W, p)
    return W, np.asarray(P, np.int64), np.asarray(Q, np.int64), int(r)
