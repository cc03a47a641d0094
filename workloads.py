"""Seeded synthetic inputs for the tests and the benchmark.

This module holds only input synthesis: a counter-based generator
(splitmix64), uniform residues by rejection sampling, random permutations by
Fisher-Yates, and matrices of prescribed rank built as products of random
triangular factors.  Neither the GPU library nor the CPU oracle imports it;
the tests and the benchmark call it and hand the same arrays to both.

Workloads (shapes and structure follow the paper's experiments: dense uniform
matrices modulo a prime of about 17-23 bits, Section 3 and Table 3, and a
rank-deficient matrix whose independent rows and columns are spread uniformly
over the dimension, the S16K input of Section 4.1):

  * ``uniform(m, n, p, seed)``    entries uniform in [0, p-1];
  * ``lowrank(m, n, r, p, seed)`` A = Pr * L * U * Qr with L (m x r) unit lower
    trapezoidal, U (r x n) upper trapezoidal with nonzero diagonal, Pr, Qr
    random permutations: rank exactly r, pivots scattered;
  * ``batch(count, lo, hi, p, seed)`` many small matrices of uneven shapes and
    ranks, packed row-major one after the other.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of splitmix64 seeded with ``seed``.

    Output i is mix(seed + (i + 1) * gamma) with the published splitmix64
    finaliser, so any slice of the stream can be produced independently."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class Stream:
    """Sequential reader over one splitmix64 stream."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def raw(self, count: int) -> np.ndarray:
        out = splitmix64(self.seed, self.pos, count)
        self.pos += count
        return out

    def below(self, bound: int, count: int) -> np.ndarray:
        """``count`` integers uniform in [0, bound) by masked rejection."""
        bound = int(bound)
        if bound <= 0:
            raise ValueError("bound must be positive")
        if bound == 1:
            return np.zeros(count, np.int64)
        mask = np.uint64((1 << int(bound - 1).bit_length()) - 1)
        out = np.empty(count, np.int64)
        got = 0
        while got < count:
            need = count - got
            z = self.raw(need + need // 2 + 16) & mask
            z = z[z < np.uint64(bound)][:need]
            out[got:got + len(z)] = z.astype(np.int64)
            got += len(z)
        return out

    def range(self, lo: int, hi: int, count: int) -> np.ndarray:
        """``count`` integers uniform in [lo, hi] (inclusive)."""
        return lo + self.below(hi - lo + 1, count)

    def permutation(self, n: int) -> np.ndarray:
        """Fisher-Yates shuffle of 0..n-1: for i = n-1 down to 1 swap i with
        j_i = floor(u_i * (i + 1)), u_i the top 53 bits of one draw."""
        perm = np.arange(n, dtype=np.int64)
        if n < 2:
            return perm
        u = (self.raw(n - 1) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
        i = np.arange(n - 1, 0, -1, dtype=np.int64)
        js = np.minimum((u * (i + 1)).astype(np.int64), i).tolist()
        pl = perm.tolist()
        for k, ii in enumerate(range(n - 1, 0, -1)):
            j = js[k]
            pl[ii], pl[j] = pl[j], pl[ii]
        return np.array(pl, dtype=np.int64)


def uniform(m: int, n: int, p: int, seed: int) -> np.ndarray:
    """m x n int32 matrix, entries uniform in [0, p-1]."""
    s = Stream(seed)
    return s.below(p, m * n).astype(np.int32).reshape(m, n)


def _mod_product(X: np.ndarray, Y: np.ndarray, p: int) -> np.ndarray:
    """Exact X @ Y mod p for int64 residue matrices, through float64 products
    of operand slices small enough that every partial sum stays below 2^53."""
    k = X.shape[1]
    if k == 0:
        return np.zeros((X.shape[0], Y.shape[1]), np.int64)
    bits = int(p - 1).bit_length()
    # split Y into base-2^s digits so that k * (p-1) * (2^s - 1) < 2^53
    s = bits
    while s > 1 and k * (p - 1) * ((1 << s) - 1) >= (1 << 53):
        s -= 1
    Xf = X.astype(np.float64)
    out = np.zeros((X.shape[0], Y.shape[1]), np.int64)
    shift = 0
    rest = Y.astype(np.int64)
    while True:
        digit = rest & ((1 << s) - 1)
        part = np.rint(Xf @ digit.astype(np.float64)).astype(np.int64) % p
        out = (out + part * (pow(2, shift, p))) % p
        rest = rest >> s
        shift += s
        if not rest.any():
            break
    return out


def lowrank(m: int, n: int, r: int, p: int, seed: int) -> np.ndarray:
    """A = Pr * L * U * Qr mod p with rank exactly r (requires r <= min(m, n)).

    L is m x r unit lower trapezoidal with entries below the diagonal uniform
    in [0, p-1]; U is r x n upper trapezoidal with diagonal uniform in
    [1, p-1] and entries above it uniform in [0, p-1]; Pr and Qr are uniform
    random permutations (Fisher-Yates)."""
    if not 0 <= r <= min(m, n):
        raise ValueError("rank out of range")
    s = Stream(seed)
    L = np.zeros((m, r), np.int64)
    if r:
        low = np.tril_indices(m, -1, r)
        L[low] = s.below(p, len(low[0]))
        L[np.arange(r), np.arange(r)] = 1
    U = np.zeros((r, n), np.int64)
    if r:
        up = np.triu_indices(r, 1, n)
        U[up] = s.below(p, len(up[0]))
        U[np.arange(r), np.arange(r)] = s.range(1, p - 1, r)
    pr = s.permutation(m)
    qr = s.permutation(n)
    LU = _mod_product(L, U, p)
    A = np.empty((m, n), np.int64)
    # (Pr * M)[i, :] = M[pr^-1 ...]: row i of M goes to position pr[i]
    A[pr, :] = LU
    B = np.empty_like(A)
    B[:, qr] = A
    return B.astype(np.int32)


def batch(count: int, lo: int, hi: int, p: int, seed: int):
    """``count`` matrices with m_i, n_i uniform in [lo, hi] and rank r_i
    uniform in [1, min(m_i, n_i)], each A_i = lowrank(m_i, n_i, r_i).

    Returns (ms, ns, ranks, A_packed, A_off) where A_packed holds the
    matrices row-major (leading dimension n_i) at offsets A_off."""
    s = Stream(seed)
    ms = s.range(lo, hi, count)
    ns = s.range(lo, hi, count)
    rs = np.array([s.range(1, min(a, b), 1)[0] for a, b in zip(ms, ns)], np.int64)
    sizes = ms * ns
    off = np.zeros(count + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    A = np.empty(int(off[-1]), np.int32)
    sub = s.raw(count)
    for i in range(count):
        A[off[i]:off[i + 1]] = lowrank(int(ms[i]), int(ns[i]), int(rs[i]), p,
                                       int(sub[i] & np.uint64(0x7FFFFFFFFFFFFFFF))).ravel()
    return ms.astype(np.int32), ns.astype(np.int32), rs.astype(np.int32), A, off[:-1].copy()


# The five benchmark workloads (seed = workload number).
WORKLOADS = {
    "pluq512_p65521": dict(kind="uniform", m=512, n=512, p=65521, seed=1),
    "pluq8192_p131071": dict(kind="uniform", m=8192, n=8192, p=131071, seed=2),
    "pluq8192_r4096_p131071": dict(kind="lowrank", m=8192, n=8192, r=4096, p=131071, seed=3),
    "n16384_p251": dict(kind="uniform", m=16384, n=16384, p=251, seed=4),
    "n16384_p8388593": dict(kind="uniform", m=16384, n=16384, p=8388593, seed=4),
    "batch4096_p65521": dict(kind="batch", count=4096, lo=16, hi=512, p=65521, seed=5),
}


def make(name: str):
    w = WORKLOADS[name]
    if w["kind"] == "uniform":
        return uniform(w["m"], w["n"], w["p"], w["seed"])
    if w["kind"] == "lowrank":
        return lowrank(w["m"], w["n"], w["r"], w["p"], w["seed"])
    return batch(w["count"], w["lo"], w["hi"], w["p"], w["seed"])
