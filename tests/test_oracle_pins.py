"""Pins of the CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself:
trial division, Python big integers, residuals, ranks of leading blocks by
minor enumeration (no elimination), textbook special cases, a direct block
implementation of the tile recursion, and the exactness bound of Section 3.1.
"""
import itertools

import numpy as np
import pytest

import blockref
import checks
import workloads as wl

PRIMES = [2, 3, 5, 7, 251, 65521, 131071, 8388593]


# ---------------------------------------------------------------- scalars
def test_is_prime_matches_trial_division(orc):
    def trial(n):
        if n < 2:
            return False
        d = 2
        while d * d <= n:
            if n % d == 0:
                return False
            d += 1
        return True
    for n in range(0, 5000):
        assert orc.is_prime(n) == trial(n), n
    for n in [65521, 131071, 8388593, 2147483647, 94906249]:
        assert orc.is_prime(n) == trial(n), n
    for n in [65535, 131073, 8388595, 4294967291 // 3, 25326001, 3215031751 % (1 << 31)]:
        assert orc.is_prime(n) == trial(n), n


def test_inverse(orc):
    rng = np.random.default_rng(1)
    for p in PRIMES:
        for a in rng.integers(1, p, 200):
            assert (int(a) * orc.inv(int(a), p)) % p == 1


# ---------------------------------------------------------------- gemm
@pytest.mark.parametrize("p", [2, 251, 131071, 8388593])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_fgemm_bigint(orc, p, ta, tb):
    rng = np.random.default_rng(p + 2 * ta + tb)
    m, n, k = 7, 5, 9
    A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
    B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
    C = rng.integers(0, p, (m, n)).astype(np.int32)
    alpha, beta = int(rng.integers(0, p)), int(rng.integers(0, p))
    got = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
    Ao = (A.T if ta else A).astype(object)
    Bo = (B.T if tb else B).astype(object)
    want = (alpha * Ao.dot(Bo) + beta * C.astype(object)) % p
    assert np.array_equal(got.astype(object), want)


def test_fgemm_k_zero_and_empty(orc):
    p = 131071
    C = np.full((3, 4), 5, np.int32)
    got = orc.fgemm(np.zeros((3, 0), np.int32), np.zeros((0, 4), np.int32), C, p, 1, 2)
    assert (got == 10).all()


# ---------------------------------------------------------------- trsm
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_ftrsm_residual(orc, side, uplo, trans, diag):
    p = 131071
    rng = np.random.default_rng(side * 8 + uplo * 4 + trans * 2 + diag)
    m, n = 6, 5
    d = m if side == 0 else n
    T = rng.integers(0, p, (d, d)).astype(np.int32)
    T[np.arange(d), np.arange(d)] = rng.integers(1, p, d)
    B = rng.integers(0, p, (m, n)).astype(np.int32)
    alpha = 7
    X = orc.ftrsm(side, uplo, trans, diag, T, B, p, alpha)
    To = T.astype(object)
    To = np.tril(To) if uplo == 0 else np.triu(To)
    if diag:
        for i in range(d):
            To[i, i] = 1
    if trans:
        To = To.T
    Xo = X.astype(object)
    lhs = To.dot(Xo) if side == 0 else Xo.dot(To)
    assert np.array_equal(lhs % p, (alpha * B.astype(object)) % p)
    # entries of the strictly opposite triangle must not be read
    T2 = T.copy()
    if uplo == 0:
        T2[np.triu_indices(d, 1)] = 0
    else:
        T2[np.tril_indices(d, -1)] = 0
    if diag:
        T2[np.arange(d), np.arange(d)] = 0
    assert np.array_equal(orc.ftrsm(side, uplo, trans, diag, T2, B, p, alpha), X)


def test_ftrsm_singular(orc):
    T = np.eye(3, dtype=np.int32)
    T[1, 1] = 0
    with pytest.raises(orc.OracleError):
        orc.ftrsm(0, 0, 0, 0, T, np.ones((3, 2), np.int32), 7)


# ------------------------------------------- rank profile matrix by minors
def _det_stack(M, p):
    s = M.shape[1]
    tot = np.zeros(M.shape[0], np.int64)
    for perm in itertools.permutations(range(s)):
        inv = sum(1 for a in range(s) for b in range(a + 1, s) if perm[a] > perm[b])
        prod = np.ones(M.shape[0], np.int64)
        for i in range(s):
            prod = (prod * M[:, i, perm[i]]) % p
        tot = (tot + (-prod if inv % 2 else prod)) % p
    return tot


def _rank_by_minors(M, p):
    """Rank of each matrix of the stack: the largest order of a nonzero minor."""
    N, a, b = M.shape
    rank = np.zeros(N, np.int64)
    for s in range(1, min(a, b) + 1):
        found = np.zeros(N, bool)
        for rows in itertools.combinations(range(a), s):
            sub = M[:, list(rows), :]
            for cols in itertools.combinations(range(b), s):
                found |= _det_stack(sub[:, :, list(cols)], p) != 0
        if not found.any():
            break
        rank = np.where(found, s, rank)
    return rank


def _rank_profile_matrix(M, p):
    """R_A[i, j] = rho(i+1, j+1) - rho(i, j+1) - rho(i+1, j) + rho(i, j), with
    rho(i, j) the rank of the leading i x j block."""
    N, m, n = M.shape
    rho = np.zeros((N, m + 1, n + 1), np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            rho[:, i, j] = _rank_by_minors(M[:, :i, :j], p)
    return rho[:, 1:, 1:] - rho[:, :-1, 1:] - rho[:, 1:, :-1] + rho[:, :-1, :-1], rho[:, m, n]


def _all_matrices(p, m, n):
    idx = np.arange(p ** (m * n), dtype=np.int64)
    digits = np.stack([(idx // p ** k) % p for k in range(m * n)], axis=1)
    return digits.reshape(-1, m, n)


EXHAUSTIVE = [(2, 3, 3), (2, 2, 4), (2, 4, 2), (2, 3, 4), (2, 4, 3), (2, 4, 4), (3, 3, 3), (3, 2, 2), (2, 1, 4)]


@pytest.mark.parametrize("p,m,n", EXHAUSTIVE)
def test_pivots_equal_rank_profile_matrix_exhaustive(orc, p, m, n):
    Ms = _all_matrices(p, m, n)
    R, rank = _rank_profile_matrix(Ms, p)
    for t in range(Ms.shape[0]):
        A = Ms[t].astype(np.int32)
        r, pr, pc = orc.pivots(A, p)
        assert r == rank[t]
        got = np.zeros((m, n), np.int64)
        got[pr, pc] = 1
        assert np.array_equal(got, R[t]), (A, got, R[t])
        f = orc.pluq(A, p)
        assert f.rank == r
        assert np.array_equal(np.sort(f.P[:r]), f.rrp)
        # pluq pivots are the same pairs, possibly in another order
        pairs = set(zip(f.P[:r].tolist(), f.Q[:r].tolist()))
        assert pairs == set(zip(pr.tolist(), pc.tolist()))
        assert np.array_equal(f.rrp, np.sort(pr)) and np.array_equal(f.crp, np.sort(pc))


def test_pivots_rank_profile_random_5x5(orc):
    rng = np.random.default_rng(7)
    for p in (2, 3, 5, 251):
        Ms = np.stack([wl.lowrank(5, 5, int(rng.integers(0, 6)), p, int(rng.integers(1 << 40)))
                       for _ in range(60)]).astype(np.int64)
        R, rank = _rank_profile_matrix(Ms, p)
        for t in range(Ms.shape[0]):
            r, pr, pc = orc.pivots(Ms[t].astype(np.int32), p)
            got = np.zeros((5, 5), np.int64)
            got[pr, pc] = 1
            assert r == rank[t] and np.array_equal(got, R[t])


# ---------------------------------------------------------------- special cases
def test_identity(orc):
    p = 65521
    A = np.eye(6, 6, dtype=np.int32)
    f = orc.pluq(A, p)
    assert f.rank == 6
    assert np.array_equal(f.P, np.arange(6)) and np.array_equal(f.Q, np.arange(6))
    assert np.array_equal(f.LU, np.eye(6, dtype=np.int32))


def test_permutation_matrix(orc):
    p = 131071
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(1, 12))
        pi = rng.permutation(n)
        A = np.zeros((n, n), np.int32)
        A[np.arange(n), pi] = 1
        f = orc.pluq(A, p)
        assert f.rank == n
        # R_A = the permutation itself, L = U = I
        assert np.array_equal(pi[f.P], f.Q)
        assert np.array_equal(f.LU, np.eye(n, dtype=np.int32))


def test_zero_and_empty(orc):
    for m, n in [(0, 0), (0, 5), (4, 0), (3, 7), (1, 1)]:
        A = np.zeros((m, n), np.int32)
        f = orc.pluq(A, 7)
        assert f.rank == 0
        assert np.array_equal(f.P, np.arange(m)) and np.array_equal(f.Q, np.arange(n))
        assert (f.LU == 0).all()


def test_rank_one(orc):
    p = 251
    rng = np.random.default_rng(5)
    for _ in range(40):
        m, n = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        u = rng.integers(0, p, m) * (rng.random(m) < 0.6)
        v = rng.integers(0, p, n) * (rng.random(n) < 0.6)
        if not u.any():
            u[int(rng.integers(m))] = 1
        if not v.any():
            v[int(rng.integers(n))] = 3
        A = (np.outer(u, v) % p).astype(np.int32)
        f = orc.pluq(A, p)
        assert f.rank == 1
        assert f.P[0] == np.flatnonzero(u)[0] and f.Q[0] == np.flatnonzero(v)[0]


def test_generic_rank_profile_is_doolittle(orc):
    """All leading principal minors nonzero -> P = Q = I and L U = A."""
    p = 131071
    rng = np.random.default_rng(11)
    for n in (1, 2, 5, 17, 40):
        A = rng.integers(0, p, (n, n)).astype(np.int32)
        Ms = A[None].astype(np.int64)
        if n <= 5:
            for k in range(1, n + 1):
                assert _det_stack(Ms[:, :k, :k], p)[0] != 0
        f = orc.pluq(A, p)
        if f.rank == n and np.array_equal(f.P, np.arange(n)):
            assert np.array_equal(f.Q, np.arange(n))
            L = f.L().astype(object)
            U = f.U().astype(object)
            assert np.array_equal(L.dot(U) % p, A.astype(object))


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("p", [2, 3, 251, 65521, 131071, 8388593])
def test_reconstruction_and_structure(orc, p):
    rng = np.random.default_rng(p)
    for _ in range(25):
        m, n = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        r = int(rng.integers(0, min(m, n) + 1))
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        f = orc.pluq(A, p)
        assert f.rank == r
        assert checks.full_check(A, f.LU, f.P, f.Q, f.rank, p, orc.order) is None


# ------------------------------------- direct block recursion (tile recursive)
@pytest.mark.parametrize("p,m,n", [(2, 3, 3), (2, 3, 4), (2, 4, 3), (2, 4, 4), (3, 2, 3), (3, 3, 3)])
def test_block_recursion_exhaustive(orc, p, m, n):
    Ms = _all_matrices(p, m, n)
    for t in range(Ms.shape[0]):
        A = Ms[t].astype(np.int32)
        f = orc.pluq(A, p)
        LU, P, Q, r = blockref.pluq(A, p)
        assert r == f.rank and np.array_equal(P, f.P) and np.array_equal(Q, f.Q)
        assert np.array_equal(LU, f.LU)


def test_block_recursion_random(orc):
    rng = np.random.default_rng(2024)
    for p in (2, 3, 5, 251, 65521):
        for trial in range(60):
            m, n = int(rng.integers(1, 24)), int(rng.integers(1, 24))
            r = int(rng.integers(0, min(m, n) + 1))
            if trial % 3 == 0:
                A = rng.integers(0, p, (m, n)).astype(np.int32)
            else:
                A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
            f = orc.pluq(A, p)
            LU, P, Q, rr = blockref.pluq(A, p)
            assert rr == f.rank and np.array_equal(P, f.P) and np.array_equal(Q, f.Q)
            assert np.array_equal(LU, f.LU)


# ------------------------------------------------- the property checks themselves
def _other_pluq(A, p, rng):
    """A valid PLUQ with arbitrary (random) pivot choices, for negative tests."""
    W = A.astype(np.int64).copy()
    m, n = W.shape
    rows, cols = list(range(m)), list(range(n))
    k = 0
    while True:
        nz = [(i, j) for i in range(k, m) for j in range(k, n) if W[i, j] % p]
        if not nz:
            break
        i, j = nz[int(rng.integers(len(nz)))]
        W[[k, i]] = W[[i, k]]
        rows[k], rows[i] = rows[i], rows[k]
        W[:, [k, j]] = W[:, [j, k]]
        cols[k], cols[j] = cols[j], cols[k]
        inv = pow(int(W[k, k]), p - 2, p)
        for ii in range(k + 1, m):
            l = (W[ii, k] * inv) % p
            W[ii, k] = l
            W[ii, k + 1:] = (W[ii, k + 1:] - l * W[k, k + 1:]) % p
        k += 1
    return W, np.array(rows), np.array(cols), k


def test_property_checks_reject_wrong_pivots(orc):
    rng = np.random.default_rng(99)
    p = 5
    rejected = 0
    for _ in range(300):
        m, n = int(rng.integers(2, 7)), int(rng.integers(2, 7))
        A = wl.lowrank(m, n, int(rng.integers(1, min(m, n) + 1)), p, int(rng.integers(1 << 40)))
        W, P, Q, r = _other_pluq(A, p, rng)
        assert checks.reconstruct_ok(A, W, P, Q, r, p)
        _, pr, pc = orc.pivots(A, p)
        same = set(zip(P[:r].tolist(), Q[:r].tolist())) == set(zip(pr.tolist(), pc.tolist()))
        # the Bruhat-type criterion accepts no pivot set other than R_A
        ok = checks.reveals_rank_profile_matrix(W, P, Q, r)
        if ok:
            assert same
        rejected += not ok
    assert rejected > 50


def test_property_checks_reject_corruption(orc):
    p = 131071
    A = wl.lowrank(30, 25, 12, p, 77)
    f = orc.pluq(A, p)
    assert checks.full_check(A, f.LU, f.P, f.Q, f.rank, p, orc.order) is None
    bad = f.LU.copy()
    bad[20, 3] = (bad[20, 3] + 1) % p
    assert checks.full_check(A, bad, f.P, f.Q, f.rank, p, orc.order) is not None
    # Freivalds path
    assert not checks.reconstruct_ok(A, bad, f.P, f.Q, f.rank, p, exact_limit=0)
    assert checks.reconstruct_ok(A, f.LU, f.P, f.Q, f.rank, p, exact_limit=0)
    # swapping two non-pivot rows keeps A = PLUQ but breaks the order convention
    P2 = f.P.copy()
    P2[-1], P2[-2] = P2[-2], P2[-1]
    LU2 = f.LU.copy()
    LU2[[-1, -2]] = LU2[[-2, -1]]
    assert checks.reconstruct_ok(A, LU2, P2, f.Q, f.rank, p)
    assert checks.full_check(A, LU2, P2, f.Q, f.rank, p, orc.order) is not None


# ---------------------------------------------------------------- exactness bound
def test_delayed_reduction_bound():
    """Section 3.1: sums of k products of residues in [0, p-1] are exact in a
    53-bit mantissa while k (p-1)^2 < 2^53."""
    def kmax(p):
        return ((1 << 53) - 1) // ((p - 1) ** 2)
    assert kmax(65521) == 2098176
    assert kmax(131071) == 524304
    assert kmax(8388593) == 128
    for p in (65521, 131071, 8388593):
        k = kmax(p)
        assert k * (p - 1) ** 2 < 2 ** 53 <= (k + 1) * (p - 1) ** 2
        # the largest such sum is an integer below 2^53, so float64 holds it exactly
        s = float(k * (p - 1) ** 2)
        assert int(s) == k * (p - 1) ** 2
