"""GPU parity: every output of the HIP library equals the CPU oracle's, bit for bit.

Sizes span several kernel tiles with ragged tails; primes cover both paths'
limits and the delayed-reduction regimes (no reduction in the K loop, a
reduction every few hundred products, one every four).
"""
import sys

import numpy as np
import pytest

import checks
import workloads as wl

pytestmark = pytest.mark.gpu

PRIMES = [2, 3, 251, 65521, 131071, 8388593, 94906249]


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


def paths_for(p):
    from paper_1402_3501_amd import PATH_FP64, PATH_INT8, int8_limbs
    out = []
    if p <= 94906249:
        out.append(PATH_FP64)
    if int8_limbs(p) > 0:
        out.append(PATH_INT8)
    return out


# ---------------------------------------------------------------- fgemm
FGEMM_SHAPES = [(1, 1, 1), (7, 5, 3), (64, 64, 16), (130, 70, 33), (257, 300, 129), (200, 513, 700)]


@pytest.mark.parametrize("p", PRIMES)
def test_fgemm_parity(lib, orc, p):
    rng = np.random.default_rng(p)
    for path in paths_for(p):
        for (m, n, k) in FGEMM_SHAPES:
            for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
                if (m, n, k) == (200, 513, 700) and (ta, tb) != (0, 0):
                    continue
                A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
                B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
                C = rng.integers(0, p, (m, n)).astype(np.int32)
                for alpha, beta in [(1, 0), (p - 1, 1), (int(rng.integers(0, p)), int(rng.integers(0, p)))]:
                    note("fgemm", p, path, m, n, k, ta, tb, alpha, beta)
                    want = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
                    Cd = dev(C)
                    lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=path)
                    got = host(Cd)
                    assert np.array_equal(got, want), (p, path, m, n, k, ta, tb, alpha, beta)


@pytest.mark.parametrize("p", [251, 65521, 131071, 8388593])
def test_fgemm_int8_split_k(lib, orc, p):
    """INT8 products with few output blocks and a long K run as several K
    parts per block plus a combining pass: 4 equal parts, 4 uneven parts
    (18 K tiles as 5 + 5 + 5 + 3) and 2 parts, with alpha, beta and
    transposed operands."""
    from paper_1402_3501_amd import PATH_INT8
    rng = np.random.default_rng(p + 3)
    for (m, n, k) in [(150, 260, 2000), (33, 17, 1100), (129, 128, 600)]:
        for ta, tb in [(0, 0), (1, 1)]:
            A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
            B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
            C = rng.integers(0, p, (m, n)).astype(np.int32)
            for alpha, beta in [(1, 0), (int(rng.integers(0, p)), int(rng.integers(0, p)))]:
                note("fgemm split-k", p, m, n, k, ta, tb, alpha, beta)
                want = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
                Cd = dev(C)
                lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=PATH_INT8)
                assert np.array_equal(host(Cd), want), (p, m, n, k, ta, tb, alpha, beta)


def test_fgemm_long_k_reductions(lib, orc):
    """k far beyond the exactness bound: p = 8388593 needs a reduction every
    ~512 products, p = 94906249 one every 4."""
    from paper_1402_3501_amd import PATH_FP64
    rng = np.random.default_rng(5)
    for p, k in [(8388593, 2100), (94906249, 300)]:
        m, n = 70, 90
        A = rng.integers(0, p, (m, k)).astype(np.int32)
        B = rng.integers(0, p, (k, n)).astype(np.int32)
        C = np.zeros((m, n), np.int32)
        A[:, : k // 2] = p - 1   # worst-case magnitudes
        B[: k // 2, :] = p - 1
        note("fgemm long k", p, k)
        want = orc.fgemm(A, B, C, p, 1, 0)
        Cd = dev(C)
        lib.fgemm(dev(A), dev(B), Cd, p, 1, 0, path=PATH_FP64)
        assert np.array_equal(host(Cd), want)


@pytest.mark.parametrize("p", [251, 65521, 8388593])
def test_fgemm_int8_k_chunks(lib, orc, p):
    """INT8 products whose k exceeds one chunk of the INT8 path (the int32
    shift-class accumulators are reduced mod p after every chunk: 131072
    products with one limb, 65536 with two, 32768 with three), so a later
    chunk adds onto the reduced result of the earlier ones with its operands
    read at the chunk's offset; alpha, beta and transposed operands."""
    from paper_1402_3501_amd import PATH_INT8, int8_limbs
    L = int8_limbs(p)
    chunk = {1: 131072, 2: 65536, 3: 32768}[L]
    rng = np.random.default_rng(p + 11)
    m, n, k = 64, 48, chunk + 232
    for ta, tb in [(0, 0), (1, 1)]:
        A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
        B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
        C = rng.integers(0, p, (m, n)).astype(np.int32)
        alpha, beta = int(rng.integers(1, p)), int(rng.integers(1, p))
        note("fgemm int8 k chunks", p, L, m, n, k, ta, tb, alpha, beta)
        want = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
        Cd = dev(C)
        lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=PATH_INT8)
        assert np.array_equal(host(Cd), want), (p, ta, tb)


@pytest.mark.parametrize("p", [131071, 94906249])
def test_fgemm_f64_large_tiles_transposed(lib, orc, p):
    """FP64 products large enough for the 128 x 128 tile kernel (at least 192
    output tiles of 128), with every transpose combination, ragged edges on
    all three dimensions and, for p = 94906249, reductions inside the K loop;
    40 sampled rows (plus the first and last) checked against the oracle."""
    from paper_1402_3501_amd import PATH_FP64
    rng = np.random.default_rng(p + 13)
    m, n, k = 2000, 1700, 333
    assert ((m + 127) // 128) * ((n + 127) // 128) >= 192
    rows = np.unique(np.concatenate([[0, m - 1], rng.choice(m, 40, replace=False)]))
    for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
        B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
        C = rng.integers(0, p, (m, n)).astype(np.int32)
        alpha, beta = int(rng.integers(1, p)), int(rng.integers(1, p))
        note("fgemm f64 128-tiles", p, m, n, k, ta, tb)
        Cd = dev(C)
        lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=PATH_FP64)
        got = host(Cd)
        As = np.ascontiguousarray(A[:, rows] if ta else A[rows])
        want = orc.fgemm(As, B, np.ascontiguousarray(C[rows]), p, alpha, beta, bool(ta), bool(tb))
        assert np.array_equal(got[rows], want), (p, ta, tb)


@pytest.mark.parametrize("p", [257, 32749])
def test_fgemm_int8_two_limbs(lib, orc, p):
    """Primes whose centred residues take two INT8 limbs (257 <= p <= 32749
    here): three shift classes, on the 64 x 64 blocks (with and without
    split K) and on the 128 x 128 blocks (sampled rows), all transposes."""
    from paper_1402_3501_amd import PATH_INT8, int8_limbs
    assert int8_limbs(p) == 2
    rng = np.random.default_rng(p + 17)
    for (m, n, k) in [(7, 5, 3), (130, 70, 333), (150, 260, 2000)]:
        for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
            B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
            C = rng.integers(0, p, (m, n)).astype(np.int32)
            alpha, beta = int(rng.integers(1, p)), int(rng.integers(0, p))
            note("fgemm two limbs", p, m, n, k, ta, tb)
            want = orc.fgemm(A, B, C, p, alpha, beta, bool(ta), bool(tb))
            Cd = dev(C)
            lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=PATH_INT8)
            assert np.array_equal(host(Cd), want), (p, m, n, k, ta, tb)
    m, n, k = 2100, 2050, 300  # 17 x 17 blocks of 128
    A = rng.integers(0, p, (m, k)).astype(np.int32)
    B = rng.integers(0, p, (k, n)).astype(np.int32)
    C = rng.integers(0, p, (m, n)).astype(np.int32)
    note("fgemm two limbs, 128 blocks", p)
    Cd = dev(C)
    lib.fgemm(dev(A), dev(B), Cd, p, 3, 5, path=PATH_INT8)
    got = host(Cd)
    rows = np.unique(np.concatenate([[0, m - 1], rng.choice(m, 40, replace=False)]))
    want = orc.fgemm(np.ascontiguousarray(A[rows]), B, np.ascontiguousarray(C[rows]), p, 3, 5)
    assert np.array_equal(got[rows], want)


def test_fgemm_int8_one_limb_wide_blocks(lib, orc):
    """One-limb products large enough for the 256 x 256 blocks (at least 256
    of them), with ragged edges in both dimensions, K not a multiple of the
    64-deep K tile, every transpose combination, alpha and beta; 40 sampled
    rows (plus the first and last) against the oracle."""
    from paper_1402_3501_amd import PATH_INT8
    p = 251
    rng = np.random.default_rng(29)
    m, n, k = 4000, 4100, 300
    assert ((m + 255) // 256) * ((n + 255) // 256) >= 256
    rows = np.unique(np.concatenate([[0, m - 1], rng.choice(m, 40, replace=False)]))
    for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        A = rng.integers(0, p, (k, m) if ta else (m, k)).astype(np.int32)
        B = rng.integers(0, p, (n, k) if tb else (k, n)).astype(np.int32)
        C = rng.integers(0, p, (m, n)).astype(np.int32)
        alpha, beta = int(rng.integers(1, p)), int(rng.integers(1, p))
        note("fgemm one limb wide", m, n, k, ta, tb)
        Cd = dev(C)
        lib.fgemm(dev(A), dev(B), Cd, p, alpha, beta, bool(ta), bool(tb), path=PATH_INT8)
        got = host(Cd)
        As = np.ascontiguousarray(A[:, rows] if ta else A[rows])
        want = orc.fgemm(As, B, np.ascontiguousarray(C[rows]), p, alpha, beta, bool(ta), bool(tb))
        assert np.array_equal(got[rows], want), (ta, tb)


def test_pluq_int8_two_limbs(lib, orc):
    """The factorisation with every product on two INT8 limbs (p = 32749),
    uniform and rank-deficient, element by element against the oracle."""
    from paper_1402_3501_amd import PATH_INT8
    p = 32749
    for A in [wl.uniform(600, 520, p, 41), wl.lowrank(700, 640, 300, p, 42)]:
        note("pluq two limbs", A.shape)
        want = orc.pluq(A, p)
        Ad = dev(A)
        res = lib.pluq(Ad, p, path=PATH_INT8)
        assert res.rank == want.rank
        assert np.array_equal(host(Ad), want.LU)
        assert np.array_equal(res.P.cpu().numpy(), want.P) and np.array_equal(res.Q.cpu().numpy(), want.Q)


def test_fgemm_int8_very_tall(lib, orc):
    """An INT8 request for a product taller than the limb split's grid
    (more than 65535 x 64 plane rows) runs on the FP64 path with the same
    bits instead of failing."""
    from paper_1402_3501_amd import PATH_INT8
    p = 251
    rng = np.random.default_rng(31)
    m, n, k = 4300000, 2, 3
    A = rng.integers(0, p, (m, k)).astype(np.int32)
    B = rng.integers(0, p, (k, n)).astype(np.int32)
    C = rng.integers(0, p, (m, n)).astype(np.int32)
    note("fgemm very tall", m, n, k)
    want = orc.fgemm(A, B, C, p, 7, 3)
    Cd = dev(C)
    lib.fgemm(dev(A), dev(B), Cd, p, 7, 3, path=PATH_INT8)
    assert np.array_equal(host(Cd), want)


def test_fgemm_submatrix_views(lib, orc):
    """Operands as strided views (leading dimension > columns, unaligned offsets)."""
    import torch
    p = 131071
    rng = np.random.default_rng(9)
    big = rng.integers(0, p, (300, 400)).astype(np.int32)
    G = dev(big)
    A = G[3:140, 5:70]        # 137 x 65
    B = G[150:215, 1:200]     # 65 x 199
    Cbig = torch.zeros((200, 260), dtype=torch.int32, device="cuda")
    Cv = Cbig[7:144, 31:230]
    note("fgemm views")
    lib.fgemm(A, B, Cv, p, 1, 0)
    want = orc.fgemm(big[3:140, 5:70], big[150:215, 1:200], np.zeros((137, 199), np.int32), p, 1, 0)
    got = host(Cbig)
    assert np.array_equal(got[7:144, 31:230], want)
    assert (got[:7] == 0).all() and (got[144:] == 0).all() and (got[:, :31] == 0).all()
    assert (got[:, 230:] == 0).all()


# ---------------------------------------------------------------- ftrsm
@pytest.mark.parametrize("p", [3, 65521, 131071, 8388593, 94906249])
def test_ftrsm_parity(lib, orc, p):
    rng = np.random.default_rng(p + 1)
    for path in paths_for(p):
        for side in (0, 1):
            for uplo in (0, 1):
                for trans in (0, 1):
                    for diag in (0, 1):
                        # d = 5 .. 600: the single-block, fused (<= 256) and recursive solves
                        for (m, n) in [(5, 3), (70, 33), (200, 129), (257, 40), (40, 600)]:
                            d = m if side == 0 else n
                            T = rng.integers(0, p, (d, d)).astype(np.int32)
                            T[np.arange(d), np.arange(d)] = rng.integers(1, p, d)
                            B = rng.integers(0, p, (m, n)).astype(np.int32)
                            alpha = int(rng.integers(1, p))
                            note("ftrsm", p, path, side, uplo, trans, diag, m, n)
                            want = orc.ftrsm(side, uplo, trans, diag, T, B, p, alpha)
                            Bd = dev(B)
                            lib.ftrsm(side, uplo, trans, diag, dev(T), Bd, p, alpha, path=path)
                            assert np.array_equal(host(Bd), want), (p, path, side, uplo, trans, diag, m, n)


# ---------------------------------------------------------------- flaswp
def test_flaswp_parity(lib):
    import torch
    rng = np.random.default_rng(3)
    for (m, n) in [(1, 1), (5, 7), (300, 129), (64, 1000)]:
        A = rng.integers(0, 1 << 30, (m, n)).astype(np.int32)
        for dim in (0, 1):
            perm = rng.permutation(m if dim == 0 else n).astype(np.int32)
            for inverse in (0, 1):
                note("flaswp", m, n, dim, inverse)
                Ad = dev(A)
                lib.flaswp(dim, Ad, torch.from_numpy(perm).cuda(), bool(inverse))
                got = host(Ad)
                want = A.copy()
                if dim == 0:
                    if inverse:
                        want[perm] = A
                    else:
                        want = A[perm]
                else:
                    if inverse:
                        want[:, perm] = A
                    else:
                        want = A[:, perm]
                assert np.array_equal(got, want)
                # apply then apply the inverse: identity
                lib.flaswp(dim, Ad, torch.from_numpy(perm).cuda(), not bool(inverse))
                assert np.array_equal(host(Ad), A)


# ---------------------------------------------------------------- pluq
def _pluq_compare(lib, orc, A, p, path, tag):
    note("pluq", tag, A.shape, p, path)
    want = orc.pluq(A, p, selfcheck=False)
    Ad = dev(A)
    res = lib.pluq(Ad, p, path=path)
    got = host(Ad)
    assert res.rank == want.rank, (tag, res.rank, want.rank)
    assert np.array_equal(host(res.P), want.P), tag
    assert np.array_equal(host(res.Q), want.Q), tag
    assert np.array_equal(got, want.LU), tag
    assert np.array_equal(host(res.rrp), want.rrp), tag
    assert np.array_equal(host(res.crp), want.crp), tag


def test_pluq_workload_512(lib, orc):
    """The 512 x 512 uniform matrix over Z/65521Z, on every path."""
    A = wl.make("pluq512_p65521")
    for path in paths_for(65521) + [0]:
        _pluq_compare(lib, orc, A, 65521, path, "512")


@pytest.mark.parametrize("p", [2, 3, 251, 65521, 131071, 8388593, 94906249])
def test_pluq_random_shapes(lib, orc, p):
    rng = np.random.default_rng(p * 7 + 1)
    shapes = [(1, 1), (1, 9), (9, 1), (2, 2), (13, 7), (40, 300), (300, 40), (129, 257), (260, 260),
              (700, 300), (1, 2000), (1500, 3)]
    for path in paths_for(p):
        for (m, n) in shapes:
            r = int(rng.integers(0, min(m, n) + 1))
            A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
            _pluq_compare(lib, orc, A, p, path, f"lowrank r={r}")
            if m * n <= 100000:
                A = rng.integers(0, p, (m, n)).astype(np.int32)
                _pluq_compare(lib, orc, A, p, path, "uniform")


@pytest.mark.parametrize("p", [251, 65521, 131071])
def test_pluq_auto_rank_deficient(lib, orc, p):
    """The AUTO path on rank-deficient inputs of moderate size: the general
    recursion with its second stream, the generic-prefix and zero-block
    shortcuts, and workspace sized by the AUTO rule."""
    rng = np.random.default_rng(p + 11)
    for (m, n, r) in [(300, 260, 170), (257, 300, 100), (700, 300, 250), (1000, 900, 600), (130, 1100, 90)]:
        A = wl.lowrank(m, n, r, p, int(rng.integers(1 << 40)))
        _pluq_compare(lib, orc, A, p, 0, f"auto lowrank r={r}")


def test_pluq_special_matrices(lib, orc):
    p = 131071
    rng = np.random.default_rng(17)
    cases = {
        "zero": np.zeros((150, 170), np.int32),
        "identity": np.eye(300, dtype=np.int32),
        "rank1": (np.outer(rng.integers(0, p, 333) * (rng.random(333) < 0.3),
                           rng.integers(0, p, 200) * (rng.random(200) < 0.5)) % p).astype(np.int32),
    }
    for n in (5, 130, 600):
        pi = rng.permutation(n)
        M = np.zeros((n, n), np.int32)
        M[np.arange(n), pi] = 1
        cases[f"perm{n}"] = M
    # scattered pivots with many empty rows / columns
    S = np.zeros((400, 500), np.int32)
    rows = rng.choice(400, 60, replace=False)
    cols = rng.choice(500, 60, replace=False)
    S[rows, cols] = rng.integers(1, p, 60)
    cases["sparse"] = S
    for tag, A in cases.items():
        for path in paths_for(p):
            _pluq_compare(lib, orc, A, p, path, tag)


def test_pluq_empty(lib):
    import torch
    for (m, n) in [(0, 0), (0, 5), (4, 0)]:
        A = torch.zeros((m, n), dtype=torch.int32, device="cuda")
        note("pluq empty", m, n)
        res = lib.pluq(A, 7)
        assert res.rank == 0
        assert np.array_equal(host(res.P), np.arange(m)) and np.array_equal(host(res.Q), np.arange(n))


def test_pluq_repeatable(lib):
    """Bitwise-identical outputs across runs and streams."""
    import torch
    p = 65521
    A = wl.lowrank(900, 700, 350, p, 4242)
    outs = []
    for trial in range(3):
        s = torch.cuda.Stream() if trial == 2 else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            Ad = dev(A)
            note("pluq repeat", trial)
            res = lib.pluq(Ad, p)
            outs.append((host(Ad), host(res.P), host(res.Q), res.rank))
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o[:3], outs[0][:3])) and o[3] == outs[0][3]


def test_pluq_checks_medium(lib, orc):
    """A rank-deficient 2000 x 1800 matrix: compare with the oracle and run the
    any-size property checks used at full size."""
    p = 131071
    A = wl.lowrank(2000, 1800, 900, p, 99)
    _pluq_compare(lib, orc, A, p, 1, "medium")
    Ad = dev(A)
    res = lib.pluq(Ad, p)
    err = checks.full_check(A, host(Ad), host(res.P), host(res.Q), res.rank, p, orc.order, exact_limit=0)
    assert err is None, err


def test_pluq_general_path_on_generic_inputs(lib, orc):
    """Generic-rank-profile inputs normally take the speculative path; the
    general recursion (FFP_PLUQ_GENERAL_ONLY=1) must give the same bits."""
    import os
    p = 65521
    rng = np.random.default_rng(31)
    for (m, n) in [(300, 300), (257, 129), (129, 400)]:
        A = rng.integers(0, p, (m, n)).astype(np.int32)
        os.environ["FFP_PLUQ_GENERAL_ONLY"] = "1"
        try:
            _pluq_compare(lib, orc, A, p, 0, "general-only")
        finally:
            del os.environ["FFP_PLUQ_GENERAL_ONLY"]
        _pluq_compare(lib, orc, A, p, 0, "speculative")


@pytest.mark.parametrize("p", [131071, 8388593, 94906249])
def test_pluq_tall_and_wide_generic_panels(lib, orc, p):
    """Generic blocks with one long side: a leading 128 x 128 tile whose two
    panel solves together span more than 16384 vectors run the paired base
    solve on 32-vector slabs, here with ragged slabs on both sides (72 and
    16372 vectors); p = 94906249 reduces inside those solves."""
    rng = np.random.default_rng(p % 1000 + 5)
    for (m, n) in [(16500, 200), (200, 16500)]:
        A = rng.integers(0, p, (m, n)).astype(np.int32)
        _pluq_compare(lib, orc, A, p, 0, f"generic panels {m}x{n}")


@pytest.mark.parametrize("p", [251, 32749, 8388593])
def test_pluq_int8_paired_panel_products(lib, orc, p):
    """Generic blocks on the INT8 path whose leading tile exceeds the 256
    base, so the paired solves run their two inner products (64 x 524 x 512
    and 724 x 64 x 512 here, ragged in every dimension) as one limb split
    and one product grid, for one, two and three limbs."""
    from paper_1402_3501_amd import PATH_INT8
    rng = np.random.default_rng(p % 997 + 11)
    m, n = 1300, 1100
    # A = L U with L unit lower trapezoidal and U upper with a nonzero
    # diagonal: every leading minor is nonzero, so the whole factorisation
    # takes the generic path (sums below 1100 p^2 < 2^63)
    Lm = np.tril(rng.integers(0, p, (m, n), dtype=np.int64), -1)
    Lm[np.arange(n), np.arange(n)] = 1
    U = np.triu(rng.integers(0, p, (n, n), dtype=np.int64), 1)
    U[np.arange(n), np.arange(n)] = rng.integers(1, p, n)
    A = ((Lm @ U) % p).astype(np.int32)
    want = orc.pluq(A, p, selfcheck=False)
    assert np.array_equal(want.P, np.arange(m)) and np.array_equal(want.Q, np.arange(n))
    _pluq_compare(lib, orc, A, p, PATH_INT8, "int8 paired panel products")


def test_pluq_generic_prefix_shortcuts(lib, orc):
    """Rank-deficient inputs whose leading minors are nonzero up to some order
    k0: the failed generic attempt's k0 lets leading tiles within that order
    factor as plain LU, and zero sub-blocks skip their recursion.  Cases: the
    shortcut at the top node's tile, one level down, with a nonzero Schur
    complement after it, and a full-rank input whose first vanishing minor is
    planted at order 200 (the rest of the recursion is the general one)."""
    p = 131071
    rng = np.random.default_rng(77)
    cases = [("lowrank 1024 r300", wl.lowrank(1024, 1024, 300, p, 701)),
             ("lowrank 600 r450", wl.lowrank(600, 600, 450, p, 702)),
             ("lowrank 700x900 r500", wl.lowrank(700, 900, 500, p, 703))]
    B = rng.integers(0, p, (640, 640)).astype(np.int32)
    B[:200, :200] = wl.lowrank(200, 200, 199, p, 704)
    cases.append(("planted minor 200", B))
    for tag, A in cases:
        for path in paths_for(p):
            _pluq_compare(lib, orc, A, p, path, tag)
    # 4096 x 4096 with its first vanishing minor at order 300: the generic
    # attempt stops at its checkpoint after the leading 1024 block
    B = rng.integers(0, p, (4096, 4096)).astype(np.int32)
    B[:300, :300] = wl.lowrank(300, 300, 299, p, 705)
    _pluq_compare(lib, orc, B, p, 0, "planted minor 300, 4096")
