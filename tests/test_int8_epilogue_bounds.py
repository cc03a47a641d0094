"""Host-side check of the INT8 product epilogue's arithmetic (no GPU).

The kernel recombines the shift-class sums S_s (int32, |S_s| < 2^31) of a
limb product by Horner's rule in doubles,
    t = (..(S_{NS-1} 256 + S_{NS-2}) 256 ..) 256 + S_0,
with one rounded-quotient reduction after the third class when there are
five classes (three limbs), and a floored-quotient reduction at the end.
The delayed-reduction argument of Section 3.1 makes this exact when every
intermediate stays below 2^53.  This test replays those steps with exact
integers for the values and float64 for the quotients, as the device does,
on extreme class sums and the largest primes of each limb count, and
compares the result with sum_s 256^s S_s mod p.
"""
import itertools

import numpy as np

LIM = 2 ** 53
S_MAX = 2 ** 31 - 1


def _q_round(x, p):
    return int(np.rint(np.float64(x) * np.float64(1.0 / p)))


def _q_floor(x, p):
    return int(np.floor(np.float64(x) * np.float64(1.0 / p)))


def _epilogue(S, p):
    """The kernel's recombination of the class sums S[0..NS-1]."""
    ns = len(S)
    seen = []
    t = S[ns - 1]
    for s in range(ns - 2, -1, -1):
        t = t * 256 + S[s]
        seen.append(t)
        if ns == 5 and s == 2:
            t = t - _q_round(t, p) * p
            seen.append(t)
    q = _q_floor(t, p)
    seen.append(q * p)
    r = t - q * p
    r = r + p if r < 0 else r
    r = r - p if r >= p else r
    return r, max(abs(v) for v in seen)


def _digits(c, limbs):
    """Balanced base-256 digits of the centred residues c, as the limb split
    forms them (the last digit takes what remains)."""
    out = []
    for d in range(limbs):
        if d == limbs - 1:
            out.append(c)
        else:
            dig = ((c + 128) & 255) - 128
            out.append(dig)
            c = (c - dig) >> 8
    return out


# the largest prime of each limb count, and the inner-dimension chunk after
# which the product reduces (one int32 accumulator per shift class)
LARGEST = {1: (251, 131072), 2: (65269, 65536), 3: (16711421, 32768)}


def test_largest_primes_have_their_limb_counts():
    import paper_1402_3501_amd as ffp
    lib = ffp.load()
    for limbs, (p, _) in LARGEST.items():
        assert lib.ffp_is_prime(p) == 1 and lib.ffp_int8_limbs(p) == limbs
        # the next primes take more limbs (or none)
        for q in range(p + 1, p + 400):
            if lib.ffp_is_prime(q):
                assert lib.ffp_int8_limbs(q) != limbs, (limbs, q)


def test_class_sums_fit_int32():
    """Over a K chunk every shift class sum fits an int32, by the exact
    digit ranges of all centred residues of the largest prime."""
    for limbs, (p, kchunk) in LARGEST.items():
        h = (p - 1) // 2
        c = np.arange(-h, h + 1, dtype=np.int64)
        dmax = [int(np.abs(x).max()) for x in _digits(c, limbs)]
        for s in range(2 * limbs - 1):
            per_k = sum(dmax[i] * dmax[s - i] for i in range(limbs) if 0 <= s - i < limbs)
            assert kchunk * per_k < 2 ** 31, (limbs, p, s, dmax)


def test_horner_recombination_exact_at_extremes():
    primes = {3: [65521, 8388593, 16711421], 2: [257, 32749, 65269]}
    rng = np.random.default_rng(7)
    for limbs, ps in primes.items():
        ns = 2 * limbs - 1
        cases = [list(c) for c in itertools.product([S_MAX, -S_MAX, 0], repeat=ns)]
        cases += [[int(x) for x in rng.integers(-S_MAX, S_MAX + 1, ns)] for _ in range(2000)]
        for p in ps:
            for S in cases:
                got, peak = _epilogue(S, p)
                want = sum(s * 256 ** i for i, s in enumerate(S)) % p
                assert peak < LIM, (p, S, peak)
                assert got == want, (p, S, got, want)


def test_one_limb_needs_no_recombination():
    for p in [2, 3, 251]:
        for s in [S_MAX, -S_MAX, 12345, -1]:
            got, peak = _epilogue([s], p)
            assert peak < LIM and got == s % p
