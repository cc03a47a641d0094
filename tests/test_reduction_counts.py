"""The modular-reduction counts of Section 3.1 (Table 2), reproduced by
running the library's tile-iterative LU loops in counting mode (host only,
no kernel launched) and the halving recursions of the two recursive
algorithms, under the model the paper states: a product m x k by k x n
costs m n reductions, a unit triangular solve (m - 1) n, a non-unit one
(2 m - 1) n, a k x k base case 3/2 k^2 - 7/2 k + 3.

Closed forms, n x n, tile k dividing n (Table 2):
  right-looking  n^3 / (3k) + (1 - 1/k) n^2 + (k/6 - 5/2 + 3/k) n
  Crout          (5/2 - 1/k) n^2 + (-2k - 5/2 + 3/k) n + k^2
  left-looking   (2 - 1/(2k)) n^2 + (-5k/2 - 1 + 2/k) n + 2k^2 - 2k + 1
  tile recursive 2 n^2 - n log2 n - n
  slab recursive (1 + log2(n) / 4) n^2 - n log2(n) / 2 - n

Right-looking, Crout and both recursive counts come out exactly.  The
left-looking loop of Table 1 under the same model gives the printed form
plus (n/k - 1)(2k - 1)(k - 1), which vanishes at k = 1 (the iterative
left-looking row); the printed form cannot come from that loop (see the
design notes, reading 13).
"""
from fractions import Fraction as Fr
import math

import pytest

import paper_1402_3501_amd as ffp


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(ffp.LIB_PATH):
        from paper_1402_3501_amd import build
        build.build()
    return ffp.load()


SIZES = [(8, 1), (8, 2), (8, 4), (12, 3), (24, 4), (60, 5), (64, 8), (96, 12), (212 * 5, 212), (3000, 1000)]


def right_cf(n, k):
    return Fr(n ** 3, 3 * k) + (1 - Fr(1, k)) * n * n + (Fr(k, 6) - Fr(5, 2) + Fr(3, k)) * n


def crout_cf(n, k):
    return (Fr(5, 2) - Fr(1, k)) * n * n + (-2 * k - Fr(5, 2) + Fr(3, k)) * n + k * k


def left_cf(n, k):
    return (2 - Fr(1, 2 * k)) * n * n + (-Fr(5, 2) * k - 1 + Fr(2, k)) * n + 2 * k * k - 2 * k + 1


@pytest.mark.parametrize("n,k", SIZES)
def test_right_looking(lib, n, k):
    assert ffp.reduction_count(ffp.LU_RIGHT, n, k) == right_cf(n, k)


@pytest.mark.parametrize("n,k", SIZES)
def test_crout(lib, n, k):
    assert ffp.reduction_count(ffp.LU_CROUT, n, k) == crout_cf(n, k)


@pytest.mark.parametrize("n,k", SIZES)
def test_left_looking(lib, n, k):
    got = ffp.reduction_count(ffp.LU_LEFT, n, k)
    assert got == left_cf(n, k) + (n // k - 1) * (2 * k - 1) * (k - 1)
    if k == 1:
        assert got == Fr(3, 2) * n * n - Fr(3, 2) * n + 1   # the iterative left-looking row


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 256, 4096, 16384])
def test_tile_recursive(lib, n):
    L = int(math.log2(n))
    assert ffp.reduction_count(ffp.LU_TILE_RECURSIVE, n) == 2 * n * n - n * L - n


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 256, 4096, 16384])
def test_slab_recursive(lib, n):
    L = int(math.log2(n))
    assert ffp.reduction_count(ffp.LU_SLAB_RECURSIVE, n) == (1 + Fr(L, 4)) * n * n - Fr(n * L, 2) - n


def test_k1_rows():
    """The k = 1 rows of Table 2 against the blocked forms at k = 1: the
    right-looking and Crout rows leave out the 1 x 1 base case (n and 2n - 2
    fewer), the left-looking row equals its blocked form."""
    for n in (4, 10, 100):
        assert ffp.reduction_count(ffp.LU_RIGHT, n, 1) - (Fr(n ** 3, 3) - Fr(n, 3)) == n
        assert ffp.reduction_count(ffp.LU_CROUT, n, 1) - (Fr(3, 2) * n * n - Fr(7, 2) * n + 3) == 2 * n - 2
        assert ffp.reduction_count(ffp.LU_LEFT, n, 1) == Fr(3, 2) * n * n - Fr(3, 2) * n + 1


def test_orderings_stated_in_the_text():
    """Section 3.1: the tiled recursive algorithm needs fewer reductions than
    the Crout variant for 2 <= k <= n/4, and the right-looking variant needs
    the most."""
    for n in (256, 1024, 4096):
        tr = ffp.reduction_count(ffp.LU_TILE_RECURSIVE, n)
        k = 2
        while k <= n // 4:
            c = ffp.reduction_count(ffp.LU_CROUT, n, k)
            r = ffp.reduction_count(ffp.LU_RIGHT, n, k)
            assert tr < c, (n, k)
            assert r > c and r > ffp.reduction_count(ffp.LU_LEFT, n, k), (n, k)
            k *= 2
