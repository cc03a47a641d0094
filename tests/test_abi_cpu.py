"""Host-side checks of the C-ABI library (no GPU needed: no kernel is launched).

The library must load, export every function declared in include/ffpluq.h,
reject invalid arguments with the documented codes before touching the
device, and convert between index vectors and swap sequences.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1402_3501_amd as ffp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffpluq.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ffp.LIB_PATH):
        from paper_1402_3501_amd import build
        build.build()
    return ffp.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_scalar_helpers(lib):
    for p in (2, 3, 251, 65521, 131071, 8388593, 94906249, 16711421):
        assert ffp.is_prime(p)
    for p in (0, 1, 4, 65535, 131073):
        assert not ffp.is_prime(p)
    assert ffp.int8_limbs(251) == 1
    assert ffp.int8_limbs(65521) == 3 and ffp.int8_limbs(131071) == 3
    assert ffp.int8_limbs(8388593) == 3
    assert ffp.int8_limbs(16711421) == 3 and ffp.int8_limbs(16711423 + 2) == 0
    assert ffp.int8_limbs(2 * 127 * 257 + 1) == 2
    assert "ffpluq" in ffp.version()
    assert lib.ffp_error_string(-103) == b"workspace missing or too small"
    for code in range(-101, -109, -1):  # every documented code has its own message
        assert lib.ffp_error_string(code) not in (b"", b"unknown error")


def test_argument_validation_before_device(lib):
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    # negative sizes -> -i
    assert lib.ffp_fgemm(0, 0, -1, 4, 4, 7, 1, fake, 4, fake, 4, 0, fake, 4, 0, None, 0, None) == -3
    assert lib.ffp_fgemm(2, 0, 4, 4, 4, 7, 1, fake, 4, fake, 4, 0, fake, 4, 0, None, 0, None) == -1
    # non-prime and out-of-range p
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 9, 1, fake, 4, fake, 4, 0, fake, 4, 0, None, 0, None) == -101
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 8388593, 1, fake, 4, fake, 4, 0, fake, 4, 0, None, 0, None) != -102
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 2147483647, 1, fake, 4, fake, 4, 0, fake, 4, 1, None, 0, None) == -102
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 94906249 + 2 * 3, 1, fake, 4, fake, 4, 0, fake, 4, 1, None, 0,
                         None) in (-101, -102)
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 65537, 1, fake, 4, fake, 4, 0, fake, 4, 2, None, 0, None) != -102
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 16777259, 1, fake, 4, fake, 4, 0, fake, 4, 2, None, 0, None) == -102
    # alpha / beta outside [0, p)
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 7, 7, fake, 4, fake, 4, 0, fake, 4, 0, None, 0, None) == -7
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 7, 1, fake, 4, fake, 4, 9, fake, 4, 0, None, 0, None) == -12
    # leading dimensions
    assert lib.ffp_fgemm(0, 0, 4, 5, 3, 7, 1, fake, 2, fake, 5, 0, fake, 5, 0, None, 0, None) == -9
    assert lib.ffp_fgemm(0, 0, 4, 5, 3, 7, 1, fake, 3, fake, 4, 0, fake, 5, 0, None, 0, None) == -11
    assert lib.ffp_fgemm(0, 0, 4, 5, 3, 7, 1, fake, 3, fake, 5, 0, fake, 4, 0, None, 0, None) == -14
    # bad path
    assert lib.ffp_fgemm(0, 0, 4, 4, 4, 7, 1, fake, 4, fake, 4, 0, fake, 4, 5, None, 0, None) == -15
    # empty problems succeed without touching memory
    assert lib.ffp_fgemm(0, 0, 0, 4, 4, 7, 1, None, 4, None, 4, 0, None, 4, 0, None, 0, None) == 0
    # ftrsm
    assert lib.ffp_ftrsm(3, 0, 0, 0, 4, 4, 7, 1, fake, 4, fake, 4, 0, None, 0, None) == -1
    assert lib.ffp_ftrsm(0, 0, 0, 0, 4, 4, 7, 1, fake, 3, fake, 4, 0, None, 0, None) == -10
    assert lib.ffp_ftrsm(0, 0, 0, 0, 4, 4, 10, 1, fake, 4, fake, 4, 0, None, 0, None) == -101
    # flaswp: workspace required
    assert lib.ffp_flaswp(0, 4, 4, fake, 4, fake, 0, None, 0, None) == -103
    assert lib.ffp_flaswp(2, 4, 4, fake, 4, fake, 0, None, 0, None) == -1
    # pluq
    r = ctypes.c_int64(0)
    assert lib.ffp_pluq(4, 4, 6, fake, 4, fake, fake, None, ctypes.byref(r), None, None, 0, None, 0,
                        None) == -101
    assert lib.ffp_pluq(4, 4, 7, fake, 3, fake, fake, None, ctypes.byref(r), None, None, 0, None, 0,
                        None) == -5
    assert lib.ffp_pluq(4, 4, 7, fake, 4, fake, fake, None, ctypes.byref(r), None, None, 0, None, 0,
                        None) == -103
    # batched
    assert lib.ffp_pluq_batched(-1, fake, fake, 4, 4, 7, fake, fake, fake, fake, fake, fake, fake, None,
                                None, 0, None, 0, None) == -1
    assert lib.ffp_pluq_batched(3, fake, fake, 2000, 4, 7, fake, fake, fake, fake, fake, fake, fake, None,
                                None, 0, None, 0, None) == -4
    # lu_nopiv
    assert lib.ffp_lu_nopiv(4, 4, 9, fake, 4, fake, 0, None, 0, None) == -101
    assert lib.ffp_lu_nopiv(4, 4, 7, fake, 4, fake, 4, None, 0, None) == -7
    assert lib.ffp_lu_nopiv(4, 4, 7, fake, 3, fake, 0, None, 0, None) == -5
    assert lib.ffp_lu_nopiv(4, 4, 7, fake, 4, None, 0, None, 0, None) == -6
    assert lib.ffp_lu_nopiv(4, 4, 7, fake, 4, fake, 0, None, 0, None) == -103
    # check_range
    assert lib.ffp_check_range(-1, 4, 7, fake, 4, None) == -1
    assert lib.ffp_check_range(4, 4, 1, fake, 4, None) == -3
    assert lib.ffp_check_range(4, 4, 7, fake, 3, None) == -5
    assert lib.ffp_check_range(0, 4, 7, None, 4, None) == 0


def test_workspace_queries(lib):
    assert lib.ffp_fgemm_workspace(0, 0, 64, 64, 64, 131071, 1) == 0
    assert lib.ffp_pluq_workspace(512, 512, 65521, 1) >= 512 * 512 * 4
    assert lib.ffp_flaswp_workspace(0, 100, 50) >= 100 * 50 * 4
    assert lib.ffp_pluq_workspace(0, 0, 7, 1) > 0


def test_auto_path_crossover(lib):
    """AUTO takes INT8 products from 0.5e9 field operations (several limbs) and,
    with one limb, from k >= 128 and 256 x 256 outputs."""
    assert lib.ffp_auto_path(131071, 768, 768, 768) == 2       # 0.91e9
    assert lib.ffp_auto_path(131071, 512, 512, 512) == 1       # 0.27e9
    assert lib.ffp_auto_path(131071, 1024, 1024, 256) == 2     # 0.54e9
    assert lib.ffp_auto_path(8388593, 256, 2048, 256) == 1     # 0.27e9
    assert lib.ffp_auto_path(8388593, 992, 1008, 250) == 1     # 0.49999e9
    assert lib.ffp_auto_path(8388593, 1000, 1000, 250) == 2    # exactly 0.5e9
    assert lib.ffp_auto_path(251, 256, 256, 128) == 2
    assert lib.ffp_auto_path(251, 256, 256, 127) == 1
    assert lib.ffp_auto_path(94906249, 8192, 8192, 8192) == 1  # beyond the INT8 limbs


def test_workspace_covers_split_k(lib):
    """A lone INT8 product's workspace holds the limb planes and room for the
    split-K partial results (at most 4 parts of m x n int32, at most 32 MiB);
    the AUTO PLUQ workspace is at least the FP64 one."""
    m, n, k = 300, 260, 2000                 # 3 x 3 output blocks, 32 K tiles
    planes = 3 * (384 + 384) * 2048          # 3 limbs, padded rows x padded K
    split = 4 * 384 * 384 * 4
    assert lib.ffp_fgemm_workspace(0, 0, m, n, k, 131071, 2) >= planes + split
    big = lib.ffp_fgemm_workspace(0, 0, 16384, 16384, 16384, 131071, 2)
    assert big >= 3 * 2 * 16384 * 16384 and big < 3 * 2 * 16384 * 16384 + (33 << 20)
    for (mm, nn) in [(300, 260), (2048, 2048), (8192, 8192)]:
        assert lib.ffp_pluq_workspace(mm, nn, 131071, 0) >= lib.ffp_pluq_workspace(mm, nn, 131071, 1)


def test_perm_swaps_roundtrip(lib):
    rng = np.random.default_rng(0)
    for n in (0, 1, 2, 5, 17, 100):
        perm = rng.permutation(n).astype(np.int32)
        ipiv = ffp.perm_to_swaps(perm)
        assert (ipiv >= np.arange(n)).all()
        # applying the swaps in order to the identity gives back the permutation
        arr = list(range(n))
        for i, j in enumerate(ipiv):
            arr[i], arr[j] = arr[j], arr[i]
        assert arr == perm.tolist()
        assert np.array_equal(ffp.swaps_to_perm(ipiv), perm)
    with pytest.raises(ffp.FFPError):
        ffp.perm_to_swaps(np.array([0, 0, 1], np.int32))


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU: asked for more it exits with a message
    before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
