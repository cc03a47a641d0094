"""The allocation-free product (ffp_fgemm_noalloc) against ffp_fgemm.

Both are called directly through the C ABI on the same device buffers; the
no-allocation call must give the same bits as the call with a caller
workspace, on two calls in a row (the second smaller, so that it reuses the
fixed scratch array with stale contents of the first), on both arithmetic
paths and on AUTO, and an INT8 request beyond the scratch array must be
refused before anything runs.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FFP_E_SCRATCH = -109


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _call(lib, fn, ta, tb, A, B, C, p, alpha, beta, path, ws=None):
    import torch
    m, n = C.shape
    k = A.shape[0] if ta else A.shape[1]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [ta, tb, m, n, k, p, alpha, ctypes.c_void_p(A.data_ptr()), A.shape[1], ctypes.c_void_p(B.data_ptr()),
            B.shape[1], beta, ctypes.c_void_p(C.data_ptr()), C.shape[1], path]
    if fn == "ffp_fgemm":
        need = lib.ffp_fgemm_workspace(ta, tb, m, n, k, p, path)
        w = torch.empty(max(int(need), 1), dtype=torch.uint8, device="cuda")
        rc = lib.ffp_fgemm(*args, ctypes.c_void_p(w.data_ptr()), int(need), s)
    else:
        rc = lib.ffp_fgemm_noalloc(*args, s)
    torch.cuda.synchronize()
    return rc


def _rand(rng, shape, p):
    import torch
    return torch.from_numpy(rng.integers(0, p, shape).astype(np.int32)).cuda()


@pytest.mark.parametrize("p", [251, 131071, 8388593])
def test_noalloc_matches_fgemm(lib, p):
    raw = lib.load()
    from paper_1402_3501_amd import PATH_AUTO, PATH_FP64, PATH_INT8
    rng = np.random.default_rng(p + 17)
    # a product that fills the chip, then a smaller one (split K over
    # several workgroups, transposed operands) that reuses the scratch array
    for path in (PATH_INT8, PATH_AUTO, PATH_FP64):
        for (m, n, k, ta, tb) in [(1500, 1300, 1100, 0, 0), (150, 260, 2000, 1, 1)]:
            A = _rand(rng, (k, m) if ta else (m, k), p)
            B = _rand(rng, (n, k) if tb else (k, n), p)
            C0 = _rand(rng, (m, n), p)
            alpha, beta = int(rng.integers(0, p)), int(rng.integers(0, p))
            note("noalloc", p, path, m, n, k, ta, tb)
            Cw = C0.clone()
            Cs = C0.clone()
            assert _call(raw, "ffp_fgemm", ta, tb, A, B, Cw, p, alpha, beta, path) == 0
            assert _call(raw, "ffp_fgemm_noalloc", ta, tb, A, B, Cs, p, alpha, beta, path) == 0
            assert np.array_equal(Cs.cpu().numpy(), Cw.cpu().numpy()), (p, path, m, n, k)


def test_noalloc_refuses_oversized_int8(lib):
    raw = lib.load()
    import torch
    from paper_1402_3501_amd import PATH_AUTO, PATH_INT8
    p = 131071
    cap = int(raw.ffp_noalloc_scratch_bytes())
    assert cap == 64 << 20
    # 3 limbs x (4096 + 4096) rows x 4096 deep = 96 MiB of limb planes
    m = n = k = 4096
    assert raw.ffp_fgemm_workspace(0, 0, m, n, k, p, PATH_INT8) > cap
    A = torch.zeros((m, k), dtype=torch.int32, device="cuda")
    B = torch.zeros((k, n), dtype=torch.int32, device="cuda")
    C = torch.full((m, n), 5, dtype=torch.int32, device="cuda")
    note("noalloc refuse", m, n, k)
    assert _call(raw, "ffp_fgemm_noalloc", 0, 0, A, B, C, p, 1, 1, PATH_INT8) == FFP_E_SCRATCH
    assert int((C != 5).sum()) == 0  # nothing ran
    # AUTO takes the FP64 path for it (no workspace): 0 * 0 + 1 * C = C
    B.fill_(1)
    A[:, 0] = 2
    assert _call(raw, "ffp_fgemm_noalloc", 0, 0, A, B, C, p, 1, 1, PATH_AUTO) == 0
    assert int((C != 7).sum()) == 0
