"""GPU checks of the asynchronous and validating entry points.

ffp_lu_nopiv (the plain LU of a generic-rank-profile input, no host
synchronisation) against the oracle's PLUQ, whose P and Q are then the
identity; its zero-pivot report against the leading minors the oracle finds;
ffp_check_range on in-range and out-of-range entries; the batched call's
handling of a shape beyond its declared bounds.
"""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("p", [65521, 131071, 8388593])
def test_lu_nopiv_matches_oracle(lib, orc, p):
    """Uniform inputs (generic rank profile with high probability, which the
    oracle confirms: P = Q = identity) give the oracle's L\\U bit for bit."""
    for path in (lib.PATH_FP64, lib.PATH_INT8, lib.PATH_AUTO):
        for (m, n, seed) in [(64, 64, 1), (200, 130, 2), (513, 700, 3), (1100, 1000, 4)]:
            note("lu_nopiv", m, n, p, path)
            A = wl.uniform(m, n, p, seed)
            want = orc.pluq(A, p, selfcheck=False)
            k = min(m, n)
            assert want.rank == k
            assert np.array_equal(want.P, np.arange(m)) and np.array_equal(want.Q, np.arange(n))
            Ad = dev(A)
            info = lib.lu_nopiv(Ad, p, path=path)
            assert int(host(info)[0]) == 0
            assert np.array_equal(host(Ad), want.LU)


def test_lu_nopiv_reports_first_zero_pivot(lib, orc):
    """A matrix whose leading minors are nonzero up to order t and vanish at
    order t + 1: info = t + 1 (1 + the index of the zero pivot)."""
    p = 131071
    rng = np.random.default_rng(5)
    for (n, t) in [(70, 0), (300, 99), (600, 256), (900, 640)]:
        A = wl.uniform(n, n, p, 10 + t).astype(np.int64)
        # row t restricted to the first t + 1 columns: a combination of rows 0..t-1
        c = rng.integers(0, p, t)
        A[t, :t + 1] = (c @ A[:t, :t + 1]) % p if t else 0
        A = A.astype(np.int32)
        # the oracle's ranks of the leading blocks confirm the construction
        assert orc.pluq(np.ascontiguousarray(A[:t + 1, :t + 1]), p, selfcheck=False).rank == t
        if t:
            assert orc.pluq(np.ascontiguousarray(A[:t, :t]), p, selfcheck=False).rank == t
        note("lu_nopiv zero pivot", n, t)
        info = lib.lu_nopiv(dev(A), p)
        assert int(host(info)[0]) == t + 1


def test_lu_nopiv_graph_capture(lib, orc):
    """The asynchronous LU captured in a HIP graph and replayed: every replay
    equals the eager result."""
    import torch
    p = 65521
    A = wl.uniform(384, 384, p, 21)
    want = orc.pluq(A, p, selfcheck=False).LU
    A0 = dev(A)
    Ad = A0.clone()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(lib.lu_nopiv_workspace(384, 384, p), dtype=torch.uint8, device="cuda")
    lib.lu_nopiv(Ad, p, info=info, ws=ws)
    assert np.array_equal(host(Ad), want)
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    Ad.copy_(A0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        lib.lu_nopiv(Ad, p, info=info, ws=ws)
    for rep in range(3):
        Ad.copy_(A0)
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(host(info)[0]) == 0, rep
        assert np.array_equal(host(Ad), want), rep


def test_check_range(lib):
    p = 251
    A = wl.uniform(300, 500, p, 3)
    assert lib.check_range(dev(A), p)
    for (i, j, v) in [(0, 0, p), (299, 499, -1), (150, 3, 1 << 30)]:
        B = A.copy()
        B[i, j] = v
        assert not lib.check_range(dev(B), p)
    import ctypes
    import torch
    B = dev(np.full((4, 4), p, np.int32))
    rc = lib.load().ffp_check_range(4, 4, p, ctypes.c_void_p(B.data_ptr()), 4,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -105


def test_batched_rejects_shape_beyond_bounds(lib, orc):
    """A matrix whose declared shape exceeds max_m / max_n is left untouched
    with rank -1; the others are factored as usual."""
    import torch
    p = 65521
    ms, ns, rs, Ab, off = wl.batch(5, 16, 60, p, 31)
    max_m, max_n = int(ms.max()), int(ns.max())
    ns_bad = ns.copy()
    ns_bad[2] = max_n + 5
    ms_d, ns_d = dev(ms).view(-1), dev(ns_bad).view(-1)
    P_off = np.zeros(5, np.int64)
    Q_off = np.zeros(5, np.int64)
    P_off[1:] = np.cumsum(ms)[:-1]
    Q_off[1:] = np.cumsum(ns)[:-1]
    Abd = dev(Ab).view(-1)
    P = torch.zeros(int(ms.sum()), dtype=torch.int32, device="cuda")
    Q = torch.zeros(int(ns.sum()) + 8, dtype=torch.int32, device="cuda")
    rank = torch.zeros(5, dtype=torch.int32, device="cuda")
    ws = torch.empty(lib.load().ffp_pluq_batched_workspace(5, max_m, max_n, p, 0), dtype=torch.uint8,
                     device="cuda")
    lib.pluq_batched_into(ms_d, ns_d, max_m, max_n, Abd, torch.from_numpy(off).cuda(), P,
                          torch.from_numpy(P_off).cuda(), Q, torch.from_numpy(Q_off).cuda(), rank, None, None,
                          ws, p)
    got_rank = host(rank)
    LU = host(Abd)
    for i in range(5):
        Ai = Ab[off[i]:off[i] + ms[i] * ns[i]]
        if i == 2:
            assert got_rank[i] == -1
            assert np.array_equal(LU[off[i]:off[i] + ms[i] * ns[i]], Ai)
        else:
            assert got_rank[i] == rs[i]
            want = orc.pluq(Ai.reshape(ms[i], ns[i]), p, selfcheck=False)
            assert np.array_equal(LU[off[i]:off[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]), want.LU)
