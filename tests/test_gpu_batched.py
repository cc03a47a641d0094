"""Batched PLUQ in one persistent launch: every matrix's outputs equal the
oracle's for that matrix alone (bit for bit), on mixed shapes and ranks."""
import sys

import numpy as np
import pytest

import checks
import workloads as wl

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(lib, ms, ns, A, off, p):
    import torch
    dev = "cuda"
    msd = torch.from_numpy(np.asarray(ms, np.int32)).to(dev)
    nsd = torch.from_numpy(np.asarray(ns, np.int32)).to(dev)
    Ad = torch.from_numpy(np.asarray(A, np.int32)).to(dev)
    offd = torch.from_numpy(np.asarray(off, np.int64)).to(dev)
    res = lib.pluq_batched(msd, nsd, Ad, offd, p)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), res.P.cpu().numpy(), res.Q.cpu().numpy(), res.rank.cpu().numpy(), \
        res.rrp.cpu().numpy(), res.crp.cpu().numpy()


def _compare(orc, ms, ns, A_in, off, p, out, idx):
    LU, P, Q, rank, rrp, crp = out
    po = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    qo = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    for i in idx:
        m, n = int(ms[i]), int(ns[i])
        Ai = A_in[off[i]:off[i] + m * n].reshape(m, n)
        want = orc.pluq(Ai, p, selfcheck=False)
        got = LU[off[i]:off[i] + m * n].reshape(m, n)
        assert rank[i] == want.rank, (i, m, n)
        assert np.array_equal(P[po[i]:po[i] + m], want.P), i
        assert np.array_equal(Q[qo[i]:qo[i] + n], want.Q), i
        assert np.array_equal(got, want.LU), i
        r = want.rank
        assert np.array_equal(rrp[po[i]:po[i] + r], want.rrp), i
        assert np.array_equal(crp[qo[i]:qo[i] + r], want.crp), i


@pytest.mark.parametrize("p", [2, 251, 65521, 8388593])
def test_batched_small_mixed(lib, orc, p):
    rng = np.random.default_rng(p)
    count = 90
    ms = rng.integers(1, 80, count)
    ns = rng.integers(1, 80, count)
    mats = []
    for i in range(count):
        r = int(rng.integers(0, min(ms[i], ns[i]) + 1))
        mats.append(wl.lowrank(int(ms[i]), int(ns[i]), r, p, int(rng.integers(1 << 40))) if i % 3
                    else rng.integers(0, p, (ms[i], ns[i])).astype(np.int32))
    off = np.concatenate([[0], np.cumsum(ms * ns)[:-1]]).astype(np.int64)
    A = np.concatenate([x.ravel() for x in mats]).astype(np.int32)
    note("batched small", p, count)
    out = _run(lib, ms, ns, A, off, p)
    _compare(orc, ms, ns, A, off, p, out, range(count))


def test_batched_edge_shapes(lib, orc):
    p = 131071
    shapes = [(1, 1), (1, 300), (300, 1), (0, 5), (5, 0), (2, 2), (17, 513), (513, 17), (100, 100)]
    mats = []
    for (m, n) in shapes:
        mats.append(np.zeros((m, n), np.int32) if m * n == 0 else wl.lowrank(m, n, min(m, n) // 2, p, m * 1000 + n))
    ms = np.array([s[0] for s in shapes])
    ns = np.array([s[1] for s in shapes])
    off = np.concatenate([[0], np.cumsum(ms * ns)[:-1]]).astype(np.int64)
    A = np.concatenate([x.ravel() for x in mats] + [np.zeros(1, np.int32)]).astype(np.int32)
    note("batched edge shapes")
    out = _run(lib, ms, ns, A, off, p)
    _compare(orc, ms, ns, A, off, p, out, range(len(shapes)))


@pytest.mark.parametrize("p", [65521, 131071])
def test_batched_maximum_dimensions(lib, orc, p):
    """Matrices at the largest dimension the batched call takes (1024 rows or
    columns: 32 mask words, both halves of the walk's lane reductions), on
    the 16-bit (p < 2^16) and the 32-bit working copies, with full, partial
    and unit rank and a thin block beside them."""
    FFP_BATCH_MAX_DIM = 1024
    shapes = [(FFP_BATCH_MAX_DIM, FFP_BATCH_MAX_DIM, 700), (FFP_BATCH_MAX_DIM, 1000, 1000),
              (999, FFP_BATCH_MAX_DIM, 1), (FFP_BATCH_MAX_DIM, 3, 3), (5, FFP_BATCH_MAX_DIM, 5)]
    mats = [wl.lowrank(m, n, r, p, 7 * m + n) for (m, n, r) in shapes]
    ms = np.array([s[0] for s in shapes])
    ns = np.array([s[1] for s in shapes])
    off = np.concatenate([[0], np.cumsum(ms * ns)[:-1]]).astype(np.int64)
    A = np.concatenate([x.ravel() for x in mats]).astype(np.int32)
    note("batched maximum dimensions", p)
    out = _run(lib, ms, ns, A, off, p)
    assert np.array_equal(out[3][:len(ms)], [s[2] for s in shapes])
    _compare(orc, ms, ns, A, off, p, out, range(len(shapes)))


def test_batched_workload_4096(lib, orc):
    """The 4096-matrix workload (m, n uniform in [16, 512], rank uniform in
    [1, min]): every rank equals the constructed one, a sample of matrices is
    compared with the oracle element by element, and every matrix passes the
    any-size property checks."""
    p = 65521
    ms, ns, rs, A, off = wl.make("batch4096_p65521")
    note("batched 4096")
    out = _run(lib, ms, ns, A, off, p)
    LU, P, Q, rank, rrp, crp = out
    assert np.array_equal(rank[:len(ms)], rs)
    sample = np.random.default_rng(0).choice(len(ms), 48, replace=False)
    _compare(orc, ms, ns, A, off, p, out, sample)
    po = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    qo = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    for i in range(0, len(ms), 16):
        m, n = int(ms[i]), int(ns[i])
        Ai = A[off[i]:off[i] + m * n].reshape(m, n)
        err = checks.full_check(Ai, LU[off[i]:off[i] + m * n].reshape(m, n), P[po[i]:po[i] + m],
                                Q[qo[i]:qo[i] + n], int(rank[i]), p, orc.order, exact_limit=0)
        assert err is None, (i, err)


def test_batched_graph_capture_replays(lib, orc):
    """The batched call captured in a HIP graph (two kernel launches, no host
    synchronisation, no allocation): three replays, each after eager work and
    a synchronisation, each equal to the eager result bit for bit; a sample
    of matrices also against the oracle."""
    import torch
    p = 65521
    ms, ns, rs, A, off = wl.batch(192, 16, 160, p, 77)
    dev = "cuda"
    msd = torch.from_numpy(ms.astype(np.int32)).to(dev)
    nsd = torch.from_numpy(ns.astype(np.int32)).to(dev)
    offd = torch.from_numpy(off.astype(np.int64)).to(dev)
    A0 = torch.from_numpy(A.astype(np.int32)).to(dev)
    note("batched graph: eager reference")
    Ae = A0.clone()
    ref = lib.pluq_batched(msd, nsd, Ae, offd, p)
    torch.cuda.synchronize()
    max_m, max_n = int(ms.max()), int(ns.max())
    tm, tn, batch = int(ms.sum()), int(ns.sum()), len(ms)
    po = torch.from_numpy(np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)).to(dev)
    qo = torch.from_numpy(np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)).to(dev)
    P = torch.empty(tm, dtype=torch.int32, device=dev)
    Q = torch.empty(tn, dtype=torch.int32, device=dev)
    rrp = torch.empty(tm, dtype=torch.int32, device=dev)
    crp = torch.empty(tn, dtype=torch.int32, device=dev)
    rank = torch.empty(batch, dtype=torch.int32, device=dev)
    ws = torch.empty(lib.load().ffp_pluq_batched_workspace(batch, max_m, max_n, p, 0), dtype=torch.uint8,
                     device=dev)
    Aw = A0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # one eager run on the capture stream's side before capturing
        lib.pluq_batched_into(msd, nsd, max_m, max_n, Aw, offd, P, po, Q, qo, rank, rrp, crp, ws, p)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    note("batched graph: capture")
    with torch.cuda.graph(g):
        Aw.copy_(A0)
        lib.pluq_batched_into(msd, nsd, max_m, max_n, Aw, offd, P, po, Q, qo, rank, rrp, crp, ws, p)
    for rep in range(3):
        # eager work between replays: clobber the outputs
        Aw.fill_(7)
        P.fill_(-1)
        Q.fill_(-1)
        rank.fill_(-1)
        torch.cuda.synchronize()
        note(f"batched graph: replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Aw, Ae), rep
        assert torch.equal(P, ref.P[:tm]) and torch.equal(Q, ref.Q[:tn]), rep
        assert torch.equal(rank, ref.rank[:batch]), rep
        for i in range(batch):
            r = int(rank[i])
            a, b = int(po[i]), int(qo[i])
            assert torch.equal(rrp[a:a + r], ref.rrp[a:a + r]) and torch.equal(crp[b:b + r], ref.crp[b:b + r])
    assert np.array_equal(rank.cpu().numpy(), rs)
    out = (Aw.cpu().numpy(), P.cpu().numpy(), Q.cpu().numpy(), rank.cpu().numpy(), rrp.cpu().numpy(),
           crp.cpu().numpy())
    _compare(orc, ms, ns, A, off, p, out, range(0, batch, 12))


def test_batched_autotune(lib, orc):
    """The autotuner times every launch shape on the batch, leaves the batch
    factored (equal to the plain batched call bit for bit), and later calls
    on the same batch description give the same bits again."""
    import torch
    p = 131071
    ms, ns, rs, A, off = wl.batch(300, 8, 300, p, 91)
    dev = "cuda"
    msd = torch.from_numpy(ms.astype(np.int32)).to(dev)
    nsd = torch.from_numpy(ns.astype(np.int32)).to(dev)
    offd = torch.from_numpy(off.astype(np.int64)).to(dev)
    A0 = torch.from_numpy(A.astype(np.int32)).to(dev)
    note("batched autotune: plain call")
    Ae = A0.clone()
    ref = lib.pluq_batched(msd, nsd, Ae, offd, p)
    note("batched autotune: tune")
    At = A0.clone()
    res, shape, times = lib.pluq_batched_tune(msd, nsd, At, offd, p)
    torch.cuda.synchronize()
    assert 0 <= shape < lib.BATCH_SHAPES and len(times) == lib.BATCH_SHAPES and all(t > 0 for t in times)
    assert times[shape] == min(times)
    assert torch.equal(At, Ae)
    assert torch.equal(res.P, ref.P) and torch.equal(res.Q, ref.Q) and torch.equal(res.rank, ref.rank)
    note("batched autotune: call with the tuned shape")
    A2 = A0.clone()
    res2 = lib.pluq_batched(msd, nsd, A2, offd, p)
    torch.cuda.synchronize()
    assert torch.equal(A2, Ae) and torch.equal(res2.rank, ref.rank)
    assert np.array_equal(res2.rank.cpu().numpy(), rs)
    out = (A2.cpu().numpy(), res2.P.cpu().numpy(), res2.Q.cpu().numpy(), res2.rank.cpu().numpy(),
           res2.rrp.cpu().numpy(), res2.crp.cpu().numpy())
    _compare(orc, ms, ns, A, off, p, out, range(0, len(ms), 25))


def test_batched_every_launch_shape(lib, orc):
    """Each launch shape, chosen explicitly, gives the oracle's bits on a
    mixed batch (shapes differ in workgroup size, so in the compaction
    rounds and the number of update waves)."""
    import torch
    p = 65521
    ms, ns, rs, A, off = wl.batch(120, 16, 400, p, 33)
    max_m, max_n = int(ms.max()), int(ns.max())
    for shape in range(lib.BATCH_SHAPES):
        note("batched shape", shape)
        lib.pluq_batched_set_shape(len(ms), max_m, max_n, shape)
        out = _run(lib, ms, ns, A, off, p)
        assert np.array_equal(out[3][:len(ms)], rs), shape
        _compare(orc, ms, ns, A, off, p, out, range(len(ms)))
    lib.pluq_batched_set_shape(len(ms), max_m, max_n, 0)
