"""Full-size parity against stored oracle outputs: SHA-256 digests of the
oracle's PLUQ (L\\U in place, P, Q, rank, row and column rank profiles) on
the full workloads, written by tests/golden/make_full_digests.py (which runs
only the oracle), compared with the digests of the GPU outputs on the same
seeded inputs.  Equal digests mean every output bit equals the oracle's."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "full_size_digests.json")


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def _names():
    if not os.path.exists(DIGESTS):
        return []
    return sorted(json.load(open(DIGESTS)))


@pytest.mark.parametrize("name", _names())
def test_full_size_outputs_equal_oracle(lib, name):
    import torch
    want = json.load(open(DIGESTS))[name]
    spec = wl.WORKLOADS[name]
    assert (want["m"], want["n"], want["p"], want["seed"]) == (spec["m"], spec["n"], spec["p"], spec["seed"])
    A = torch.from_numpy(wl.make(name)).cuda()
    note("golden", name)
    res = lib.pluq(A, spec["p"])
    torch.cuda.synchronize()
    r = res.rank
    assert r == want["rank"]
    got = {"LU": _digest(A.cpu().numpy()), "P": _digest(res.P.cpu().numpy()), "Q": _digest(res.Q.cpu().numpy()),
           "rrp": _digest(res.rrp.cpu().numpy()[:r]), "crp": _digest(res.crp.cpu().numpy()[:r])}
    for k, v in got.items():
        assert v == want[k], (name, k)


@pytest.mark.parametrize("name", [x for x in _names() if x.startswith("pluq8192")])
def test_full_size_fp64_path_equals_oracle(lib, name):
    """The same 8192 workloads with every product forced onto the FP64 MFMA
    path (the AUTO run takes INT8 limbs for the large products)."""
    from paper_1402_3501_amd import PATH_FP64
    import torch
    want = json.load(open(DIGESTS))[name]
    spec = wl.WORKLOADS[name]
    A = torch.from_numpy(wl.make(name)).cuda()
    note("golden fp64", name)
    res = lib.pluq(A, spec["p"], path=PATH_FP64)
    torch.cuda.synchronize()
    r = res.rank
    assert r == want["rank"]
    got = {"LU": _digest(A.cpu().numpy()), "P": _digest(res.P.cpu().numpy()), "Q": _digest(res.Q.cpu().numpy()),
           "rrp": _digest(res.rrp.cpu().numpy()[:r]), "crp": _digest(res.crp.cpu().numpy()[:r])}
    for k, v in got.items():
        assert v == want[k], (name, k)
