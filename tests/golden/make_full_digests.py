"""Write tests/golden/full_size_digests.json: SHA-256 digests of the oracle's
PLUQ outputs (L\\U in place, P, Q, rank, row and column rank profiles) on the
full-size workloads, so that the GPU tests can compare their outputs with the
oracle's bit for bit without running the oracle for minutes each time.

Only the oracle (``oracle/``) computes anything here; the inputs come from the
seeded generators in ``workloads.py``.  Run on a CPU host (minutes per
workload; pass 2 of the oracle runs only where the quadrant pivot order
differs from the row-sorted one):

    python tests/golden/make_full_digests.py [workload ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402
from oracle import oracle  # noqa: E402

OUT = os.path.join(HERE, "full_size_digests.json")
DEFAULT = ["pluq8192_p131071", "pluq8192_r4096_p131071", "n16384_p8388593", "n16384_p251"]


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def digests(LU, P, Q, rank, rrp, crp) -> dict:
    """The digests a GPU result must reproduce (int32 little-endian, row-major)."""
    return {"LU": digest(LU), "P": digest(P), "Q": digest(Q), "rank": int(rank),
            "rrp": digest(rrp[:rank]), "crp": digest(crp[:rank])}


def main(names):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    src = hashlib.sha256(open(os.path.join(ROOT, "oracle", "ffp_oracle.c"), "rb").read()).hexdigest()
    for name in names:
        spec = wl.WORKLOADS[name]
        A = wl.make(name)
        t0 = time.time()
        f = oracle.pluq(A, spec["p"], selfcheck=False)
        dt = time.time() - t0
        rec = digests(f.LU, f.P, f.Q, f.rank, f.rrp, f.crp)
        rec.update({"m": spec["m"], "n": spec["n"], "p": spec["p"], "seed": spec["seed"],
                    "oracle_source_sha256": src, "oracle_seconds": round(dt, 1),
                    "oracle_threads": oracle.num_threads()})
        out[name] = rec
        print(name, rec, flush=True)
        with open(OUT + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or DEFAULT)
