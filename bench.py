"""Benchmark: rank-profile-revealing PLUQ over Z/pZ on one MI355X.

A step is one whole PLUQ of the workload matrix (pluq8192_p131071 by default:
8192 x 8192, entries uniform mod p = 131071), i.e. one pass of the hot path:
leaf eliminations, ftrsm, fgemm (Schur updates), flaswp rotations and the
rank-profile extraction.  The pristine input stays resident in HBM; each step
starts with a device-to-device copy of it (PLUQ works in place), which costs
about 0.1% of the step.  value = (2 n^3 / 3) / step time, the paper's
effective rate.

Also printed (outside the timed steps): the same PLUQ on the other path,
the 8192^3 fgemm on both paths, and bit-exact agreement between paths; the
rank-deficient 8192 workload (rank 4096); PLUQ and the n^3 product at
n = 16384 mod 251 (one INT8 limb) and mod 8388593 (three limbs) on both
paths with bit-exact agreement; the batched workload.

The roofline object is for the dominant contraction kernel (the modular
matrix product family with the most time in the step), from HIP events that
the library records around each of its launches on the launching stream,
during a second pass of the same K steps right after the timed ones (the
events stay out of the timed steps); share_of_step says how much of the step it covers
(the single-workgroup leaf and the triangular solves are latency-bound and
take the rest).  The CPU baseline is the plain
oracle on a bounded sample (the leading 4096 x 4096 block of the same matrix).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--path auto|fp64|int8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PLUQ mod p effective Gop/s (2n³/3) + MFMA util; INT8-limb vs FP64, bit-exact"
PEAK_FP64 = 78.6e12      # dense FP64 matrix peak, MI355X
PEAK_INT8 = 5.0e15       # dense INT8 matrix peak, MI355X


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(family: str):
    """HBM bytes per launch of a product kernel family, from the committed
    rocprofv3 counter summary, or None when that summary is missing or was
    taken on a different source of the kernel."""
    import hashlib
    import re
    src = {"k_fgemm_f64": "fgemm_f64.hip", "k_fgemm_i8": "fgemm_i8.hip"}[family]
    prof = os.path.join(ROOT, "profiles", family.replace("k_", "") + "_pluq8192_p131071_traffic.md")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1402_3501_amd", "csrc", src), "rb").read()).hexdigest()
    except OSError:
        return None
    m1 = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    m2 = re.search(r"traffic_bytes_per_launch: ([0-9.]+)", text)
    if not m1 or not m2 or m1.group(1) != sha:
        return None
    return float(m2.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="auto", choices=["auto", "fp64", "int8"])
    ap.add_argument("--workload", default="pluq8192_p131071")
    ap.add_argument("--no-extra", action="store_true", help="skip the comparison runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the factorisation here is not sharded across GPUs "
              "(see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1402_3501_amd as ffp
    from paper_1402_3501_amd import workloads as wl

    ffp.load()
    dev = torch.device("cuda:0")
    spec = wl.WORKLOADS[args.workload]
    assert spec["kind"] in ("uniform", "lowrank"), "bench workloads are single matrices"
    m, n, p = spec["m"], spec["n"], spec["p"]
    path = {"auto": ffp.PATH_AUTO, "fp64": ffp.PATH_FP64, "int8": ffp.PATH_INT8}[args.path]
    log(f"[bench] generating {args.workload} ...")
    A_host = wl.make(args.workload)
    A0 = torch.from_numpy(A_host).to(dev)
    A = torch.empty_like(A0)
    P = torch.empty(m, dtype=torch.int32, device=dev)
    Q = torch.empty(n, dtype=torch.int32, device=dev)
    k = min(m, n)
    rrp = torch.empty(k, dtype=torch.int32, device=dev)
    crp = torch.empty(k, dtype=torch.int32, device=dev)
    rdev = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(ffp.pluq_workspace(m, n, p, path), dtype=torch.uint8, device=dev)
    eff_path = path
    if path == ffp.PATH_AUTO:
        lib = ffp.load()
        eff_path = lib.ffp_auto_path(p, m // 2, n // 2, k // 2)
    limbs = ffp.int8_limbs(p) if eff_path == ffp.PATH_INT8 else 0

    def step():
        A.copy_(A0)
        return ffp.pluq_into(A, p, P, Q, rdev, rrp, crp, ws, path=path)

    for i in range(args.warmup):
        log(f"[bench] warmup {i}")
        r = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # the same K steps again with the library's per-launch events on: the
    # event records add ~0.1 ms of stream work per step, so they stay out of
    # the timed steps above
    ffp.profile_reset()
    ffp.profile_enable(True)
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ffp.profile_enable(False)
    nominal = 2.0 * n ** 3 / 3.0 if m == n else 2.0 * m * n * k - (m + n) * k * k + 2.0 * k ** 3 / 3.0
    algorithmic = 2.0 * m * n * r - (m + n) * r * r + 2.0 * r ** 3 / 3.0
    value = nominal / (ms * 1e-3) / 1e9
    log(f"[bench] rank {r}  {ms:.2f} ms/step  {value:.1f} Gop/s")

    # dominant product kernel: the path whose launches took the most time
    prof = {pth: ffp.profile_read(pth) for pth in (ffp.PATH_FP64, ffp.PATH_INT8)}
    dom = max(prof, key=lambda k: prof[k][1])
    launches, kms, kops = prof[dom]
    roof = None
    if launches and kms > 0:
        if dom == ffp.PATH_INT8:
            L = ffp.int8_limbs(p)
            roof = {"bound": "mfma", "achieved": kops * L * L / (kms * 1e-3) / 1e12, "peak": PEAK_INT8 / 1e12,
                    "unit": "TOP/s"}
        else:
            roof = {"bound": "mfma", "achieved": kops / (kms * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12,
                    "unit": "TFLOP/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        family = "k_fgemm_i8" if dom == ffp.PATH_INT8 else "k_fgemm_f64"
        roof["traffic"] = measured_traffic(family)
        roof["kernel"] = family
        roof["algorithmic_bytes_per_launch"] = ffp.profile_read_bytes(dom) / launches
        roof["launches_per_step"] = launches / max(args.steps, 1)
        roof["avg_launch_us"] = kms * 1e3 / launches
        roof["field_ops_per_launch"] = kops / launches
        roof["kernel_ms_per_step"] = kms / max(args.steps, 1)
        roof["share_of_step"] = roof["kernel_ms_per_step"] / ms
        other = ffp.PATH_FP64 if dom == ffp.PATH_INT8 else ffp.PATH_INT8
        roof["other_path_kernel_ms_per_step"] = prof[other][1] / max(args.steps, 1)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gop/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8" if eff_path == ffp.PATH_INT8 else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "p": p, "seed": spec["seed"],
                   "path": "int8" if eff_path == ffp.PATH_INT8 else "fp64", "limbs": limbs or None,
                   "rank": r, "algorithmic_gops": round(algorithmic / (ms * 1e-3) / 1e9, 3)},
        "roofline": roof,
    }

    if not args.no_extra:
        extra = {}
        # the other path on the same input: time one run and compare outputs bit for bit
        ref = (A.clone(), P.clone(), Q.clone(), r)
        for other in (ffp.PATH_FP64, ffp.PATH_INT8):
            if other == eff_path or (other == ffp.PATH_INT8 and ffp.int8_limbs(p) == 0):
                continue
            ws2 = torch.empty(ffp.pluq_workspace(m, n, p, other), dtype=torch.uint8, device=dev)
            A.copy_(A0)
            ffp.pluq_into(A, p, P, Q, rdev, rrp, crp, ws2, path=other)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            A.copy_(A0)
            r2 = ffp.pluq_into(A, p, P, Q, rdev, rrp, crp, ws2, path=other)
            torch.cuda.synchronize()
            t2 = (time.perf_counter() - t0) * 1e3
            same = bool(r2 == ref[3] and torch.equal(A, ref[0]) and torch.equal(P, ref[1]) and torch.equal(Q, ref[2]))
            name = "int8" if other == ffp.PATH_INT8 else "fp64"
            extra[f"pluq_{name}_ms"] = round(t2, 3)
            extra[f"pluq_{name}_gops"] = round(nominal / (t2 * 1e-3) / 1e9, 3)
            extra[f"pluq_{name}_bit_exact_vs_primary"] = same
            del ws2
        # the n^3 modular product on both paths (same random operands)
        X = torch.from_numpy(wl.uniform(n, n, p, 102)).to(dev)
        Y = torch.from_numpy(wl.uniform(n, n, p, 103)).to(dev)
        results = {}
        for pth, name in ((ffp.PATH_FP64, "fp64"), (ffp.PATH_INT8, "int8")):
            if pth == ffp.PATH_INT8 and ffp.int8_limbs(p) == 0:
                continue
            Z = torch.zeros((n, n), dtype=torch.int32, device=dev)
            ffp.fgemm(X, Y, Z, p, path=pth)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                ffp.fgemm(X, Y, Z, p, path=pth)
            torch.cuda.synchronize()
            tg = (time.perf_counter() - t0) * 1e3 / reps
            extra[f"fgemm{n}_{name}_ms"] = round(tg, 3)
            extra[f"fgemm{n}_{name}_gops"] = round(2.0 * n ** 3 / (tg * 1e-3) / 1e9, 3)
            results[name] = Z
        if len(results) == 2:
            extra["fgemm_paths_bit_exact"] = bool(torch.equal(results["fp64"], results["int8"]))
        del X, Y, results
        # the other single-matrix workloads: rank-deficient 8192 (rank 4096,
        # rank-deficient pivot blocks), and n = 16384 with one limb (p = 251)
        # and three limbs (p = 8388593), each PLUQ and n^3 product on both
        # paths with bit-exact agreement
        def timed(fn, reps=1):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r_ = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / reps, r_

        def pluq_on(name, pth):
            spec2 = wl.WORKLOADS[name]
            mm2, nn2, p2 = spec2["m"], spec2["n"], spec2["p"]
            B0 = torch.from_numpy(wl.make(name)).to(dev)
            B = torch.empty_like(B0)
            P2 = torch.empty(mm2, dtype=torch.int32, device=dev)
            Q2 = torch.empty(nn2, dtype=torch.int32, device=dev)
            k2 = min(mm2, nn2)
            rp2 = torch.empty(k2, dtype=torch.int32, device=dev)
            cp2 = torch.empty(k2, dtype=torch.int32, device=dev)
            rd2 = torch.empty(1, dtype=torch.int64, device=dev)
            ws3 = torch.empty(ffp.pluq_workspace(mm2, nn2, p2, pth), dtype=torch.uint8, device=dev)

            def run():
                B.copy_(B0)
                return ffp.pluq_into(B, p2, P2, Q2, rd2, rp2, cp2, ws3, path=pth)
            t, rk = timed(run)
            return t, rk, (B.clone(), P2.clone(), Q2.clone())

        log("[bench] rank-deficient 8192 ...")
        t, rk, _ = pluq_on("pluq8192_r4096_p131071", ffp.PATH_AUTO)
        extra["pluq8192_r4096_ms"] = round(t, 3)
        extra["pluq8192_r4096_rank"] = rk
        extra["pluq8192_r4096_algorithmic_gops"] = round(
            (2.0 * 8192 * 8192 * rk - 2 * 8192 * rk * rk + 2.0 * rk ** 3 / 3) / (t * 1e-3) / 1e9, 3)
        for name in ("n16384_p251", "n16384_p8388593"):
            log(f"[bench] {name} ...")
            p2 = wl.WORKLOADS[name]["p"]
            n2 = wl.WORKLOADS[name]["n"]
            outs = {}
            for pth, pn in ((ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
                t, rk, o = pluq_on(name, pth)
                extra[f"{name}_pluq_{pn}_ms"] = round(t, 3)
                extra[f"{name}_pluq_{pn}_gops"] = round(2.0 * n2 ** 3 / 3 / (t * 1e-3) / 1e9, 3)
                outs[pn] = o
            extra[f"{name}_pluq_paths_bit_exact"] = all(torch.equal(a, b) for a, b in zip(outs["int8"], outs["fp64"]))
            del outs
            X = torch.from_numpy(wl.uniform(n2, n2, p2, 202)).to(dev)
            Y = torch.from_numpy(wl.uniform(n2, n2, p2, 203)).to(dev)
            zs = {}
            for pth, pn in ((ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
                Z = torch.zeros((n2, n2), dtype=torch.int32, device=dev)
                t, _ = timed(lambda: ffp.fgemm(X, Y, Z, p2, path=pth), reps=2)
                extra[f"{name}_fgemm_{pn}_ms"] = round(t, 3)
                extra[f"{name}_fgemm_{pn}_gops"] = round(2.0 * n2 ** 3 / (t * 1e-3) / 1e9, 3)
                zs[pn] = Z
            extra[f"{name}_fgemm_paths_bit_exact"] = bool(torch.equal(zs["int8"], zs["fp64"]))
            del X, Y, zs
        # the batched persistent PLUQ on its own workload (4096 matrices,
        # m, n uniform in [16, 512], ranks uniform in [1, min]); ranks checked
        log("[bench] batched workload ...")
        bs = wl.WORKLOADS["batch4096_p65521"]
        ms_h, ns_h, rs_h, Ab_h, off_h = wl.make("batch4096_p65521")
        ms_d = torch.from_numpy(ms_h).to(dev)
        ns_d = torch.from_numpy(ns_h).to(dev)
        off_d = torch.from_numpy(off_h).to(dev)
        Ab0 = torch.from_numpy(Ab_h).to(dev)
        Ab = Ab0.clone()
        # autotune the launch shape on this batch once (untimed), then time
        # the plain call, which uses the chosen shape
        _, shape, shape_ms = ffp.pluq_batched_tune(ms_d, ns_d, Ab, off_d, bs["p"])
        Ab.copy_(Ab0)
        res = ffp.pluq_batched(ms_d, ns_d, Ab, off_d, bs["p"])
        torch.cuda.synchronize()
        Ab.copy_(Ab0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ffp.pluq_batched(ms_d, ns_d, Ab, off_d, bs["p"])
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        mm, nn, rr = (x.astype(np.float64) for x in (ms_h, ns_h, rs_h))
        alg = float(np.sum(2 * mm * nn * rr - (mm + nn) * rr ** 2 + 2 * rr ** 3 / 3))
        extra["batched_workload"] = "batch4096_p65521"
        extra["batched_ms"] = round(tb * 1e3, 3)
        extra["batched_tuned_shape"] = shape
        extra["batched_shape_ms"] = [round(x, 3) for x in shape_ms]
        extra["batched_matrices_per_s"] = round(len(ms_h) / tb, 1)
        extra["batched_algorithmic_gops"] = round(alg / tb / 1e9, 3)
        extra["batched_ranks_ok"] = bool(np.array_equal(res.rank.cpu().numpy()[:len(ms_h)], rs_h))
        out["extra"] = extra

    if not args.no_cpu:
        from oracle import oracle as orc
        s = 4096 if min(m, n) >= 4096 else min(m, n)
        sub = np.ascontiguousarray(A_host[:s, :s])
        log(f"[bench] CPU oracle on a {s}x{s} sample ...")
        t0 = time.perf_counter()
        f = orc.pluq(sub, p, selfcheck=False)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(2.0 * s ** 3 / 3.0 / tc / 1e9, 4), "unit": "Gop/s",
                               "cores": orc.num_threads(), "kind": "oracle",
                               "sample": f"leading {s}x{s} block of the workload matrix, oracle PLUQ "
                                         f"(rank {f.rank}), {tc:.2f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
