"""Benchmark: rank-profile-revealing PLUQ over Z/pZ on one MI355X.

A step is one whole PLUQ of the workload matrix, i.e. one pass of the hot
path: leaf eliminations, ftrsm, fgemm (Schur updates), flaswp rotations and
the rank-profile extraction.  The default workload is the largest
single-GPU configuration, n16384_p8388593 (16384 x 16384, entries uniform
mod p = 8388593, whose centred residues take three signed 8-bit limbs), on
the library's AUTO path (INT8-limb products from 0.5e9 field operations,
FP64 below).  The pristine input stays resident in HBM; each step starts
with a device-to-device copy of it (PLUQ works in place).
value = (2 n^3 / 3) / step time, the paper's effective rate.

The roofline object is for the kernel family with the most time in the
step, from HIP events the library records around each of its launches on
the launching stream (per-family launches, time, algorithmic work and
bytes), during a second pass of the same K steps right after the timed
ones (the events stay out of the timed steps).  Every family's share is
listed; `traffic` (measured HBM bytes per launch) and `mfma_busy` (matrix
core busy fraction) come from the committed rocprofv3 counter summaries
when their kernel source hash still matches.

Also printed (outside the timed steps): the same PLUQ forced onto each
path with bit-exact agreement, the n^3 product on both paths, and every
other configuration: 512 x 512 mod 65521, 8192 x 8192 mod 131071 (uniform
and rank 4096), 16384 mod 251 (one limb), the batched workload; the
Strassen-Winograd products against the plain ones at 8192 and at the
workload size; the factorisation variants at 8192 (tile-iterative
right-looking, Crout and left-looking with their modelled reduction counts,
slab-recursive) against the tile recursion; echelon form and nullspace of
the rank-4096 input.  The CPU
baseline is the plain oracle, on all host threads on the leading block of
the workload matrix, and on one thread on the 512 x 512 matrix and on a
sample of the batched workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME] [--path auto|fp64|int8]
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
PEAK_HBM = 8.0e12        # HBM3E bandwidth, MI355X

# The paper's own figures (Section 3.2 Table 3, Section 4.1), all on one
# 32-core Intel Xeon E5-4620 at 2.2 GHz (Sandy Bridge, 16 MB L3), ATLAS
# 3.11.4 dgemm under FFLAS-FFPACK, residues stored in double.
PAPER = {
    "hardware": "32-core Intel Xeon E5-4620 2.2 GHz (Sandy Bridge), ATLAS 3.11.4, FFLAS-FFPACK, FP64-embedded residues",
    "table3_tile_recursive_1core_s": {"3000": 2.16, "5000": 7.98, "7000": 20.81},
    "table3_tile_recursive_1core_gops_derived": {"3000": 8.33, "5000": 10.44, "7000": 10.99},
    "tile_recursive_speedup_32cores_S16K": 13.6,
    "pfgemm_speedup_32cores": 27,
    "note": "the paper's multicore Gflops curves are figures absent from the text; only these numbers survive",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _summary(kernel: str, workload: str, what: str):
    """Key/value pairs of a committed rocprofv3 summary, or None when it is
    missing or its kernel source changed since it was taken."""
    import hashlib
    import re
    src = {"k_fgemm_f64": "fgemm_f64.hip", "k_fgemm_i8": "fgemm_i8.hip", "k_leaf_gen": "leaf64.hip",
           "k_trsm": "ftrsm.hip", "k_split": "fgemm_i8.hip", "k_pluq_batched": "batched.hip"}.get(kernel)
    prof = os.path.join(ROOT, "profiles", f"{kernel.replace('k_', '')}_{workload}_{what}.md")
    if src is None:
        return None
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1402_3501_amd", "csrc", src), "rb").read()).hexdigest()
    except OSError:
        return None
    m1 = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    if not m1 or m1.group(1) != sha:
        return None
    return {k: float(v) for k, v in re.findall(r"^([a-z0-9_]+): ([0-9.eE+-]+)\s*$", text, flags=re.M)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="auto", choices=["auto", "fp64", "int8"])
    ap.add_argument("--workload", default="n16384_p8388593")
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
    import workloads as wl

    ffp.load()
    dev = torch.device("cuda:0")
    spec = wl.WORKLOADS[args.workload]
    if spec["kind"] == "batch":
        return bench_batched(args, spec)
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
    L = ffp.int8_limbs(p)
    big_path = path if path != ffp.PATH_AUTO else ffp.auto_path(p, m // 2, n // 2, k // 2)

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
    primary = (A.clone(), P.clone(), Q.clone(), r)
    # the same K steps again with the library's per-launch events on (they
    # add stream work, so they stay out of the timed steps above)
    ffp.profile_reset()
    ffp.profile_enable(True)
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ffp.profile_enable(False)
    fams = ffp.profile_read_all()
    nominal = 2.0 * n ** 3 / 3.0 if m == n else 2.0 * m * n * k - (m + n) * k * k + 2.0 * k ** 3 / 3.0
    algorithmic = 2.0 * m * n * r - (m + n) * r * r + 2.0 * r ** 3 / 3.0
    value = nominal / (ms * 1e-3) / 1e9
    log(f"[bench] rank {r}  {ms:.2f} ms/step  {value:.1f} Gop/s")

    K = max(args.steps, 1)
    families = {}
    for name, (nl, kms, kops, kbytes) in sorted(fams.items(), key=lambda x: -x[1][1]):
        families[name] = {"launches_per_step": round(nl / K, 2), "ms_per_step": round(kms / K, 4),
                          "avg_launch_us": round(kms * 1e3 / nl, 3), "share_of_step": round(kms / K / ms, 4)}
        # algorithmic rate against the peak of the unit the family runs on
        # (INT8 products count their L^2 digit products)
        if kops > 0:
            peak = PEAK_INT8 if name == "k_fgemm_i8" else PEAK_FP64
            ops = kops * (L * L if name == "k_fgemm_i8" else 1)
            families[name]["frac_of_peak"] = round(ops / (kms * 1e-3) / peak, 6)
        elif kbytes > 0:
            families[name]["frac_of_hbm"] = round(kbytes / (kms * 1e-3) / PEAK_HBM, 4)
    dom = max(fams, key=lambda x: fams[x][1]) if fams else None
    roof = None
    if dom:
        nl, kms, kops, kbytes = fams[dom]
        if dom == "k_fgemm_i8":
            ach, peak, unit, bound = kops * L * L / (kms * 1e-3), PEAK_INT8, "TOP/s", "mfma"
        elif dom in ("k_fgemm_f64", "k_leaf_gen", "k_trsm"):
            ach, peak, unit, bound = kops / (kms * 1e-3), PEAK_FP64, "TFLOP/s", "mfma"
        else:
            ach, peak, unit, bound = kbytes / (kms * 1e-3), PEAK_HBM, "GB/s", "hbm"
        scale = 1e9 if unit == "GB/s" else 1e12
        roof = {"bound": bound, "achieved": ach / scale, "peak": peak / scale, "unit": unit,
                "frac": ach / peak, "traffic": None, "kernel": dom,
                "launches_per_step": nl / K, "avg_launch_us": kms * 1e3 / nl,
                "ops_per_launch": kops / nl * (L * L if dom == "k_fgemm_i8" else 1),
                "algorithmic_bytes_per_launch": kbytes / nl, "kernel_ms_per_step": kms / K,
                "share_of_step": kms / K / ms}
        tr = _summary(dom, args.workload, "traffic")
        if tr and "traffic_bytes_per_launch" in tr:
            roof["traffic"] = tr["traffic_bytes_per_launch"]
        mf = _summary(dom, args.workload, "mfma")
        if mf:
            roof["mfma_busy"] = mf.get("mfma_busy_frac")
            roof["mfma_ops_per_launch_counted"] = mf.get("mfma_ops_per_launch")
        roof["families"] = families

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gop/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8" if big_path == ffp.PATH_INT8 else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "p": p, "seed": spec["seed"],
                   "path": args.path, "large_product_path": "int8" if big_path == ffp.PATH_INT8 else "fp64",
                   "limbs": L if big_path == ffp.PATH_INT8 else None,
                   "rank": r, "algorithmic_gops": round(algorithmic / (ms * 1e-3) / 1e9, 3)},
        "roofline": roof,
    }

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r_ = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, r_

    def pluq_on(name, pth, reps=3, B0=None):
        spec2 = wl.WORKLOADS[name]
        mm2, nn2, p2 = spec2["m"], spec2["n"], spec2["p"]
        if B0 is None:
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
        t, rk = timed(run, reps)
        return t, rk, (B, P2, Q2)

    def fgemm_pair(nn, p2, seed, reps=3):
        X = torch.from_numpy(wl.uniform(nn, nn, p2, seed)).to(dev)
        Y = torch.from_numpy(wl.uniform(nn, nn, p2, seed + 1)).to(dev)
        res, zs = {}, {}
        for pth, pn in ((ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
            if pth == ffp.PATH_INT8 and ffp.int8_limbs(p2) == 0:
                continue
            Z = torch.zeros((nn, nn), dtype=torch.int32, device=dev)
            t, _ = timed(lambda: ffp.fgemm(X, Y, Z, p2, path=pth), reps)
            res[f"fgemm{nn}_{pn}_ms"] = round(t, 3)
            res[f"fgemm{nn}_{pn}_gops"] = round(2.0 * nn ** 3 / (t * 1e-3) / 1e9, 3)
            zs[pn] = Z
        if len(zs) == 2:
            res[f"fgemm{nn}_paths_bit_exact"] = bool(torch.equal(zs["int8"], zs["fp64"]))
        return res

    if not args.no_extra:
        extra = {}
        # the headline input forced onto each path: time and bit-exact agreement
        for pth, pn in ((ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
            if pth == ffp.PATH_INT8 and L == 0:
                continue
            log(f"[bench] {args.workload} on the {pn} path ...")
            t, rk, o = pluq_on(args.workload, pth, reps=3, B0=A0)
            extra[f"pluq_{pn}_ms"] = round(t, 3)
            extra[f"pluq_{pn}_gops"] = round(nominal / (t * 1e-3) / 1e9, 3)
            extra[f"pluq_{pn}_bit_exact_vs_primary"] = bool(
                rk == primary[3] and all(torch.equal(a, b) for a, b in zip(o, primary[:3])))
            del o
        torch.cuda.empty_cache()
        log("[bench] n^3 products ...")
        for kk, v in fgemm_pair(n, p, 202).items():
            extra[f"{args.workload}_{kk}"] = v
        # the other configurations
        others = [("pluq512_p65521", 20), ("pluq8192_p131071", 5), ("pluq8192_r4096_p131071", 3), ("n16384_p251", 2)]
        for name, reps in others:
            if name == args.workload:
                continue
            log(f"[bench] {name} ...")
            s2 = wl.WORKLOADS[name]
            nn2, p2 = s2["n"], s2["p"]
            B0 = torch.from_numpy(wl.make(name)).to(dev)
            outs = {}
            for pth, pn in ((ffp.PATH_AUTO, "auto"), (ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
                if pth == ffp.PATH_INT8 and ffp.int8_limbs(p2) == 0:
                    continue
                t, rk, o = pluq_on(name, pth, reps=reps, B0=B0)
                mm2 = s2["m"]
                extra[f"{name}_pluq_{pn}_ms"] = round(t, 3)
                extra[f"{name}_pluq_{pn}_gops"] = round(2.0 * nn2 ** 3 / 3 / (t * 1e-3) / 1e9, 3)
                if pn == "auto":
                    extra[f"{name}_rank"] = rk
                    extra[f"{name}_algorithmic_gops"] = round(
                        (2.0 * mm2 * nn2 * rk - (mm2 + nn2) * rk * rk + 2.0 * rk ** 3 / 3) / (t * 1e-3) / 1e9, 3)
                outs[pn] = (rk,) + tuple(x.clone() for x in o)
            ref = outs["auto"]
            extra[f"{name}_paths_bit_exact"] = all(
                v[0] == ref[0] and all(torch.equal(a, b) for a, b in zip(v[1:], ref[1:])) for v in outs.values())
            del outs, B0
            torch.cuda.empty_cache()
            if name in ("pluq8192_p131071", "n16384_p251"):
                for kk, v in fgemm_pair(nn2, p2, 302).items():
                    extra[f"{name}_{kk}"] = v
        # Strassen-Winograd over the n^3 product (automatic levels and one
        # level) against the plain product, both paths, bit-exact
        log("[bench] Strassen-Winograd products ...")
        for nn, p2 in ((8192, 131071), (n, p)):
            X = torch.from_numpy(wl.uniform(nn, nn, p2, 501)).to(dev)
            Y = torch.from_numpy(wl.uniform(nn, nn, p2, 502)).to(dev)
            for pth, pn in ((ffp.PATH_INT8, "int8"), (ffp.PATH_FP64, "fp64")):
                if pth == ffp.PATH_INT8 and ffp.int8_limbs(p2) == 0:
                    continue
                Z0 = torch.zeros((nn, nn), dtype=torch.int32, device=dev)
                t0_, _ = timed(lambda: ffp.fgemm(X, Y, Z0, p2, path=pth), 2)
                for lv, ln_ in ((ffp.WINO_AUTO, "auto"), (1, "1")):
                    Z = torch.zeros((nn, nn), dtype=torch.int32, device=dev)
                    t_, _ = timed(lambda: ffp.fgemm_wino(X, Y, Z, p2, path=pth, levels=lv), 2)
                    key = f"fgemm{nn}_p{p2}_{pn}"
                    extra[f"{key}_plain_ms"] = round(t0_, 3)
                    extra[f"{key}_wino{ln_}_ms"] = round(t_, 3)
                    extra[f"{key}_wino{ln_}_bit_exact"] = bool(torch.equal(Z, Z0))
                    del Z
                del Z0
            del X, Y
            torch.cuda.empty_cache()
        # the factorisation variants of Sections 3.1 and 4.1 on the 8192
        # uniform input: tile-iterative right-looking / Crout / left-looking
        # (tiles of 512 and 1024), slab-recursive, against the tile recursion
        log("[bench] factorisation variants at 8192 ...")
        B0 = torch.from_numpy(wl.make("pluq8192_p131071")).to(dev)
        ref_t, _, ref_o = pluq_on("pluq8192_p131071", ffp.PATH_AUTO, reps=3, B0=B0)
        extra["variants8192_tile_recursive_ms"] = round(ref_t, 3)
        Bv = torch.empty_like(B0)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        for vname, var in (("right", ffp.LU_RIGHT), ("crout", ffp.LU_CROUT), ("left", ffp.LU_LEFT)):
            for kt in (512, 1024):
                wsv = torch.empty(ffp.lu_tiled_workspace(var, 8192, 8192, kt, 131071), dtype=torch.uint8, device=dev)

                def run_v():
                    Bv.copy_(B0)
                    ffp.lu_tiled(Bv, 131071, var, kt, info=info, ws=wsv)
                t_, _ = timed(run_v, 3)
                extra[f"variants8192_{vname}_k{kt}_ms"] = round(t_, 3)
                extra[f"variants8192_{vname}_k{kt}_bit_exact"] = bool(torch.equal(Bv, ref_o[0])) and int(info) == 0
                extra[f"variants8192_{vname}_k{kt}_model_reductions"] = ffp.reduction_count(var, 8192, kt)
                del wsv
        extra["variants8192_tile_recursive_model_reductions"] = ffp.reduction_count(ffp.LU_TILE_RECURSIVE, 8192)
        extra["variants8192_slab_recursive_model_reductions"] = ffp.reduction_count(ffp.LU_SLAB_RECURSIVE, 8192)
        for name in ("pluq8192_p131071", "pluq8192_r4096_p131071"):
            S0 = torch.from_numpy(wl.make(name)).to(dev)
            Sv = torch.empty_like(S0)
            out_s = {}

            def run_s():
                Sv.copy_(S0)
                out_s["r"] = ffp.pluq_slab(Sv, 131071)
            t_, _ = timed(run_s, 2)
            extra[f"{name}_slab_recursive_ms"] = round(t_, 3)
            extra[f"{name}_slab_recursive_rank"] = out_s["r"].rank
            del S0, Sv
        del B0, Bv, ref_o
        torch.cuda.empty_cache()
        # echelon forms of the rank-4096 input from its factorisation
        log("[bench] echelon forms ...")
        E0 = torch.from_numpy(wl.make("pluq8192_r4096_p131071")).to(dev)
        res_e = ffp.pluq(E0, 131071)
        t_, _ = timed(lambda: ffp.echelon(res_e, 131071, form=0), 2)
        extra["pluq8192_r4096_row_echelon_ms"] = round(t_, 3)
        t_, _ = timed(lambda: ffp.nullspace(res_e, 131071, side=0), 2)
        extra["pluq8192_r4096_nullspace_ms"] = round(t_, 3)
        del E0, res_e
        torch.cuda.empty_cache()
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
        _, shape, shape_ms = ffp.pluq_batched_tune(ms_d, ns_d, Ab, off_d, bs["p"])
        res = None

        def run_b():
            nonlocal res
            Ab.copy_(Ab0)
            res = ffp.pluq_batched(ms_d, ns_d, Ab, off_d, bs["p"])
        tb, _ = timed(run_b, 3)
        mm, nn, rr = (x.astype(np.float64) for x in (ms_h, ns_h, rs_h))
        alg = float(np.sum(2 * mm * nn * rr - (mm + nn) * rr ** 2 + 2 * rr ** 3 / 3))
        extra["batched_workload"] = "batch4096_p65521"
        extra["batched_ms"] = round(tb, 3)
        extra["batched_tuned_shape"] = shape
        extra["batched_shape_ms"] = [round(x, 3) for x in shape_ms]
        extra["batched_matrices_per_s"] = round(len(ms_h) / (tb * 1e-3), 1)
        extra["batched_algorithmic_gops"] = round(alg / (tb * 1e-3) / 1e9, 3)
        extra["batched_ranks_ok"] = bool(np.array_equal(res.rank.cpu().numpy()[:len(ms_h)], rs_h))
        out["extra"] = extra
        out["paper_reference"] = PAPER

    if not args.no_cpu:
        from oracle import oracle as orc
        s = 6144 if min(m, n) >= 6144 else min(m, n)
        sub = np.ascontiguousarray(A_host[:s, :s])
        threads = orc.num_threads()
        log(f"[bench] CPU oracle on a {s}x{s} sample, {threads} threads ...")
        t0 = time.perf_counter()
        f = orc.pluq(sub, p, selfcheck=False)
        tc = time.perf_counter() - t0
        cpu = {"value": round(2.0 * s ** 3 / 3.0 / tc / 1e9, 4), "unit": "Gop/s", "cores": threads, "kind": "oracle",
               "sample": f"leading {s}x{s} block of the {args.workload} matrix, oracle PLUQ (rank {f.rank}), "
                         f"{tc:.2f} s on {threads} threads",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
        # one thread: the 512 x 512 configuration and a sample of the batch
        orc.set_threads(1)
        try:
            A1 = wl.make("pluq512_p65521")
            t0 = time.perf_counter()
            orc.pluq(A1, 65521, selfcheck=False)
            t1c = time.perf_counter() - t0
            cpu["one_thread_pluq512_p65521_s"] = round(t1c, 4)
            cpu["one_thread_pluq512_p65521_gops"] = round(2.0 * 512 ** 3 / 3 / t1c / 1e9, 4)
            ms_h, ns_h, rs_h, Ab_h, off_h = wl.batch(128, 16, 512, 65521, 5)
            t0 = time.perf_counter()
            for i in range(len(ms_h)):
                Ai = Ab_h[off_h[i]:off_h[i] + ms_h[i] * ns_h[i]].reshape(ms_h[i], ns_h[i])
                orc.pluq(Ai, 65521, selfcheck=False)
            tbc = time.perf_counter() - t0
            cpu["one_thread_batch_sample"] = "128 matrices drawn like batch4096_p65521"
            cpu["one_thread_batch_matrices_per_s"] = round(len(ms_h) / tbc, 2)
            cpu["one_thread_batch4096_s_projected"] = round(tbc * 4096 / len(ms_h), 2)
        finally:
            orc.set_threads(threads)
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_batched(args, spec):
    """The batched workload as the step: one persistent launch over all its
    matrices (device copy of the pristine batch + the factorisation), the
    launch shape chosen by the autotuner first.  value = sum over the
    matrices of the algorithmic work 2mnr - (m+n)r^2 + 2r^3/3, per second."""
    import numpy as np
    import torch
    import paper_1402_3501_amd as ffp
    import workloads as wl
    dev = torch.device("cuda:0")
    p = spec["p"]
    log(f"[bench] generating {args.workload} ...")
    ms_h, ns_h, rs_h, Ab_h, off_h = wl.make(args.workload)
    ms_d, ns_d, off_d = (torch.from_numpy(x).to(dev) for x in (ms_h, ns_h, off_h))
    Ab0 = torch.from_numpy(Ab_h).to(dev)
    Ab = Ab0.clone()
    _, shape, shape_ms = ffp.pluq_batched_tune(ms_d, ns_d, Ab, off_d, p)
    holder = {}

    def step():
        Ab.copy_(Ab0)
        holder["res"] = ffp.pluq_batched(ms_d, ns_d, Ab, off_d, p)
    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ranks_ok = bool(np.array_equal(holder["res"].rank.cpu().numpy()[:len(ms_h)], rs_h))
    mm, nn, rr = (x.astype(np.float64) for x in (ms_h, ns_h, rs_h))
    alg = float(np.sum(2 * mm * nn * rr - (mm + nn) * rr ** 2 + 2 * rr ** 3 / 3))
    # the same steps again with the library's launch events on: the batched
    # kernel's own time per launch
    ffp.profile_reset()
    ffp.profile_enable(True)
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ffp.profile_enable(False)
    fams = ffp.profile_read_all()
    roof = None
    if "k_pluq_batched" in fams:
        nl, kms = fams["k_pluq_batched"][0], fams["k_pluq_batched"][1]
        # every multiply-add of the elimination is one FP64 fma (2 flops), as
        # counted by 2mnr - (m+n)r^2 + 2r^3/3; the kernel is latency-bound,
        # so its bound is the FP64 vector rate of the VALUs
        ach = alg / (kms / nl * 1e-3)
        roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64, "traffic": None, "kernel": "k_pluq_batched",
                "launches_per_step": nl / max(args.steps, 1), "avg_launch_us": kms * 1e3 / nl,
                "ops_per_launch": alg, "algorithmic_bytes_per_launch": 8.0 * float(np.sum(mm * nn)),
                "share_of_step": kms / max(args.steps, 1) / ms}
        tr = _summary("k_pluq_batched", args.workload, "traffic")
        if tr and "traffic_bytes_per_launch" in tr:
            roof["traffic"] = tr["traffic_bytes_per_launch"]
    out = {"metric": "batched PLUQ mod p algorithmic Gop/s (sum of 2mnr - (m+n)r^2 + 2r^3/3)",
           "value": round(alg / (ms * 1e-3) / 1e9, 3), "unit": "Gop/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "matrices": int(len(ms_h)), "p": p, "seed": spec["seed"],
                      "tuned_shape": shape, "shape_ms": [round(x, 3) for x in shape_ms],
                      "matrices_per_s": round(len(ms_h) / (ms * 1e-3), 1), "ranks_ok": ranks_ok},
           "roofline": roof}
    if not args.no_cpu:
        from oracle import oracle as orc
        threads = orc.num_threads()
        ms_c, ns_c, rs_c, Ab_c, off_c = wl.batch(256, 16, 512, p, 5)
        log(f"[bench] CPU oracle on a 256-matrix sample, {threads} threads ...")
        t0 = time.perf_counter()
        for i in range(len(ms_c)):
            orc.pluq(Ab_c[off_c[i]:off_c[i] + ms_c[i] * ns_c[i]].reshape(ms_c[i], ns_c[i]), p, selfcheck=False)
        tc = time.perf_counter() - t0
        mc, nc, rc = (x.astype(np.float64) for x in (ms_c, ns_c, rs_c))
        alg_c = float(np.sum(2 * mc * nc * rc - (mc + nc) * rc ** 2 + 2 * rc ** 3 / 3))
        out["cpu_baseline"] = {"value": round(alg_c / tc / 1e9, 4), "unit": "Gop/s", "cores": threads, "kind": "oracle",
                               "sample": f"256 matrices drawn like {args.workload} (seed 5), oracle PLUQ one after "
                                         f"another, {tc:.2f} s on {threads} threads",
                               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
