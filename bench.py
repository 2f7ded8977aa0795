"""Throughput of the shearing-box Poisson solve on one MI355X.

Default workload: one 256^3 box (Lx = Ly = 4, Lz = 6, H = 1, z padded to 512, VGF-HybridBC),
density = Gaussian stratification x (1 + 0.1 delta), delta a unit Gaussian random field with
P(k) ~ k^-2; q = 1.5, Omega = 1, t = 0.3, G = 1.  A step is one full solve (remap, padded
3-D transform, Green multiply, inverse, extraction) with rho and phi resident in HBM.

Prints progress on stderr and ONE JSON line on stdout.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Poisson solves/s + HBM GB/s at 256^3 (FP32 vs FP64) at stated rel-L2 error"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_plan(plan, rho, phi, shear, steps: int, warmup: int, profile: bool):
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.solve(rho, phi, shear, stream=stream)
    torch.cuda.synchronize()
    if profile:
        plan.profile_read()  # drop warm-up records
        plan.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        plan.solve(rho, phi, shear, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kernels = {}
    if profile:
        plan.profile_enable(False)
        kernels = plan.profile_read()
    return ms, kernels


# (name, precision, plain path, graph replay, remap, per-kernel events)
# Direct launches are the headline mode: on this stack a graph replay costs about 8 us more GPU
# time per solve than the same kernels launched directly.  The *_direct legs repeat the direct
# launches with a HIP event around every kernel, for the per-kernel split (not clean timings).
LEGS = (("fp32", "fp32", False, False, "spectral", False), ("fp32_graph", "fp32", False, True, "spectral", False),
        ("fp64", "fp64", False, False, "spectral", False), ("fp64_graph", "fp64", False, True, "spectral", False),
        ("plain_fp64", "fp64", True, False, "spectral", False),
        ("fp32_direct", "fp32", False, False, "spectral", True), ("fp64_direct", "fp64", False, False, "spectral", True),
        ("fp32_linear", "fp32", False, False, "linear", False))


# Summaries of rocprofv3 runs of this benchmark's FP32 leg (see each file for its command), keyed
# by pass; each is valid only while the kernel sources hash to its sources_sha256.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_passes_grf256_fp32_traffic.json")
TRACE_FILE = os.path.join(ROOT, "profiles", "fused_passes_grf256_fp32_trace.json")
COUNTER_FILE = os.path.join(ROOT, "profiles", "fused_passes_grf256_fp32_sq.json")
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s: 1024 SIMDs, 4 cycles each, 2.4 GHz


def kernel_source_digest(files) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile(path: str, kernel: str):
    """The record of `kernel` in a committed profile summary, or None when there is none or the
    kernel sources have changed since it was taken."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or kernel_source_digest(rec["sources"]) != rec["sources_sha256"]:
        return None
    return k


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel`: the L2-to-memory requests rocprofv3 counted, each weighed
    by its own size (TCC_EA0_RDREQ_32B/64B/128B, TCC_EA0_WRREQ/WRREQ_64B); None if not current."""
    k = _profile(TRAFFIC_FILE, kernel)
    return None if k is None else int(k["read_bytes"] + k["write_bytes"])


def copy_calibration(mib: int, steps: int) -> int:
    """A plain device-to-device copy of known size, for scaling hardware byte counters."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nbytes = 2 * n * 4
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "ms": round(ms, 5),
                      "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)
    return 0


def host_cpu() -> dict:
    """CPU model and core counts of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable, "threads_used": 1}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-samples", type=int, default=2, help="minimum oracle solves")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle sample length")
    ap.add_argument("--only", choices=[leg[0] for leg in LEGS],
                    help="time one leg and print its kernel split (for profiler runs)")
    ap.add_argument("--schedule", choices=["auto", "fused", "five_pass"], default="auto",
                    help="pass schedule of the non-plain legs (auto: the library's choice per precision)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="time a plain device copy of this many MiB instead (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is described in the design notes, not implemented)", file=sys.stderr)
        return 2

    if args.copy_mib:
        return copy_calibration(args.copy_mib, args.steps)

    import numpy as np
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear
    from paper_2510_10070_amd.inputs import workload

    w = workload("grf-256")
    nx, ny, nz, lx, ly, lz = w["box"]
    q, om, t, G = w["shear"]
    shear = Shear(q, om, t, G)
    log("generating the 256^3 random-field density")
    rho64 = w["make"]()
    N = nx * ny * nz

    res = {}
    phis = {}
    legs = [leg for leg in LEGS if args.only in (None, leg[0])]
    for leg, prec, plain, graph, remap, split in legs:
        dt = torch.float32 if prec == "fp32" else torch.float64
        rho = torch.tensor(rho64, dtype=dt, device="cuda:0")
        phi = torch.empty_like(rho)
        plan = Plan(Box(nx, ny, nz, lx, ly, lz, remap=remap), precision=prec, plain=plain, graph=graph,
                    autotune=not plain, schedule="auto" if plain else args.schedule)
        steps = args.steps if not plain else max(10, args.steps // 4)
        log(f"timing {leg}: {args.warmup} warm-up + {steps} steps")
        ms, kern = time_plan(plan, rho, phi, shear, steps, args.warmup, profile=split)
        w_bytes = 4 if prec == "fp32" else 8
        b_alg = 6 * N * w_bytes  # rho in, 3 round trips of the half spectrum (N w bytes each), phi out
        res[leg] = dict(ms=ms, solves_per_s=1e3 / ms, gbs_alg=b_alg / (ms * 1e-3) / 1e9, kernels=kern,
                        describe=plan.describe(), steps=steps, w=w_bytes)
        phis[leg] = (phi.double().cpu().numpy(), rho.double().cpu().numpy())
        log(f"{leg}: {ms * 1e3:.1f} us/solve, {1e3 / ms:.0f} solves/s, {res[leg]['gbs_alg']:.0f} GB/s (algorithmic)")
        plan.close()
        del rho, phi
        torch.cuda.empty_cache()

    # the batched workload: 64 boxes of uneven size and shear in one FP32 plan (grouped launches,
    # autotuned five-pass tiles where the fused schedule does not apply, graph-replayed)
    batch = None
    if args.only in (None, "fp32"):
        from paper_2510_10070_amd.inputs import batch_workload

        ws = batch_workload()
        brho = [torch.tensor(wb["make"](), dtype=torch.float32, device="cuda:0") for wb in ws]
        bphi = [torch.empty_like(r) for r in brho]
        bsh = [Shear(*wb["shear"]) for wb in ws]
        cells = sum(wb["box"][0] * wb["box"][1] * wb["box"][2] for wb in ws)
        batch = {"boxes": len(ws), "cells": cells}
        for mode, graph in (("direct", False), ("graph", True)):
            bplan = Plan([Box(*wb["box"]) for wb in ws], precision="fp32", graph=graph, autotune=True)
            for _ in range(5):
                bplan.solve(brho, bphi, bsh)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                bplan.solve(brho, bphi, bsh)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 20
            d = bplan.describe()
            batch[mode] = {"us_per_batch": round(ms * 1e3, 1), "boxes_per_s": round(len(ws) / (ms * 1e-3), 1),
                           "gbs_alg": round(6 * cells * 4 / (ms * 1e-3) / 1e9, 1), "launches": d.get("launches")}
            log(f"batch of {len(ws)} boxes fp32 ({mode}): {ms * 1e3:.1f} us per batch, "
                f"{batch[mode]['gbs_alg']:.0f} GB/s (algorithmic)")
            bplan.close()
        del brho, bphi
        torch.cuda.empty_cache()

    # acceleration -grad Phi from the FP32 potential (a streaming stencil: Phi in, three fields out)
    grav = None
    if args.only in (None, "fp32"):
        plan = Plan(Box(nx, ny, nz, lx, ly, lz), precision="fp32")
        rho = torch.tensor(rho64, dtype=torch.float32, device="cuda:0")
        phi = torch.empty_like(rho)
        g = [torch.empty_like(rho) for _ in range(3)]
        plan.solve(rho, phi, shear)
        for _ in range(5):
            plan.gravity(phi, *g, shear)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            plan.gravity(phi, *g, shear)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        gb = 4 * N * 4  # Phi read once, gx, gy, gz written
        grav = {"us": round(ms * 1e3, 2), "gbs_alg": round(gb / (ms * 1e-3) / 1e9, 1), "bytes_alg": gb}
        log(f"gravity fp32: {ms * 1e3:.1f} us, {grav['gbs_alg']:.0f} GB/s (algorithmic)")
        plan.close()
        del rho, phi, g
        torch.cuda.empty_cache()

    if args.only:
        r = res[args.only]
        print(json.dumps({"leg": args.only, "ms_per_step": round(r["ms"], 5), "solves_per_s": round(r["solves_per_s"], 1),
                          "kernels_us": {kk: round(v[1] / v[0] * 1e3, 2) for kk, v in r["kernels"].items()},
                          "schedule": r["describe"]}), flush=True)
        return 0

    # accuracy against the FP64 CPU oracle, and the oracle's own throughput on this host
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle

        ob = oracle.Box(nx, ny, nz, lx, ly, lz)
        osh = oracle.Shear(q, om, t, G)
        times = []
        ref64 = None
        # a bounded sample: whole solves until about cpu_seconds of work (at least cpu_samples)
        while len(times) < max(1, args.cpu_samples) or sum(times) < args.cpu_seconds:
            log(f"oracle solve {len(times) + 1} (FP64 input)")
            t0 = time.perf_counter()
            ref64 = oracle.solve(phis["fp64"][1], ob, osh)
            times.append(time.perf_counter() - t0)
        log("oracle solve on the FP32-rounded input")
        t0 = time.perf_counter()
        ref32 = oracle.solve(phis["fp32"][1], ob, osh)
        times.append(time.perf_counter() - t0)
        log("oracle solve with the linear remap (FP32-rounded input)")
        ref32l = oracle.solve(phis["fp32_linear"][1], oracle.Box(nx, ny, nz, lx, ly, lz, remap="linear"), osh)
        for leg, ref in (("fp32", ref32), ("fp64", ref64), ("plain_fp64", ref64), ("fp32_linear", ref32l)):
            errs[leg] = float(np.linalg.norm(phis[leg][0] - ref) / np.linalg.norm(ref))
        med = float(np.median(times))
        cpu = {"value": round(1.0 / med, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(times)} full 256^3 FP64 oracle solves of the same input (numpy, one thread), "
                         f"{sum(times):.1f} s in total, median {med:.2f} s per solve",
               "host": host_cpu()}

    # roofline of the dominant kernel of the headline (FP32) leg: HBM, with the kernel's duration
    # from HIP events around each launch in this run (avg_us) and, beside it, the mean duration the
    # committed kernel trace of the same leg records (no event between launches)
    k = res["fp32_direct"]["kernels"]
    name, (launches, tot) = max(k.items(), key=lambda kv: kv[1][1])
    avg_ms = tot / launches
    per_launch_bytes = 2 * N * 4  # each pass reads and writes N*w bytes (rho/phi or the half spectrum)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name), "kernel": name,
            "avg_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": per_launch_bytes}
    tr = _profile(TRACE_FILE, name)
    if tr is not None:
        roof["avg_us_trace"] = round(tr["mean_ns"] * 1e-3, 2)
        roof["frac_trace"] = round(per_launch_bytes / (tr["mean_ns"] * 1e-9) / 1e9 / HBM_PEAK_GBS, 4)
    sq = _profile(COUNTER_FILE, name)
    if sq is not None:
        # the same kernel against the VALU issue limit, which bounds it: committed instruction count
        # over this run's duration, against 1024 SIMDs x one wave64 instruction per 4 cycles at 2.4 GHz
        roof["valu"] = {"insts_per_launch": sq["SQ_INSTS_VALU"],
                        "issue_frac": round(sq["SQ_INSTS_VALU"] / (avg_ms * 1e-3) / VALU_ISSUE_PEAK, 4)}

    # the three byte counts of one FP32 solve: algorithmic (3 HBM round trips of the half spectrum),
    # the schedule's model, and what the counters recorded for the three passes
    fp32_b_alg = 6 * N * 4
    sched = res["fp32"]["describe"].get("bytes_model")
    counted = [measured_traffic(kk) for kk in ("fused_a", "fused_b", "fused_c")]
    counted = sum(counted) if all(c is not None for c in counted) else None
    t_s = res["fp32"]["ms"] * 1e-3
    bytes_per_solve = {"algorithmic": fp32_b_alg, "schedule_model": sched, "counters": counted,
                       "gbs_algorithmic": round(fp32_b_alg / t_s / 1e9, 1),
                       "gbs_schedule_model": round(sched / t_s / 1e9, 1) if sched else None,
                       "gbs_counters": round(counted / t_s / 1e9, 1) if counted else None,
                       "counters_note": "L2-to-memory requests of the three passes weighed by their size, from the "
                                        "committed summary; they include hits in the 256 MB MALL, which the counters "
                                        "available on gfx950 do not separate from HBM"}

    head = res["fp32"]
    out = {
        "metric": METRIC,
        "value": round(head["solves_per_s"], 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian random field x stratification)",
        "config": {"workload": "grf-256: one 256x256x256 box, Lx=Ly=4, Lz=6, H=1, z padded to 512, VGF-HybridBC, "
                               "q=1.5, Omega=1, t=0.3, G=1, FP32 bulk with FP64-derived Green coefficients, "
                               "twiddles and k=0 pencil, direct launches (per-solve shear staged in each call)",
                   "box": [nx, ny, nz], "padded_nz": 2 * nz, "precision": "fp32", "launch": "direct",
                   "boxes_per_step": 1},
        "gbs_alg": round(head["gbs_alg"], 1),
        "hbm_frac_alg": round(head["gbs_alg"] / HBM_PEAK_GBS, 4),
        "rel_l2_vs_oracle": {k2: v for k2, v in errs.items()},
        "fp64": {"solves_per_s": round(res["fp64"]["solves_per_s"], 1), "ms_per_step": round(res["fp64"]["ms"], 5),
                 "gbs_alg": round(res["fp64"]["gbs_alg"], 1)},
        "fp32_graph": {"solves_per_s": round(res["fp32_graph"]["solves_per_s"], 1),
                       "ms_per_step": round(res["fp32_graph"]["ms"], 5)},
        "fp64_graph": {"solves_per_s": round(res["fp64_graph"]["solves_per_s"], 1),
                       "ms_per_step": round(res["fp64_graph"]["ms"], 5)},
        "plain_fp64": {"solves_per_s": round(res["plain_fp64"]["solves_per_s"], 1),
                       "ms_per_step": round(res["plain_fp64"]["ms"], 5)},
        "speedup_vs_plain_fp64": {"fp32": round(head["solves_per_s"] / res["plain_fp64"]["solves_per_s"], 2),
                                  "fp64": round(res["fp64"]["solves_per_s"] / res["plain_fp64"]["solves_per_s"], 2)},
        "fp32_linear_remap": {"solves_per_s": round(res["fp32_linear"]["solves_per_s"], 1),
                              "ms_per_step": round(res["fp32_linear"]["ms"], 5)},
        "gravity_fp32": grav,
        "batch64_fp32": batch,
        "fp32_direct": {"solves_per_s": round(res["fp32_direct"]["solves_per_s"], 1),
                        "ms_per_step": round(res["fp32_direct"]["ms"], 5)},
        "fp64_direct": {"solves_per_s": round(res["fp64_direct"]["solves_per_s"], 1),
                        "ms_per_step": round(res["fp64_direct"]["ms"], 5)},
        "kernels_us": {leg: {kk: round(v[1] / v[0] * 1e3, 2) for kk, v in res[leg]["kernels"].items()}
                       for leg in res if res[leg]["kernels"]},
        "schedule": head["describe"],
        "roofline": roof,
        "bytes_per_solve": bytes_per_solve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
