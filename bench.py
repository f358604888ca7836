#!/usr/bin/env python3
"""Throughput of one full FMM evaluation on one MI355X.

Default workload (the configuration the headline metric is quoted on): the
1,048,576-particle jittered Lamb-Oseen lattice, sigma = 0.002, depth 8,
p = 17, every stage in FP64.  A "step" is one complete evaluation -- tree
build (z-order keys, counting sort, leaf ranges), P2M, M2M, M2L, L2L, L2P and
P2P -- with inputs already resident in HBM.

Prints ONE JSON line.  ``value`` is particles per second over the timed
steps (wall clock, bracketed by device synchronisation).  ``roofline``
describes the stage with the largest GPU time, measured with HIP events
recorded on the evaluation's own stream during the timed steps.
``cpu_baseline`` times the FP64 CPU oracle on the host cores for one full
evaluation of the same workload (rank 0, N = 1 only) and, from the same run,
reports the parity of the GPU result and its accuracy against the direct sums.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "particles/s per full FMM eval at ≤1e-6 rel. L2 vs direct; FP64 vs mixed"

# MI355X published peaks used for the roofline.  Packed FP32 instructions are
# disabled in this build, so FP32 vector arithmetic issues at the FP64 rate:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s.
PEAK_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit:
#  P2P: 14 flops per near pair (2 differences, 3 for |d|^2, 1 scaling, 1 exp,
#       1 for 1 - e, 1 product, 1 division, 4 for the complex accumulation).
#  M2L: 8 p^2 flops per interaction-list pair (dense complex p x p product).
P2P_FLOPS_PER_PAIR = 14


def m2l_pairs(L: int) -> int:
    """Interaction-list pairs over levels 2..L of a full uniform quadtree."""
    return sum(3 * ((1 << l) - 2) * (9 * (1 << l) - 10) for l in range(2, L + 1))


def near_pairs(leaf_start: np.ndarray, L: int) -> int:
    """Sum over leaves of n_t * (particles in the 3x3 neighbourhood), minus self pairs."""
    side = 1 << L
    cnt_z = np.diff(leaf_start.astype(np.int64))
    m = np.arange(side * side, dtype=np.uint64)
    a = np.zeros_like(m)
    b = np.zeros_like(m)
    for bit in range(16):
        a |= ((m >> np.uint64(2 * bit)) & np.uint64(1)) << np.uint64(bit)
        b |= ((m >> np.uint64(2 * bit + 1)) & np.uint64(1)) << np.uint64(bit)
    grid = np.zeros((side, side), np.int64)
    grid[b.astype(np.int64), a.astype(np.int64)] = cnt_z
    pad = np.pad(grid, 1)
    nb = sum(pad[1 + dy:1 + dy + side, 1 + dx:1 + dx + side] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return int(np.sum(grid * nb) - np.sum(grid))


def make_workload(name: str):
    wl = workloads.make(name)
    if wl.offsets is not None:
        raise SystemExit(f"workload {name} is batched; this bench runs single evaluations")
    return wl


def describe(wl) -> str:
    prec = "FP64" if wl.precision == "fp64" else f"mixed (FP32 P2P, FP32 M2L on the finest {wl.fp32_fine_levels} levels)"
    kind = {"C1": "uniform unit square", "C2": "jittered Lamb-Oseen lattice",
            "C3": "16-component Gaussian mixture", "C5": "uniform unit square"}[wl.name]
    return f"{wl.name}: {wl.n:,} particles, {kind}, sigma={wl.sigma}, depth {wl.depth}, p={wl.p}, {prec}"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C2", help="workload: C1, C2 (default), C3 or C5")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--accuracy-targets", type=int, default=1024)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import torch
    import paper_0905_2637_amd as fm

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        return 1
    dev = torch.device("cuda:0")
    wl = make_workload(args.config)
    n = wl.n
    x = torch.as_tensor(wl.x, device=dev)
    y = torch.as_tensor(wl.y, device=dev)
    g = torch.as_tensor(wl.gamma, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty(n, dtype=torch.float64, device=dev)
    plan = fm.Plan(n, wl.sigma, wl.p, wl.depth, domain=(wl.x0, wl.y0, wl.width),
                   precision=wl.precision, fp32_fine_levels=wl.fp32_fine_levels)

    for _ in range(args.warmup):
        plan.evaluate(x, y, g, u, v)
    torch.cuda.synchronize()
    if plan.out_of_domain():
        raise SystemExit("particles outside the domain")

    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.evaluate(x, y, g, u, v)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = plan.stats()
    plan.set_timing(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed

    # ---- roofline of the dominant stage ------------------------------------
    leaf_start = plan.dump(fm.DUMP_LEAF_START)
    stage_ms = {k: vv for k, vv in stages.items() if k != "evaluations"}
    dominant = max(stage_ms, key=stage_ms.get)
    pairs_near = near_pairs(leaf_start, wl.depth)
    pairs_m2l = m2l_pairs(wl.depth)
    if dominant == "p2p_l2p":
        work = pairs_near * P2P_FLOPS_PER_PAIR
        kernel = "k_p2p_l2p"
        unit_note = f"{pairs_near} near pairs x {P2P_FLOPS_PER_PAIR} flops"
    elif dominant == "m2l":
        work = pairs_m2l * 8 * wl.p * wl.p
        kernel = "k_m2l"
        unit_note = f"{pairs_m2l} M2L pairs x 8p^2 flops"
    else:
        work = None
        kernel = dominant
        unit_note = "tree/HBM-bound stage"
    t_dom = stage_ms[dominant] * 1e-3
    if work is not None:
        achieved = work / t_dom / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_VALU_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_VALU_TFLOPS, 4), "traffic": None,
                    "kernel": kernel, "stage_ms": round(stage_ms[dominant], 4), "work": unit_note}
    else:
        roofline = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                    "traffic": None, "kernel": kernel, "stage_ms": round(stage_ms[dominant], 4)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "n": n, "depth": wl.depth, "p": wl.p, "sigma": wl.sigma,
                   "precision": wl.precision, "parallelism": "single GPU"},
        "stages_ms": {k: round(vv, 4) for k, vv in stage_ms.items()},
        "work": {"near_pairs": pairs_near, "m2l_pairs": pairs_m2l},
        "roofline": roofline,
    }

    # ---- CPU oracle beside it ---------------------------------------------
    if not args.no_cpu_baseline:
        import oracle
        u_gpu = u.cpu().numpy()
        v_gpu = v.cpu().numpy()
        t1 = time.perf_counter()
        uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, wl.x0, wl.y0, wl.width)
        t_cpu = time.perf_counter() - t1
        tgt = workloads.sample_targets(n, args.accuracy_targets, 1000 + int(wl.name[1]))
        us, vs = oracle.direct_split(wl.x, wl.y, wl.gamma, wl.sigma, wl.depth, wl.x0, wl.y0, wl.width, targets=tgt)
        ur, vr = oracle.direct(wl.x, wl.y, wl.gamma, wl.sigma, targets=tgt)
        out["cpu_baseline"] = {
            "value": n / t_cpu, "unit": "particles/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one full FP64 oracle FMM evaluation of the same {n:,}-particle workload ({t_cpu:.2f} s)",
        }
        out["accuracy"] = {
            "rel_l2_vs_oracle_fmm": oracle.rel_l2(u_gpu, v_gpu, uo, vo),
            "rel_l2_vs_split_direct": oracle.rel_l2(u_gpu[tgt], v_gpu[tgt], us, vs),
            "rel_l2_vs_regularised_direct": oracle.rel_l2(u_gpu[tgt], v_gpu[tgt], ur, vr),
            "direct_targets": int(tgt.shape[0]),
        }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
