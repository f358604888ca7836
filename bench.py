#!/usr/bin/env python3
"""Throughput of one full FMM evaluation on one MI355X.

Default workload (the configuration the headline metric is quoted on, the
paper's largest run: one evaluation of 64 million particles, Section 7.2):
2^26 particles uniform in the unit square, gamma ~ U(-1, 1), sigma = 2e-4,
depth 11, p = 20, every stage in FP64.  A "step" is one complete evaluation
-- tree build (z-order keys, radix sort, leaf ranges), P2M, M2M, M2L, L2L,
L2P and P2P -- with inputs already resident in HBM.  ``--config`` picks
another workload (C1, C2, C3, C5; C4 runs the batched form: 512 uneven
instances, one graph replay per step) and ``--precision`` its precision.

Prints ONE JSON line.  ``value`` is particles per second over the timed
steps (wall clock, bracketed by device synchronisation).  ``roofline``
describes the kernel of the stage with the largest GPU time; its duration
is measured with HIP events that the library records on the evaluation's
own stream during the timed steps (for the batched form: during extra,
eagerly enqueued timed evaluations, since a replayed graph carries no
events).  ``forms`` (default workload) times the mixed-precision form of
the same workload, the 2^20-particle Lamb-Oseen workload in FP64, and the
batched form against plain FP64 single evaluations of the same instances;
``--extra-forms`` adds the vortex-method time stepping, the singular
kernel, target points, Lennard-Jones forces, the fast Gauss transform and
the 3D form.  ``cpu_baseline`` times the FP64 CPU oracle on the host cores
(rank 0, N = 1 only) and, from the same leg, reports the GPU results'
parity with the oracle and their accuracy against the direct sums on a
seeded sample of targets.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "particles/s per full FMM eval at ≤1e-6 rel. L2 vs direct; FP64 vs mixed"

# MI355X published vector peaks (256 CUs x 4 SIMDs x 16 lanes x 2 flops x
# 2.4 GHz = 78.6 TFLOP/s; FP32 counts the packed dual rate, 157.3).  Packed
# FP32 instructions are not generated in this build, so 78.6 TFLOP/s is the
# FP32 ceiling the kernels can reach; the published figure is kept as the peak.
PEAK_VALU_TFLOPS = {"f64": 78.6, "f32": 157.3}
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit:
#  P2P: 14 flops per near pair (2 differences, 3 for |d|^2, 1 scaling, 1 exp,
#       1 for 1 - e, 1 product, 1 division, 4 for the complex accumulation).
#  M2L: 8 p^2 flops per interaction-list pair (dense complex p x p product).
P2P_FLOPS_PER_PAIR = 14

# Kernel sources whose HBM traffic a committed counter summary describes.
TRAFFIC_SOURCES = {
    "k_p2p_l2p": ["paper_0905_2637_amd/csrc/fmm_near.hip", "paper_0905_2637_amd/csrc/fmm_device.h",
                  "paper_0905_2637_amd/csrc/fmm_internal.h"],
    "k_m2l": ["paper_0905_2637_amd/csrc/fmm_downward.hip", "paper_0905_2637_amd/csrc/fmm_device.h",
              "paper_0905_2637_amd/csrc/fmm_internal.h"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from profiles/<kernel>_<workload>_traffic.md, or None
    when there is no summary or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if kernel not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != source_hash(kernel):
        return None
    return int(m_bytes.group(1))


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


def describe(wl) -> str:
    prec = "FP64" if wl.precision == "fp64" else \
        f"mixed (FP32 P2P, FP32 M2L on the finest {wl.fp32_fine_levels} levels)"
    if wl.offsets is not None:
        return (f"{wl.name}: {len(wl.depths)} instances, {wl.n:,} particles in total, uniform unit square, "
                f"sigma={wl.sigma}, depths {int(wl.depths.min())}-{int(wl.depths.max())}, p={wl.p}, {prec}, batched")
    kind = {"C1": "uniform unit square", "C2": "jittered Lamb-Oseen lattice",
            "C3": "16-component Gaussian mixture", "C5": "uniform unit square"}[wl.name]
    return f"{wl.name}: {wl.n:,} particles, {kind}, sigma={wl.sigma}, depth {wl.depth}, p={wl.p}, {prec}"


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def roofline_of(stage_ms, pairs_near, pairs_m2l, p, dtype, workload_key):
    dominant = max(stage_ms, key=stage_ms.get)
    t = stage_ms[dominant] * 1e-3
    if dominant == "p2p_l2p":
        work, kernel = pairs_near * P2P_FLOPS_PER_PAIR, "k_p2p_l2p"
        note = f"{pairs_near} near pairs x {P2P_FLOPS_PER_PAIR} flops"
    elif dominant == "m2l":
        work, kernel = pairs_m2l * 8 * p * p, "k_m2l"
        note = f"{pairs_m2l} M2L pairs x 8p^2 flops"
    else:
        return {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": dominant, "stage_ms": round(stage_ms[dominant], 4)}
    achieved = work / t / 1e12
    peak = PEAK_VALU_TFLOPS[dtype]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": measured_traffic(kernel, workload_key),
            "kernel": kernel, "stage_ms": round(stage_ms[dominant], 4), "work": note}


def dev_arrays(wl, dev):
    import torch
    return tuple(torch.as_tensor(a, device=dev) for a in (wl.x, wl.y, wl.gamma))


# ---------------------------------------------------------------------------
# single evaluation
# ---------------------------------------------------------------------------

def run_single(wl, args, dev, kernel="gaussian"):
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = dev_arrays(wl, dev)
    u = torch.empty(wl.n, dtype=torch.float64, device=dev)
    v = torch.empty(wl.n, dtype=torch.float64, device=dev)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth, domain=(wl.x0, wl.y0, wl.width),
                   precision=wl.precision, fp32_fine_levels=wl.fp32_fine_levels, kernel=kernel)
    default_tuning = plan.tuning()
    tune = None
    if not args.no_autotune:
        # the launch shape the library's own autotuner picks for this problem
        # (seeded by the work model); outside the timed region
        t0 = time.perf_counter()
        plan.autotune(x, y, g, u, v, reps=3)
        tune = {"default": default_tuning, "chosen": plan.tuning(), **plan.autotune_report(),
                "seconds": round(time.perf_counter() - t0, 3)}
    for _ in range(args.warmup):
        plan.evaluate(x, y, g, u, v, check=False)
    torch.cuda.synchronize()
    if plan.out_of_domain():
        raise SystemExit("particles outside the domain")
    plan.set_timing(True)
    sec = timed(lambda: plan.evaluate(x, y, g, u, v, check=False), args.steps, 0)
    stages = plan.stats()
    plan.set_timing(False)
    stage_ms = {k: vv for k, vv in stages.items() if k != "evaluations"}
    leaf_start = plan.dump(fm.DUMP_LEAF_START)
    pn, pm = near_pairs(leaf_start, wl.depth), m2l_pairs(wl.depth)
    res = {"sec": sec, "stage_ms": stage_ms, "near_pairs": pn, "m2l_pairs": pm,
           "roofline": roofline_of(stage_ms, pn, pm, wl.p, "f64" if wl.precision == "fp64" else "f32",
                                   f"{wl.name}_{wl.precision}"),
           "u": u, "v": v, "tuning": plan.tuning(), "autotune": tune}
    plan.close()
    return res


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

def run_batch(wl, args, dev, precision=None, autotune=True, work_order=1):
    import torch
    import paper_0905_2637_amd as fm
    precision = precision or wl.precision
    x, y, g = dev_arrays(wl, dev)
    u = torch.empty(wl.n, dtype=torch.float64, device=dev)
    v = torch.empty(wl.n, dtype=torch.float64, device=dev)
    counts = np.diff(wl.offsets).tolist()
    depths = wl.depths.tolist()
    bp = fm.BatchPlan(counts, depths, wl.sigma, wl.p, domain=(wl.x0, wl.y0, wl.width), precision=precision,
                      fp32_fine_levels=wl.fp32_fine_levels)
    tune_info = None
    if autotune:
        # the whole grid first (for comparison), then the search the work model seeds
        os.environ["FMM_AUTOTUNE_EXHAUSTIVE"] = "1"
        try:
            full = bp.autotune(x, y, g, u, v, reps=2)
            full_timed = bp.autotune_report()["candidates_timed"]
        finally:
            del os.environ["FMM_AUTOTUNE_EXHAUSTIVE"]
        full_ms = timed(lambda: bp.evaluate(x, y, g, u, v, check=False), 10, 2) * 1e3
        seeded = bp.autotune(x, y, g, u, v, reps=2)
        rep = bp.autotune_report()
        seeded_ms = timed(lambda: bp.evaluate(x, y, g, u, v, check=False), 10, 2) * 1e3
        tune_info = {"seeded_choice": seeded, "seeded_candidates_timed": rep["candidates_timed"],
                     "seeded_choice_ms": round(seeded_ms, 4), "work_model_near_share": rep["near_share"],
                     "exhaustive_choice": full, "exhaustive_candidates_timed": full_timed,
                     "exhaustive_choice_ms": round(full_ms, 4)}
    if work_order != 1:
        t = bp.tuning()
        t["work_order"] = work_order
        bp.set_tuning(**t)
    bp.evaluate(x, y, g, u, v, check=False)
    torch.cuda.synchronize()
    if bp.out_of_domain():
        raise SystemExit("particles outside the domain")
    sec = timed(lambda: bp.evaluate(x, y, g, u, v, check=False), args.steps, args.warmup)
    # stage breakdown from eagerly enqueued timed evaluations (same kernels)
    bp.set_timing(True)
    for _ in range(max(3, min(args.steps, 10))):
        bp.evaluate(x, y, g, u, v, check=False)
    torch.cuda.synchronize()
    stages = bp.stats()
    bp.set_timing(False)
    stage_ms = {k: vv for k, vv in stages.items() if k != "evaluations"}
    ls = bp.dump(fm.DUMP_LEAF_START)
    pn = pm = 0
    seg = 0
    for L in depths:
        pn += near_pairs(ls[seg:seg + 4 ** L + 1] - ls[seg], L)
        pm += m2l_pairs(L)
        seg += 4 ** L + 1
    res = {"sec": sec, "stage_ms": stage_ms, "near_pairs": pn, "m2l_pairs": pm,
           "roofline": roofline_of(stage_ms, pn, pm, wl.p, "f64" if precision == "fp64" else "f32",
                                   f"{wl.name}_{precision}"),
           "u": u, "v": v, "tuning": bp.tuning(), "autotune": tune_info}
    bp.close()
    return res


def work_model_check(w4, args, dev, every=8):
    """The paper's work model (Section 5.2, eqs. 13-15) against measured cost:
    single FP64 evaluations of every `every`-th instance of the batched
    workload, GPU time per stage (HIP events) against the model's terms --
    eq. 15's whole-tree estimate for the total, its p^2 n_IL term (per box)
    for M2L, its n_nd N_i^2 term (per leaf) for the near field -- with a
    least-squares line t = a + b W and its R^2 for each."""
    import torch
    import paper_0905_2637_amd as fm
    p, pp = w4.p, float(w4.p) ** 2
    rows = []
    for i in range(0, len(w4.depths), every):
        a, b = int(w4.offsets[i]), int(w4.offsets[i + 1])
        L = int(w4.depths[i])
        x, y, g = (torch.as_tensor(arr[a:b], device=dev) for arr in (w4.x, w4.y, w4.gamma))
        u, v = torch.empty_like(x), torch.empty_like(x)
        plan = fm.Plan(b - a, w4.sigma, p, L, domain=(w4.x0, w4.y0, w4.width))
        for _ in range(3):
            plan.evaluate(x, y, g, u, v, check=False)
        plan.set_timing(True)
        for _ in range(5):
            plan.evaluate(x, y, g, u, v, check=False)
        st = plan.stats()
        plan.close()
        leaves = 4.0 ** L
        ni = (b - a) / leaves
        boxes = (4.0 ** (L + 1) - 1.0) / 3.0
        rows.append({"n": b - a, "L": L,
                     "total_ms": sum(vv for k, vv in st.items() if k != "evaluations"),
                     "m2l_ms": st["m2l"], "p2p_ms": st["p2p_l2p"],
                     "W": (leaves - 1.0) / 3.0 * pp * 35.0 + leaves * (2.0 * ni * p + pp * 27.0 + 9.0 * ni * ni),
                     "W_m2l": pp * 27.0 * boxes, "W_p2p": 9.0 * ni * ni * leaves})

    def fit(xs, ys):
        xs, ys = np.asarray(xs), np.asarray(ys)
        A = np.vstack([np.ones_like(xs), xs]).T
        (a0, b0), *_ = np.linalg.lstsq(A, ys, rcond=None)
        res = ys - (a0 + b0 * xs)
        r2 = 1.0 - float(np.sum(res ** 2)) / float(np.sum((ys - ys.mean()) ** 2))
        return {"intercept_ms": float(a0), "ms_per_unit": float(b0), "r2": r2}

    return {"instances": len(rows), "every": every,
            "total_vs_eq15": fit([r["W"] for r in rows], [r["total_ms"] for r in rows]),
            "m2l_vs_p2_nIL_term": fit([r["W_m2l"] for r in rows], [r["m2l_ms"] for r in rows]),
            "p2p_vs_nnd_Ni2_term": fit([r["W_p2p"] for r in rows], [r["p2p_ms"] for r in rows]),
            "depths": sorted(set(r["L"] for r in rows))}


def run_sequential_fp64(wl, args, dev):
    """Plain FP64 GPU FMM over the same instances, one single evaluation each."""
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = dev_arrays(wl, dev)
    u = torch.empty(wl.n, dtype=torch.float64, device=dev)
    v = torch.empty(wl.n, dtype=torch.float64, device=dev)
    counts = np.diff(wl.offsets)
    plans = {}
    for L in sorted(set(wl.depths.tolist())):
        nmax = int(counts[wl.depths == L].max())
        plans[L] = fm.Plan(nmax, wl.sigma, wl.p, L, domain=(wl.x0, wl.y0, wl.width))

    def step():
        for i, L in enumerate(wl.depths.tolist()):
            a, b = int(wl.offsets[i]), int(wl.offsets[i + 1])
            plans[L].evaluate(x[a:b], y[a:b], g[a:b], u[a:b], v[a:b])

    sec = timed(step, max(2, min(args.steps, 10)), 1)
    for p in plans.values():
        p.close()
    return sec


def run_time_stepping(wl, args, dev, steps=20):
    """Explicit midpoint steps of the vortex method (two evaluations and two
    particle updates per step, one graph replay each) on the bounding square."""
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = dev_arrays(wl, dev)
    scratch = torch.empty(4 * wl.n, dtype=torch.float64, device=dev)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth, domain=None, precision=wl.precision,
                   fp32_fine_levels=wl.fp32_fine_levels)
    dt = 1e-4
    plan.advance_rk2(x, y, g, dt, 2, scratch)              # warm-up and graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.advance_rk2(x, y, g, dt, steps, scratch)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    plan.close()
    return sec


def run_points(wl, args, dev, m_side=1024):
    """The velocity of the workload's particles on an m_side^2 vertex lattice
    of points (fmm_evaluate_at, FP64, the workload's explicit square)."""
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = dev_arrays(wl, dev)
    px, py = (torch.as_tensor(a, device=dev) for a in workloads.probe_lattice(m_side))
    m = int(px.shape[0])
    u = torch.empty(m, dtype=torch.float64, device=dev)
    v = torch.empty(m, dtype=torch.float64, device=dev)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth, domain=(wl.x0, wl.y0, wl.width), m_max=m)
    for _ in range(args.warmup):
        plan.evaluate_at(x, y, g, px, py, u, v, check=False)
    torch.cuda.synchronize()
    if plan.out_of_domain():
        raise SystemExit("particles or points outside the domain")
    plan.set_timing(True)
    sec = timed(lambda: plan.evaluate_at(x, y, g, px, py, u, v, check=False), args.steps, 0)
    stages = plan.stats()
    plan.close()
    return sec, m, {k: round(vv, 4) for k, vv in stages.items() if k != "evaluations"}


def run_lennard_jones(args, dev, m_side=1024):
    """Lennard-Jones forces on an m_side^2 jittered lattice in the unit square
    (spacing a, s = a / 1.12, cutoff 2.5 s, depth 8: leaves of 16 particles,
    wider than the cutoff), FP64, near field only."""
    import torch
    import paper_0905_2637_amd as fm
    rng = np.random.default_rng(900)
    a = 1.0 / m_side
    c = (np.arange(m_side) + 0.5) * a
    X, Y = np.meshgrid(c, c)
    n = m_side * m_side
    x = torch.as_tensor(X.ravel() + rng.uniform(-0.2 * a, 0.2 * a, n), device=dev)
    y = torch.as_tensor(Y.ravel() + rng.uniform(-0.2 * a, 0.2 * a, n), device=dev)
    g = torch.zeros(n, dtype=torch.float64, device=dev)
    fx = torch.empty_like(g)
    fy = torch.empty_like(g)
    s = a / 1.12
    plan = fm.Plan(n, s, 8, 8, kernel="lennard-jones", lj_epsilon=1.0, cutoff=2.5 * s)
    for _ in range(args.warmup):
        plan.evaluate(x, y, g, fx, fy, check=False)
    torch.cuda.synchronize()
    plan.set_timing(True)
    sec = timed(lambda: plan.evaluate(x, y, g, fx, fy, check=False), args.steps, 0)
    stages = plan.stats()
    plan.close()
    return sec, n, {k: round(vv, 4) for k, vv in stages.items() if k in ("tree", "p2p_l2p")}


def run_gauss_transform(wl, args, dev, sigma=0.02, depth=6, p=12):
    """The fast Gauss transform of the workload's particles (strengths = their
    circulations), Gaussian width sigma, leaf boxes at the given depth, p
    Hermite terms per axis, FP64."""
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = dev_arrays(wl, dev)
    G = torch.empty(wl.n, dtype=torch.float64, device=dev)
    v = torch.empty_like(G)
    plan = fm.Plan(wl.n, sigma, p, depth, domain=(wl.x0, wl.y0, wl.width), kernel="gauss-transform")
    for _ in range(args.warmup):
        plan.evaluate(x, y, g, G, v, check=False)
    torch.cuda.synchronize()
    plan.set_timing(True)
    sec = timed(lambda: plan.evaluate(x, y, g, G, v, check=False), args.steps, 0)
    stages = plan.stats()
    plan.close()
    return sec, G, {"tree": round(stages["tree"], 4), "transform": round(stages["p2m_m2m"], 4)}


def run_laplace_3d(args, dev, n=1 << 20, depth=5, p=6):
    """The 3D form: 2^20 charges uniform in the unit cube, octree depth 5
    (about 32 per leaf), Cartesian Taylor expansions of degree 6, FP64
    potential and gradient."""
    import torch
    import paper_0905_2637_amd as fm
    arrs = workloads.uniform_cube(n, 3003)
    x, y, z, q = (torch.as_tensor(a, device=dev) for a in arrs)
    out = tuple(torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4))
    plan = fm.Plan3D(n, p, depth)
    for _ in range(args.warmup):
        plan.evaluate(x, y, z, q, out, check=False)
    torch.cuda.synchronize()
    sec = timed(lambda: plan.evaluate(x, y, z, q, out, check=False), args.steps, 0)
    if plan.out_of_domain():
        raise RuntimeError("3D form: particles outside the cube")
    plan.close()
    return sec, arrs, out


# ---------------------------------------------------------------------------
# CPU oracle leg (the only part of the bench that touches the oracle)
# ---------------------------------------------------------------------------

def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pooled(pairs):
    num = sum(float(np.sum((u - uo) ** 2 + (v - vo) ** 2)) for u, v, uo, vo in pairs)
    den = sum(float(np.sum(uo ** 2 + vo ** 2)) for _, _, uo, vo in pairs)
    return (num / den) ** 0.5 if den > 0 else 0.0


def oracle_sample(wl):
    """A bounded sample of the workload for timing the CPU oracle: the
    particles in the lower-left quarter of the square, as a problem of its
    own on that quarter with one level less (same density, same leaf width,
    same sigma and p, so the same work per particle); the whole workload
    when it is small."""
    if wl.n <= (1 << 22) or wl.offsets is not None:
        return wl, "the whole workload"
    h = 0.5 * wl.width
    keep = (wl.x < wl.x0 + h) & (wl.y < wl.y0 + h)
    sub = workloads.Workload(wl.name, wl.x[keep], wl.y[keep], wl.gamma[keep], sigma=wl.sigma, depth=wl.depth - 1,
                             p=wl.p, x0=wl.x0, y0=wl.y0, width=h)
    return sub, (f"the {sub.n:,} particles in the lower-left quarter of the square, as a problem of their own "
                 f"(depth {sub.depth}: same density, leaf width, sigma and p)")


def accuracy_single(wl, res, args, forms):
    """The CPU baseline (one oracle FMM of a bounded sample of the workload,
    timed), then the GPU results against the oracle FMM and against the
    direct sums at seeded targets."""
    import oracle
    oracle.build()
    u_gpu = res["u"].cpu().numpy()
    v_gpu = res["v"].cpu().numpy()
    sub, what = oracle_sample(wl)
    t1 = time.perf_counter()
    oracle.fmm(sub.x, sub.y, sub.gamma, sub.sigma, sub.p, sub.depth, sub.x0, sub.y0, sub.width)
    t_cpu = time.perf_counter() - t1
    base = {"value": sub.n / t_cpu, "unit": "particles/s", "cores": oracle.threads(), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"one full FP64 oracle FMM evaluation of {what} ({t_cpu:.1f} s)"}
    del sub
    cfg = int(wl.name[1])
    m_split = args.accuracy_targets or (4096 if wl.n > (1 << 24) else 16384)
    tgt = workloads.sample_targets(wl.n, m_split, 1000 + cfg)
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, wl.x0, wl.y0, wl.width, targets=tgt)
    t1 = time.perf_counter()
    us, vs = oracle.direct_split(wl.x, wl.y, wl.gamma, wl.sigma, wl.depth, wl.x0, wl.y0, wl.width, targets=tgt)
    t_split = time.perf_counter() - t1
    treg = workloads.sample_targets(wl.n, min(m_split, args.regularised_targets), 2000 + cfg)
    ur, vr = oracle.direct(wl.x, wl.y, wl.gamma, wl.sigma, targets=treg)
    acc = {"rel_l2_vs_oracle_fmm": oracle.rel_l2(u_gpu[tgt], v_gpu[tgt], uo, vo),
           "oracle_fmm_targets": int(tgt.shape[0]),
           "rel_l2_vs_split_direct": oracle.rel_l2(u_gpu[tgt], v_gpu[tgt], us, vs),
           "split_direct_targets": int(tgt.shape[0]),
           "split_direct_pairs_per_s": float(tgt.shape[0]) * (wl.n - 1) / t_split,
           "rel_l2_vs_regularised_direct": oracle.rel_l2(u_gpu[treg], v_gpu[treg], ur, vr),
           "regularised_direct_targets": int(treg.shape[0]),
           "oracle_fmm_vs_split_direct": oracle.rel_l2(uo, vo, us, vs)}
    if forms and "_mixed_uv" in forms:
        um, vm = forms.pop("_mixed_uv")
        um, vm = um.cpu().numpy(), vm.cpu().numpy()
        f = forms["mixed"]
        f["rel_l2_vs_fp64_split_direct"] = oracle.rel_l2(um[tgt], vm[tgt], us, vs)
        f["split_direct_targets"] = int(tgt.shape[0])
        f["rel_l2_vs_regularised_direct"] = oracle.rel_l2(um[treg], vm[treg], ur, vr)
        f["rel_l2_vs_oracle_fmm"] = oracle.rel_l2(um[tgt], vm[tgt], uo, vo)
        f["within_gate"] = bool(f["rel_l2_vs_fp64_split_direct"] <= 1e-6)
    return {"cpu_baseline": base, "accuracy": acc}


def accuracy_c2(forms):
    """The C2 form against the oracle FMM at its 16,384 sampled targets and the
    split direct sum there."""
    import oracle
    u, v, wl = forms.pop("_c2")
    u, v = u.cpu().numpy(), v.cpu().numpy()
    tgt = workloads.sample_targets(wl.n, 16384, 1002)
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, wl.x0, wl.y0, wl.width, targets=tgt)
    us, vs = oracle.direct_split(wl.x, wl.y, wl.gamma, wl.sigma, wl.depth, wl.x0, wl.y0, wl.width, targets=tgt)
    forms["c2_fp64"].update({"rel_l2_vs_oracle_fmm": oracle.rel_l2(u[tgt], v[tgt], uo, vo),
                             "rel_l2_vs_split_direct": oracle.rel_l2(u[tgt], v[tgt], us, vs),
                             "targets": int(tgt.shape[0])})


def accuracy_batched(wl, fp64_uv, mixed_uv, per_inst_targets=64):
    """Pooled per-instance accuracy of the batched forms: FP64 against the
    oracle FMM of every instance; mixed against the FP64 split direct sum at
    seeded targets of every instance.  Also times the oracle FMM over all
    instances (the CPU baseline of the batched workload)."""
    import oracle
    oracle.build()
    u64, v64 = (a.cpu().numpy() for a in fp64_uv)
    um, vm = (a.cpu().numpy() for a in mixed_uv)
    fmm_pairs, split_pairs, worst = [], [], 0.0
    t_cpu = 0.0
    for i, L in enumerate(wl.depths.tolist()):
        a, b = int(wl.offsets[i]), int(wl.offsets[i + 1])
        t1 = time.perf_counter()
        uo, vo = oracle.fmm(wl.x[a:b], wl.y[a:b], wl.gamma[a:b], wl.sigma, wl.p, L, wl.x0, wl.y0, wl.width)
        t_cpu += time.perf_counter() - t1
        fmm_pairs.append((u64[a:b], v64[a:b], uo, vo))
        worst = max(worst, oracle.rel_l2(u64[a:b], v64[a:b], uo, vo))
        t = workloads.sample_targets(b - a, per_inst_targets, 3000 + i)
        us, vs = oracle.direct_split(wl.x[a:b], wl.y[a:b], wl.gamma[a:b], wl.sigma, L, wl.x0, wl.y0, wl.width,
                                     targets=t)
        split_pairs.append((um[a:b][t], vm[a:b][t], us, vs))
    return {"fp64_pooled_rel_l2_vs_oracle_fmm": _pooled(fmm_pairs),
            "fp64_worst_instance_rel_l2_vs_oracle_fmm": worst,
            "mixed_pooled_rel_l2_vs_fp64_split_direct": _pooled(split_pairs),
            "split_direct_targets_per_instance": per_inst_targets,
            "instances": len(wl.depths),
            "oracle_fmm_particles_per_s": wl.n / t_cpu, "oracle_fmm_seconds": t_cpu}


def run_forms(wl, res, args, dev):
    forms = {}
    value = wl.n / res["sec"]
    # the mixed-precision form of the same workload
    wm = workloads.Workload(**{**wl.__dict__})
    wm.precision, wm.fp32_fine_levels = "mixed", 2
    rm = run_single(wm, args, dev)
    forms["mixed"] = {"workload": describe(wm), "ms": round(rm["sec"] * 1e3, 4), "value": wm.n / rm["sec"],
                      "speedup_vs_fp64": res["sec"] / rm["sec"],
                      "stages_ms": {k: round(x, 4) for k, x in rm["stage_ms"].items()},
                      "roofline": rm["roofline"], "tuning": rm["tuning"], "autotune": rm["autotune"]}
    forms["_mixed_uv"] = (rm["u"], rm["v"])
    del rm
    # the Lamb-Oseen workload in FP64
    w2 = workloads.make("C2")
    r2 = run_single(w2, args, dev)
    forms["c2_fp64"] = {"workload": describe(w2), "ms": round(r2["sec"] * 1e3, 4), "value": w2.n / r2["sec"],
                        "stages_ms": {k: round(x, 4) for k, x in r2["stage_ms"].items()},
                        "roofline": r2["roofline"], "tuning": r2["tuning"], "autotune": r2["autotune"]}
    forms["_c2"] = (r2["u"], r2["v"], w2)
    # the batched form
    w4 = workloads.make("C4")
    rb = run_batch(w4, args, dev)
    rb64 = run_batch(w4, args, dev, precision="fp64")
    rb_in_order = run_batch(w4, args, dev, work_order=0)
    seq = run_sequential_fp64(w4, args, dev)
    forms["batched"] = {"workload": describe(w4), "ms": round(rb["sec"] * 1e3, 4), "value": w4.n / rb["sec"],
                        "fp64_batched_ms": round(rb64["sec"] * 1e3, 4),
                        "fp64_sequential_single_ms": round(seq * 1e3, 4),
                        "speedup_vs_fp64_sequential": seq / rb["sec"],
                        "speedup_fp64_batched_vs_sequential": seq / rb64["sec"],
                        "input_order_ms": round(rb_in_order["sec"] * 1e3, 4),
                        "work_order_speedup": rb_in_order["sec"] / rb["sec"],
                        "tuning": rb["tuning"], "autotune": rb["autotune"], "roofline": rb["roofline"],
                        "work_model": work_model_check(w4, args, dev)}
    forms["_c4"] = (w4, (rb64["u"], rb64["v"]), (rb["u"], rb["v"]))
    if args.extra_forms:
        extra_forms(forms, args, dev)
    return forms


def extra_forms(forms, args, dev):
    wl = workloads.make("C2")
    base = run_single(wl, args, dev)["sec"]
    ts = run_time_stepping(wl, args, dev)
    forms["time_stepping"] = {"workload": "C2 particles moved by the explicit midpoint rule (two FP64 "
                                          "evaluations per step, bounding-square domain)",
                              "ms_per_step": round(ts * 1e3, 4), "particle_steps_per_s": wl.n / ts,
                              "step_vs_two_evaluations": ts / (2 * base)}
    rs = run_single(workloads.make("C2"), args, dev, kernel="singular")
    forms["singular_kernel"] = {"workload": "C2 with the singular kernel of eq. 7 in the near field (point "
                                            "vortices, FP64)",
                                "ms": round(rs["sec"] * 1e3, 4), "value": wl.n / rs["sec"],
                                "stages_ms": {k: round(x, 4) for k, x in rs["stage_ms"].items()}}
    tp, mp, sp = run_points(workloads.make("C2"), args, dev)
    forms["points"] = {"workload": "C2 particles, velocity on a 1024 x 1024 vertex lattice of points "
                                   "(FP64, eq. 1 with targets apart from the sources)",
                       "ms": round(tp * 1e3, 4), "points_per_s": mp / tp, "stages_ms": sp}
    tl, nl, sl = run_lennard_jones(args, dev)
    forms["lennard_jones"] = {"workload": "2^20 Lennard-Jones particles, jittered 1024 x 1024 lattice, s = a/1.12, "
                                          "cutoff 2.5 s, depth 8 (FP64 forces, near field only)",
                              "ms": round(tl * 1e3, 4), "particles_per_s": nl / tl, "stages_ms": sl}
    tg, _, sg = run_gauss_transform(wl, args, dev)
    forms["gauss_transform"] = {"workload": "fast Gauss transform of C2's particles (strengths = circulations), "
                                            "sigma = 0.02, 4096 leaf boxes (depth 6), p = 12 per axis, FP64",
                                "ms": round(tg * 1e3, 4), "particles_per_s": wl.n / tg, "stages_ms": sg}
    t3, _, _ = run_laplace_3d(args, dev)
    forms["laplace_3d"] = {"workload": "3D form: 2^20 charges uniform in the unit cube, octree depth 5, "
                                       "Cartesian Taylor expansions of degree 6, FP64 potential and gradient",
                           "ms": round(t3 * 1e3, 4), "particles_per_s": (1 << 20) / t3}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C5", help="workload: C1, C2, C3, C4 (batched) or C5 (default)")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="precision of the headline workload (default: FP64 for C5, the workload's own otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-forms", action="store_true", help="skip the mixed, C2 and batched forms")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shape instead of the autotuner's choice")
    ap.add_argument("--extra-forms", action="store_true",
                    help="also time time stepping, the singular kernel, target points, Lennard-Jones, the fast "
                         "Gauss transform and the 3D form")
    ap.add_argument("--form", default=None, choices=["laplace_3d"],
                    help="time only this form (one JSON line with its timing; for profiling)")
    ap.add_argument("--accuracy-targets", type=int, default=0,
                    help="targets of the split direct sum (default 4,096 at C5, 16,384 otherwise)")
    ap.add_argument("--regularised-targets", type=int, default=1024,
                    help="targets of the fully regularised direct sum (reported, not gated)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed region, run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (how the evaluation "
                                   "would shard is described in the design notes)", "n_gpus": args.gpus}))
        return 2

    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        return 1
    if args.form == "laplace_3d":
        t3, _, _ = run_laplace_3d(args, torch.device("cuda"))
        print(json.dumps({"form": "laplace_3d", "ms": t3 * 1e3, "particles_per_s": (1 << 20) / t3,
                          "steps": args.steps, "warmup": args.warmup}))
        return 0
    dev = torch.device("cuda:0")
    wl = workloads.make(args.config)
    if args.precision:
        wl.precision = args.precision
        wl.fp32_fine_levels = 2 if args.precision == "mixed" else 0
    elif wl.name == "C5":
        wl.precision, wl.fp32_fine_levels = "fp64", 0
    batched = wl.offsets is not None
    res = run_batch(wl, args, dev) if batched else run_single(wl, args, dev)
    value = wl.n / res["sec"]
    print(f"# headline {wl.name} {wl.precision}: {res['sec'] * 1e3:.3f} ms", file=sys.stderr, flush=True)

    forms = None
    if not args.no_forms and not batched and wl.name == "C5":
        forms = run_forms(wl, res, args, dev)
        print("# forms timed", file=sys.stderr, flush=True)

    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "n": wl.n, "depth": wl.depth, "p": wl.p, "sigma": wl.sigma,
                   "precision": wl.precision, "parallelism": "single GPU"},
        "stages_ms": {k: round(x, 4) for k, x in res["stage_ms"].items()},
        "work": {"near_pairs": res["near_pairs"], "m2l_pairs": res["m2l_pairs"]},
        "tuning": res["tuning"],
        "autotune": res.get("autotune"),
        "roofline": res["roofline"],
    }
    if not args.no_cpu_baseline and not batched:
        out.update(accuracy_single(wl, res, args, forms))
        print("# oracle leg done", file=sys.stderr, flush=True)
        if forms is not None:
            accuracy_c2(forms)
            w4, f64uv, mixuv = forms.pop("_c4")
            forms["batched"]["accuracy"] = accuracy_batched(w4, f64uv, mixuv)
    if forms is not None:
        for k in [k for k in forms if k.startswith("_")]:
            forms.pop(k)
        out["forms"] = forms
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
