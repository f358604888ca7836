"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
map its dumps (z-order boxes, scaled coefficients) onto the oracle's layout
(row-major boxes, unscaled coefficients)."""
from __future__ import annotations

import numpy as np


def deinterleave(k: np.ndarray):
    """z-order key -> (a, b): even bits to a, odd bits to b."""
    k = np.asarray(k, dtype=np.uint64)
    a = np.zeros_like(k)
    b = np.zeros_like(k)
    for bit in range(16):
        a |= ((k >> np.uint64(2 * bit)) & np.uint64(1)) << np.uint64(bit)
        b |= ((k >> np.uint64(2 * bit + 1)) & np.uint64(1)) << np.uint64(bit)
    return a.astype(np.int64), b.astype(np.int64)


def interleave(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    k = np.zeros_like(a)
    for bit in range(16):
        k |= ((a >> np.uint64(bit)) & np.uint64(1)) << np.uint64(2 * bit)
        k |= ((b >> np.uint64(bit)) & np.uint64(1)) << np.uint64(2 * bit + 1)
    return k.astype(np.int64)


def level_offset(l: int) -> int:
    return ((1 << (2 * l)) - 1) // 3


def gpu_coeffs_to_oracle(coef: np.ndarray, L: int, W: float, kind: str) -> np.ndarray:
    """Scaled z-order coefficients [Lambda, p] -> unscaled row-major [Lambda, p].

    Multipole: a_k = ahat_k w^k; local: b_l = bhat_l / w^(l+1); w = W / 2^l.
    Levels 0 and 1 carry no expansions (nothing is far from anything there):
    the library leaves those rows of its workspace unwritten, so they stay 0.
    """
    p = coef.shape[1]
    out = np.zeros_like(coef)
    k = np.arange(p)
    for l in range(2, L + 1):
        side = 1 << l
        off = level_offset(l)
        m = np.arange(side * side)
        a, b = deinterleave(m)
        rm = b * side + a
        w = W / side
        scale = w ** k if kind == "me" else 1.0 / w ** (k + 1)
        out[off + rm] = coef[off + m] * scale[None, :]
    return out


def run(x, y, g, sigma, p, L, domain=(0.0, 0.0, 1.0), precision="fp64", fine=2, n_max=None, timing=False):
    """One evaluation through the C ABI; returns (u, v, plan) with numpy outputs."""
    import torch
    import paper_0905_2637_amd as fm
    n = len(x)
    plan = fm.Plan(n_max if n_max is not None else max(n, 1), sigma, p, L, domain=domain,
                   precision=precision, fp32_fine_levels=fine)
    dev = torch.device("cuda")
    xt = torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    yt = torch.as_tensor(np.ascontiguousarray(y, np.float64), device=dev)
    gt = torch.as_tensor(np.ascontiguousarray(g, np.float64), device=dev)
    if timing:
        plan.set_timing(True)
    u, v = plan.evaluate(xt, yt, gt, check=False)   # callers read the status themselves
    torch.cuda.synchronize()
    return u.cpu().numpy(), v.cpu().numpy(), plan
