"""A caller may capture an evaluation into a graph of its own: fmm_evaluate
and fmm_evaluate_at enqueue kernels only (no allocation, no memset node, no
synchronisation) on the caller's stream.  The binding's status check (a
synchronising read of the device status word) is turned off inside a
capture (check=False).

Each graph is replayed several times, the inputs changed in place between
replays and other device work run eagerly in between, and every replay is
compared with an eager evaluation of the same inputs (bit for bit: the same
kernels run in the same order).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _replays(plan, call, inputs, outputs, shift):
    """Capture call(), then three rounds of: move the inputs, run unrelated
    eager work, replay, synchronise, compare with an eager call."""
    import torch
    call()                                           # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for r in range(3):
        for t in inputs:
            t.add_(shift(r, t))
        junk = (junk * 1.0001).sin_()                # the program's own eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outputs]
        call()
        torch.cuda.synchronize()
        for a, b in zip(got, outputs):
            assert torch.equal(a, b), f"replay {r} differs from the eager evaluation"
    del g


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_captured_evaluate(precision):
    import torch
    import paper_0905_2637_amd as fm
    x, y, gam = (_dev(a) for a in workloads.uniform_square(20000, 701))
    x.mul_(0.9)
    y.mul_(0.9)
    u = torch.empty_like(x)
    v = torch.empty_like(x)
    plan = fm.Plan(20000, 0.004, 17, 5, precision=precision)
    _replays(plan, lambda: plan.evaluate(x, y, gam, u, v, check=False), [x, y], [u, v],
             lambda r, t: torch.full_like(t, 0.01 * (r + 1)))
    assert plan.out_of_domain() == 0
    plan.close()


def test_captured_evaluate_at_bounding_square():
    import torch
    import paper_0905_2637_amd as fm
    x, y, gam = (_dev(a) for a in workloads.uniform_square(8000, 702))
    rng = np.random.default_rng(703)
    tx, ty = _dev(rng.random(5000)), _dev(rng.random(5000))
    u = torch.empty_like(tx)
    v = torch.empty_like(tx)
    plan = fm.Plan(8000, 0.006, 12, 4, domain=None, m_max=5000)
    _replays(plan, lambda: plan.evaluate_at(x, y, gam, tx, ty, u, v, check=False), [x, ty], [u, v],
             lambda r, t: 0.05 * torch.sin(t * (r + 2)))
    plan.close()
