"""fmm_evaluate_static, the entry point that allocates nothing (its workspace
is a fixed device array of the library), against fmm_plan + fmm_evaluate on
the same inputs, through the C ABI: the same kernels in the same order, so
the velocities must agree bit for bit.  Two calls in a row, the second with
fewer particles (same parameters, so the kept operator tables are reused),
then a call with other parameters (a new plan over the same array), then
FP64 parity with the oracle FMM; the normal path's workspace is filled with
0xff bytes first, so neither side can lean on zeroed memory."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _normal(x, y, g, sigma, p, L, precision="fp64", n_max=None):
    import torch
    import paper_0905_2637_amd as fm
    fm.WORKSPACE_FILL = 0xFF
    try:
        plan = fm.Plan(len(x) if n_max is None else n_max, sigma, p, L, precision=precision)
    finally:
        fm.WORKSPACE_FILL = None
    u, v = plan.evaluate(_dev(x), _dev(y), _dev(g))
    torch.cuda.synchronize()
    plan.close()
    return u.cpu().numpy(), v.cpu().numpy()


def _static(x, y, g, sigma, p, L, precision="fp64", n_max=None):
    import torch
    import paper_0905_2637_amd as fm
    u, v = fm.evaluate_static(_dev(x), _dev(y), _dev(g), sigma, p, L, precision=precision, n_max=n_max)
    torch.cuda.synchronize()
    return u.cpu().numpy(), v.cpu().numpy()


def test_static_matches_plan_on_two_calls_then_other_parameters():
    wl = workloads.make("C1")
    print(f"static call 1: n={wl.n} depth={wl.depth} p={wl.p}", flush=True)
    u1, v1 = _static(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, n_max=wl.n)
    r1 = _normal(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, n_max=wl.n)
    assert np.array_equal(u1, r1[0]) and np.array_equal(v1, r1[1])
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth)
    assert oracle.rel_l2(u1, v1, uo, vo) < 1e-12
    # second call, same parameters, fewer particles
    m = 1500
    print(f"static call 2: n={m}", flush=True)
    u2, v2 = _static(wl.x[:m], wl.y[:m], wl.gamma[:m], wl.sigma, wl.p, wl.depth, n_max=wl.n)
    r2 = _normal(wl.x[:m], wl.y[:m], wl.gamma[:m], wl.sigma, wl.p, wl.depth, n_max=wl.n)
    assert np.array_equal(u2, r2[0]) and np.array_equal(v2, r2[1])
    uo, vo = oracle.fmm(wl.x[:m], wl.y[:m], wl.gamma[:m], wl.sigma, wl.p, wl.depth)
    assert oracle.rel_l2(u2, v2, uo, vo) < 1e-12
    # other parameters and a smaller input again: a new plan over the same array
    x, y, g = workloads.uniform_square(700, 77)
    print("static call 3: n=700 depth=3 p=8 mixed", flush=True)
    u3, v3 = _static(x, y, g, 0.01, 8, 3, precision="mixed")
    r3 = _normal(x, y, g, 0.01, 8, 3, precision="mixed")
    assert np.array_equal(u3, r3[0]) and np.array_equal(v3, r3[1])


def test_static_rejects_what_does_not_fit():
    import torch
    import paper_0905_2637_amd as fm
    z = torch.zeros(4, dtype=torch.float64, device="cuda")
    # 2^20 particles at depth 8, p = 17 need far more than the fixed array holds
    with pytest.raises(fm.FmmError) as ei:
        fm.evaluate_static(z, z, z, 0.002, 17, 8, n_max=1 << 20)
    assert ei.value.status == fm.FMM_E_CAPACITY
    with pytest.raises(fm.FmmError) as ei:
        fm.evaluate_static(z, z, z, 0.002, 17, 3, n_max=2)      # n > n_max
    assert ei.value.status == fm.FMM_E_CAPACITY
    u, v = fm.evaluate_static(z[:0], z[:0], z[:0], 0.002, 17, 3, n_max=2)   # n = 0: nothing to do
    assert u.numel() == 0
