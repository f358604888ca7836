"""The singular kernel of eq. 7 (point vortices) on the GPU: the same FMM
with the near-field pair kernel 1/z instead of the Gaussian core, so the
result approximates the singular direct sum itself (no split-kernel gap).

* FP64 parity with the oracle FMM (sigma = 0) at particles, at target
  points and over a batch of instances (1e-12);
* Kelvin's rotating polygon: N equal point vortices on a circle move along
  it with speed (N - 1) gamma / (4 pi R);
* the mixed form within its FP32 error model, particle by particle;
* time stepping: the polygon turns rigidly with angular velocity
  (N - 1) gamma / (4 pi R^2), the explicit midpoint rule's error falling at
  second order in dt.
"""
import math

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


def _evaluate(x, y, g, p, L, precision="fp64", domain=(0.0, 0.0, 1.0)):
    import torch
    import paper_0905_2637_amd as fm
    plan = fm.Plan(len(x), 0.0, p, L, domain=domain, precision=precision, kernel="singular")
    u, v = plan.evaluate(_dev(x), _dev(y), _dev(g), check=True)
    torch.cuda.synchronize()
    plan.close()
    return u.cpu().numpy(), v.cpu().numpy()


def _polygon(N, gam=0.37, R=0.3, c=(0.5, 0.5), phase=0.1):
    th = 2 * math.pi * np.arange(N) / N + phase
    return c[0] + R * np.cos(th), c[1] + R * np.sin(th), np.full(N, gam), th


@pytest.mark.parametrize("p", [12, 24])
def test_singular_matches_oracle_fmm(p):
    wl = workloads.make("C1")
    u, v = _evaluate(wl.x, wl.y, wl.gamma, p, wl.depth)
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, 0.0, p, wl.depth)
    err = oracle.rel_l2(u, v, uo, vo)
    assert err < 1e-12, f"rel L2 vs the oracle FMM {err:.3e}"
    if p == 24:
        ud, vd = oracle.direct(wl.x, wl.y, wl.gamma, 0.0)
        assert oracle.rel_l2(u, v, ud, vd) < 1e-10


def test_singular_kelvin_polygon():
    N, gam, R = 12, 0.37, 0.3
    x, y, g, th = _polygon(N, gam, R)
    u, v = _evaluate(x, y, g, 32, 3)
    speed = (N - 1) * gam / (4 * math.pi * R)
    assert np.max(np.abs(u + speed * np.sin(th))) < 1e-13
    assert np.max(np.abs(v - speed * np.cos(th))) < 1e-13


def test_singular_mixed_error_model():
    """The mixed form's near field takes differences of FP32 leaf-relative
    offsets (magnitude <= 1.5 leaf widths w, so each is off by at most about
    3 2^-24 w): a pair term gamma / (2 pi r) is off by about 2e-7 w / r of
    itself, plus the FP32 roundings of the product, the reciprocal and the
    running sum (4e-6 of itself allows for those).  Unlike the Gaussian
    core, which bounds every term, the singular kernel lets the closest pairs
    dominate, so the check is per particle against that bound, with the far
    field (FP32 M2L on the fine levels, p = 17 truncation) held to 1e-6 of
    the sum of its term magnitudes."""
    wl = workloads.make("C1")
    u, v = _evaluate(wl.x, wl.y, wl.gamma, 17, wl.depth, precision="mixed")
    ud, vd = oracle.direct(wl.x, wl.y, wl.gamma, 0.0)
    w = 1.0 / (1 << wl.depth)
    ia, ib, _ = oracle.quantize(wl.x, wl.y, wl.depth)
    near = (np.abs(ia[:, None] - ia[None, :]) <= 1) & (np.abs(ib[:, None] - ib[None, :]) <= 1)
    r = np.hypot(wl.x[:, None] - wl.x[None, :], wl.y[:, None] - wl.y[None, :])
    np.fill_diagonal(r, np.inf)
    term = np.abs(wl.gamma)[None, :] / (2 * math.pi * r)
    bound = (np.where(near, term * (2e-7 * w / r + 4e-6), 0.0).sum(axis=1)
             + 1e-6 * np.where(near, 0.0, term).sum(axis=1))
    err = np.hypot(u - ud, v - vd)
    assert np.all(err <= bound), f"worst error / bound {np.max(err / bound):.3f}"
    assert oracle.rel_l2(u, v, ud, vd) < 1e-5


def test_singular_at_points():
    import torch
    import paper_0905_2637_amd as fm
    wl = workloads.make("C1")
    rng = np.random.default_rng(601)
    tx = np.concatenate([rng.random(1999), wl.x[:40]])
    ty = np.concatenate([rng.random(1999), wl.y[:40]])
    plan = fm.Plan(wl.n, 0.0, 17, wl.depth, m_max=len(tx), kernel="singular")
    u, v = plan.evaluate_at(_dev(wl.x), _dev(wl.y), _dev(wl.gamma), _dev(tx), _dev(ty), check=True)
    torch.cuda.synchronize()
    plan.close()
    uo, vo, _ = oracle.fmm_at(wl.x, wl.y, wl.gamma, 0.0, 17, wl.depth, tx, ty)
    err = oracle.rel_l2(u.cpu().numpy(), v.cpu().numpy(), uo, vo)
    assert err < 1e-12, f"rel L2 vs the oracle FMM at points {err:.3e}"


def test_singular_batch():
    import torch
    import paper_0905_2637_amd as fm
    sizes, depths = [700, 3000, 1500, 64], [2, 4, 3, 2]
    parts = [workloads.uniform_square(n, 610 + i) for i, n in enumerate(sizes)]
    x, y, g = (np.concatenate([q[k] for q in parts]) for k in range(3))
    plan = fm.BatchPlan(sizes, depths, 0.0, 12, kernel="singular")
    u, v = plan.evaluate(_dev(x), _dev(y), _dev(g))
    torch.cuda.synchronize()
    u, v = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for i, (n, L) in enumerate(zip(sizes, depths)):
        a, b = off[i], off[i + 1]
        uo, vo = oracle.fmm(x[a:b], y[a:b], g[a:b], 0.0, 12, L)
        err = oracle.rel_l2(u[a:b], v[a:b], uo, vo)
        assert err < 1e-12, f"instance {i}: rel L2 vs the oracle FMM {err:.3e}"


def test_singular_polygon_rotates_rigidly():
    import torch
    import paper_0905_2637_amd as fm
    N, gam, R, T = 6, 0.37, 0.3, 1.0
    omega = (N - 1) * gam / (4 * math.pi * R * R)
    errs = []
    for steps in (25, 50):
        x0, y0, g, th = _polygon(N, gam, R)
        x, y = _dev(x0), _dev(y0)
        plan = fm.Plan(N, 0.0, 32, 3, domain=None, kernel="singular")
        plan.advance_rk2(x, y, _dev(g), T / steps, steps)
        torch.cuda.synchronize()
        plan.close()
        xe = 0.5 + R * np.cos(th + omega * T)
        ye = 0.5 + R * np.sin(th + omega * T)
        errs.append(float(np.max(np.hypot(x.cpu().numpy() - xe, y.cpu().numpy() - ye))))
    assert errs[0] < 1e-3, errs
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_singular_coincident_large_circulation(precision):
    """Coincident particles contribute nothing (a pair at zero distance has no
    kernel value), also when the circulations are so large that a guard term
    in the squared distance would overflow gamma / r^2: 100 particles of the
    C1 workload are duplicated exactly (inside quads of sibling leaves and in
    the general near-field path alike) and every circulation is scaled to
    about 1e9.  The velocities must stay finite and equal the oracle's."""
    wl = workloads.make("C1")
    idx = np.arange(0, wl.n, wl.n // 100)[:100]
    x = np.concatenate([wl.x, wl.x[idx]])
    y = np.concatenate([wl.y, wl.y[idx]])
    g = 1e9 * np.concatenate([wl.gamma, -wl.gamma[idx] + 0.5])
    u, v = _evaluate(x, y, g, 17, wl.depth, precision=precision)
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))
    if precision == "fp64":
        uo, vo = oracle.fmm(x, y, g, 0.0, 17, wl.depth)
        err = oracle.rel_l2(u, v, uo, vo)
        assert err < 1e-12, f"rel L2 vs the oracle FMM {err:.3e}"
    else:
        ud, vd = oracle.direct(x, y, g, 0.0)
        err = oracle.rel_l2(u, v, ud, vd)
        assert err < 1e-5, f"rel L2 vs the singular direct sum {err:.3e}"
