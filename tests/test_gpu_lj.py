"""The Lennard-Jones kernel on the GPU (the molecular-dynamics kernel
Section 8 names): forces from the near-field pass alone, the tree serving as
a cell list (cutoff at most the leaf width), no far field.

* FP64 parity with the oracle's plain O(N^2) sum with the same cutoff, on a
  jittered lattice (quads of 64 particles: the pair-once path) and on
  leaves of hundreds (chunks of 64 targets), and over a batch of instances;
* Newton's third law: the forces sum to zero to rounding;
* the parameter and entry-point checks (cutoff wider than a leaf, no
  explicit square, mixed precision, points, time stepping).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _lattice(m, jitter, seed, lo=0.0, hi=1.0):
    """m x m cell-centred lattice on [lo, hi)^2, each point moved by up to
    jitter lattice spacings per axis."""
    rng = np.random.default_rng(seed)
    a = (hi - lo) / m
    c = lo + (np.arange(m) + 0.5) * a
    X, Y = np.meshgrid(c, c)
    x = X.ravel() + rng.uniform(-jitter * a, jitter * a, m * m)
    y = Y.ravel() + rng.uniform(-jitter * a, jitter * a, m * m)
    return x, y, a


def _forces(x, y, s, eps, rc, depth, domain=(0.0, 0.0, 1.0)):
    import torch
    import paper_0905_2637_amd as fm
    plan = fm.Plan(len(x), s, 8, depth, domain=domain, kernel="lennard-jones", lj_epsilon=eps, cutoff=rc)
    fx, fy = plan.evaluate(_dev(x), _dev(y), _dev(np.zeros(len(x))), check=True)
    torch.cuda.synchronize()
    plan.close()
    return fx.cpu().numpy(), fy.cpu().numpy()


def _check(fx, fy, ox, oy):
    scale = np.sqrt(np.mean(ox ** 2 + oy ** 2))
    err = np.sqrt(np.mean((fx - ox) ** 2 + (fy - oy) ** 2)) / scale
    assert err < 1e-12, f"rel L2 vs the oracle {err:.3e}"
    assert np.max(np.hypot(fx - ox, fy - oy)) < 1e-10 * np.max(np.hypot(ox, oy))


@pytest.mark.parametrize("m,depth,rc_over_s", [(128, 5, 2.5), (96, 3, 8.0)])
def test_lj_matches_oracle(m, depth, rc_over_s):
    """m = 128, depth 5: 16 particles per leaf, quads of 64 (each pair inside a
    quad once); m = 96, depth 3: 144 per leaf (chunks of 64 targets, four per
    lane)."""
    x, y, a = _lattice(m, 0.2, 800 + m)
    s, eps = a / 1.12, 0.8
    rc = rc_over_s * s
    assert rc <= 1.0 / (1 << depth)
    fx, fy = _forces(x, y, s, eps, rc, depth)
    ox, oy = oracle.lj_forces(x, y, eps, s, rc)
    _check(fx, fy, ox, oy)
    scale = np.max(np.hypot(ox, oy))
    assert abs(fx.sum()) < 1e-12 * scale * len(x) and abs(fy.sum()) < 1e-12 * scale * len(x)


def test_lj_sparse_and_coincident():
    """A loose gas with empty leaves, two coincident particles (no force
    between them) and pairs straddling leaf edges."""
    rng = np.random.default_rng(810)
    x, y = rng.random(3000), rng.random(3000)
    x = np.concatenate([x, [0.25, 0.25, 0.5 - 0.004, 0.5 + 0.004]])
    y = np.concatenate([y, [0.75, 0.75, 0.5, 0.5]])
    s, eps, rc = 0.006, 1.3, 0.03
    fx, fy = _forces(x, y, s, eps, rc, 5)
    ox, oy = oracle.lj_forces(x, y, eps, s, rc)
    _check(fx, fy, ox, oy)


def test_lj_batch():
    import torch
    import paper_0905_2637_amd as fm
    parts = [_lattice(m, 0.25, 820 + m) for m in (40, 64, 24)]
    depths = [3, 4, 3]
    s, eps, rc = 0.009, 1.0, 0.03
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    counts = [len(p[0]) for p in parts]
    plan = fm.BatchPlan(counts, depths, s, 8, kernel="lennard-jones", lj_epsilon=eps, cutoff=rc)
    fx, fy = plan.evaluate(_dev(x), _dev(y), _dev(np.zeros(len(x))))
    torch.cuda.synchronize()
    fx, fy = fx.cpu().numpy(), fy.cpu().numpy()
    plan.close()
    off = np.concatenate([[0], np.cumsum(counts)])
    for i in range(3):
        a, b = off[i], off[i + 1]
        ox, oy = oracle.lj_forces(x[a:b], y[a:b], eps, s, rc)
        _check(fx[a:b], fy[a:b], ox, oy)


def test_lj_unsupported_combinations():
    import ctypes as C
    import paper_0905_2637_amd as fm
    lib = fm.load()
    out = C.c_size_t(0)

    def ws(**kw):
        base = dict(kernel="lennard-jones", lj_epsilon=1.0, cutoff=0.03)
        base.update(kw)
        prm = fm.make_params(1000, 0.01, 8, 5, **base)
        return lib.fmm_workspace_size(C.byref(prm), C.byref(out))

    assert ws() == fm.FMM_OK
    assert ws(cutoff=0.04) == fm.FMM_E_UNSUPPORTED          # wider than a leaf (1/32)
    assert ws(domain=None) == fm.FMM_E_UNSUPPORTED          # the leaf width must be known
    assert ws(precision="mixed") == fm.FMM_E_UNSUPPORTED
    assert ws(lj_epsilon=0.0) == fm.FMM_E_ARG
    assert ws(cutoff=-1.0) == fm.FMM_E_ARG
    x, y, _ = _lattice(20, 0.2, 830)
    plan = fm.Plan(400, 0.01, 8, 5, m_max=10, kernel="lennard-jones", lj_epsilon=1.0, cutoff=0.03)
    t = _dev(np.full(10, 0.5))
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate_at(_dev(x), _dev(y), _dev(np.zeros(400)), t, t)
    assert ei.value.status == fm.FMM_E_UNSUPPORTED
    with pytest.raises(fm.FmmError) as ei:
        plan.advance_rk2(_dev(x), _dev(y), _dev(np.zeros(400)), 1e-3, 1)
    assert ei.value.status == fm.FMM_E_UNSUPPORTED
    plan.close()
