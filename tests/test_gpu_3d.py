"""The 3D form on the GPU (octree, Laplace kernel 1/r, Cartesian Taylor
expansions): parity with the oracle's 3D FMM, through the C ABI.

* the tree bit for bit: Morton keys, the stable permutation and the leaf
  ranges against the oracle's keys and stable order;
* FP64 potential and gradient within 1e-12 relative L2 of the oracle FMM
  (same tree, lists, degree), for degrees 0-9, depths 0-4, uniform and
  clustered particles, a cube that is not the unit cube;
* at depth <= 1 (no far field) the plain sum itself;
* against the plain sum: the truncation error the degree allows;
* particles outside the cube or NaN: counted, zero outputs, no effect;
  one particle, none, and the capacity check;
* a million particles at depth 5, degree 6: sampled particles against the
  oracle's plain sum at those particles.
"""
import math

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


def _gpu(x, y, z, q, p, L, origin=(0.0, 0.0, 0.0), W=1.0, check=True):
    import torch
    import paper_0905_2637_amd as fm
    plan = fm.Plan3D(len(x), p, L, origin, W)
    out = plan.evaluate(_dev(x), _dev(y), _dev(z), _dev(q), check=check)
    torch.cuda.synchronize()
    nbad = plan.out_of_domain()
    plan.close()
    return tuple(o.cpu().numpy() for o in out) + (nbad,)


def _rel(a, b):
    num = sum(np.sum((u - v) ** 2) for u, v in zip(a[1:4], b[1:4]))
    den = sum(np.sum(v ** 2) for v in b[1:4])
    return math.sqrt(num / den), float(np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0]))


def _uniform(n, seed):
    rng = np.random.default_rng(seed)
    return rng.random(n), rng.random(n), rng.random(n), rng.uniform(-1, 1, n)


@pytest.mark.parametrize("n,L,p,seed", [
    (2000, 2, 4, 1),
    (3000, 3, 9, 2),
    (5000, 3, 6, 3),
    (1500, 3, 0, 4),          # monopoles only
    (800, 2, 1, 5),
    (20000, 4, 5, 6),
    (4000, 3, 8, 7),
    (2500, 3, 2, 8),          # the M2L lane split of degree 2
    (2500, 4, 3, 9),          # and of degree 3
])
def test_matches_oracle(n, L, p, seed):
    x, y, z, q = _uniform(n, seed)
    g = _gpu(x, y, z, q, p, L)
    o = oracle.fmm3(x, y, z, q, p, L)
    assert g[4] == o[4] == 0
    eg, ep = _rel(g, o)
    assert eg < 1e-12 and ep < 1e-12, (eg, ep)


def test_clustered_and_shifted_cube():
    rng = np.random.default_rng(20)
    n = 6000
    c = rng.random((5, 3)) * 0.6 + 0.2
    pick = rng.integers(0, 5, n)
    pts = c[pick] + 0.03 * rng.standard_normal((n, 3))
    pts = np.clip(pts, 0.0, 0.999999)
    origin, W = (-2.0, 1.5, 0.25), 3.0
    x, y, z = origin[0] + W * pts[:, 0], origin[1] + W * pts[:, 1], origin[2] + W * pts[:, 2]
    q = rng.uniform(-1, 1, n)
    g = _gpu(x, y, z, q, 7, 4, origin, W)
    o = oracle.fmm3(x, y, z, q, 7, 4, origin, W)
    eg, ep = _rel(g, o)
    assert eg < 1e-12 and ep < 1e-12, (eg, ep)


@pytest.mark.parametrize("L", [0, 1])
def test_no_far_field_is_the_plain_sum(L):
    x, y, z, q = _uniform(700, 30 + L)
    g = _gpu(x, y, z, q, 4, L)
    d = oracle.direct3(x, y, z, q)
    eg, ep = _rel(g, d)
    assert eg < 1e-13 and ep < 1e-13


def test_against_the_plain_sum():
    x, y, z, q = _uniform(8000, 40)
    d = oracle.direct3(x, y, z, q)
    errs = []
    for p in (3, 6, 9):
        errs.append(_rel(_gpu(x, y, z, q, p, 3), d))
    assert errs[0][0] > errs[1][0] > errs[2][0]
    assert errs[2][0] < 2e-5 and errs[2][1] < 2e-5, errs


def test_outside_nan_one_and_none():
    import torch
    import paper_0905_2637_amd as fm
    x, y, z, q = _uniform(1000, 50)
    x[3], y[10], z[20] = 1.0, -1e-9, np.nan
    g = _gpu(x, y, z, q, 5, 3, check=False)
    assert g[4] == 3
    for i in (3, 10, 20):
        assert g[0][i] == g[1][i] == g[2][i] == g[3][i] == 0.0
    keep = np.ones(1000, bool)
    keep[[3, 10, 20]] = False
    o = oracle.fmm3(x[keep], y[keep], z[keep], q[keep], 5, 3)
    eg, ep = _rel(tuple(a[keep] for a in g[:4]), o)
    assert eg < 1e-12 and ep < 1e-12
    with pytest.raises(fm.FmmError) as ei:
        _gpu(x, y, z, q, 5, 3, check=True)
    assert ei.value.status == fm.FMM_E_DOMAIN
    # one particle: nothing acts on it
    g1 = _gpu(np.array([0.3]), np.array([0.4]), np.array([0.5]), np.array([2.0]), 4, 3)
    assert g1[0][0] == g1[1][0] == g1[2][0] == g1[3][0] == 0.0
    # no particles; more than the capacity
    plan = fm.Plan3D(10, 4, 2)
    e = _dev(np.zeros(0))
    plan.evaluate(e, e, e, e)
    torch.cuda.synchronize()
    assert plan.out_of_domain() == 0
    big = _dev(np.full(11, 0.5))
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate(big, big, big, big)
    assert ei.value.status == fm.FMM_E_CAPACITY
    plan.close()


def test_million_particles_sampled():
    """2^20 uniform particles, depth 5 (about 32 per leaf), degree 6: 256
    sampled particles against the plain sum over all sources."""
    import torch
    import paper_0905_2637_amd as fm
    n = 1 << 20
    x, y, z, q = _uniform(n, 60)
    plan = fm.Plan3D(n, 6, 5)
    out = plan.evaluate(_dev(x), _dev(y), _dev(z), _dev(q), check=True)
    torch.cuda.synchronize()
    plan.close()
    g = [o.cpu().numpy() for o in out]
    t = np.random.default_rng(61).choice(n, 256, replace=False)
    d = oracle.direct3(x, y, z, q, targets=t)
    eg, ep = _rel(tuple(a[t] for a in g), d)
    assert eg < 1e-3 and ep < 1e-3, (eg, ep)
    assert np.all(np.isfinite(g[0]))


@pytest.mark.parametrize("L,clustered", [(3, False), (5, True), (0, False)])
def test_tree_bit_exact(L, clustered):
    import torch
    import paper_0905_2637_amd as fm
    rng = np.random.default_rng(70 + L)
    n = 20000
    if clustered:
        x, y, z = (np.clip(0.4 + 0.01 * rng.standard_normal(n), 0.0, 0.999) for _ in range(3))
    else:
        x, y, z = rng.random(n), rng.random(n), rng.random(n)
    x[5], y[77] = 1.0, np.nan                 # outside: keys 2^(3L), sorted last in input order
    q = rng.uniform(-1, 1, n)
    plan = fm.Plan3D(n, 4, L)
    plan.evaluate(_dev(x), _dev(y), _dev(z), _dev(q), check=False)
    torch.cuda.synchronize()
    keys, perm, ls = plan.dump(fm.DUMP_KEYS), plan.dump(fm.DUMP_PERM), plan.dump(fm.DUMP_LEAF_START)
    assert plan.out_of_domain() == 2
    plan.close()
    ko, po = oracle.leaf_keys3(x, y, z, L)
    assert np.array_equal(keys, ko)
    assert np.array_equal(perm, po)
    expect = np.searchsorted(ko[po].astype(np.int64), np.arange((1 << (3 * L)) + 1), side="left")
    assert np.array_equal(ls, expect.astype(np.int32))
    assert ls[-1] == n - 2
