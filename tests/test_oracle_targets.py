"""Pins of the oracle's evaluation at target points distinct from the sources
(eq. 1: the sum over sources at arbitrary points y), against what the
mathematics fixes:

* one source: the closed form gamma / (2 pi r) (1 - exp(-r^2 / 2 sigma^2)),
  perpendicular to the separation, at any point, and zero on top of it;
* the FMM at points converges to the split-kernel sum at those points (the
  sum it approximates) as p grows, and the split sum to the regularised one
  when the leaves are much wider than sigma;
* at the sources' own positions the sums equal the particle sums (a
  coincident source contributes nothing in both);
* points outside the square are counted.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def test_one_source_closed_form():
    sigma, gam = 0.05, 1.7
    tx = np.array([0.5, 0.61, 0.5, 0.43, 0.5])
    ty = np.array([0.5, 0.5, 0.32, 0.58, 0.5 + 1e-3])
    u, v = oracle.direct_at([0.5], [0.5], [gam], sigma, tx, ty)
    assert u[0] == 0.0 and v[0] == 0.0                   # on top of the source
    for t in range(1, len(tx)):
        dx, dy = tx[t] - 0.5, ty[t] - 0.5
        r2 = dx * dx + dy * dy
        speed = gam / (2 * math.pi * math.sqrt(r2)) * -math.expm1(-r2 / (2 * sigma * sigma))
        # counter-clockwise for gamma > 0: (u, v) = speed (-dy, dx) / r
        assert abs(u[t] + speed * dy / math.sqrt(r2)) < 1e-14 * speed
        assert abs(v[t] - speed * dx / math.sqrt(r2)) < 1e-14 * speed


def test_fmm_at_points_converges_to_split_sum():
    x, y, g = workloads.uniform_square(2500, 41)
    rng = np.random.default_rng(42)
    tx, ty = rng.random(400), rng.random(400)
    us, vs = oracle.direct_split_at(x, y, g, 0.004, 4, tx, ty)
    err = []
    for p in (8, 16, 40):
        u, v, nbad = oracle.fmm_at(x, y, g, 0.004, p, 4, tx, ty)
        assert nbad == 0
        err.append(oracle.rel_l2(u, v, us, vs))
    assert err[2] < 1e-13 and err[0] > err[1] > err[2], err
    ud, vd = oracle.direct_at(x, y, g, 0.004, tx, ty)
    assert oracle.rel_l2(us, vs, ud, vd) < 1e-10         # leaves are 15 sigma wide


def test_points_at_the_sources_equal_the_particle_sums():
    x, y, g = workloads.uniform_square(1500, 43)
    u1, v1 = oracle.fmm(x, y, g, 0.01, 17, 4)
    u2, v2, _ = oracle.fmm_at(x, y, g, 0.01, 17, 4, x, y)
    assert np.array_equal(u1, u2) and np.array_equal(v1, v2)
    d1 = oracle.direct(x, y, g, 0.01)
    d2 = oracle.direct_at(x, y, g, 0.01, x, y)
    assert np.array_equal(d1[0], d2[0]) and np.array_equal(d1[1], d2[1])


def test_points_outside_are_counted():
    x, y, g = workloads.uniform_square(300, 44)
    tx = np.array([0.5, 1.5, -0.1, 0.2])
    ty = np.array([0.5, 0.5, 0.3, 2.0])
    _, _, nbad = oracle.fmm_at(x, y, g, 0.01, 12, 3, tx, ty)
    assert nbad == 3
