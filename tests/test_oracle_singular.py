"""Pins of the oracle's singular kernel (eq. 7, point vortices; sigma = 0),
against what the mathematics fixes:

* two point vortices: the closed form gamma / (2 pi r), perpendicular to the
  separation;
* N equal point vortices on a circle (Kelvin's polygon) all move along the
  circle with speed (N - 1) gamma / (4 pi R), the classical closed form of
  the rotating polygon; the direct sum and the FMM both reproduce it;
* where every pair is further apart than 9 sigma, the Gaussian factor
  1 - exp(-r^2 / 2 sigma^2) rounds to 1 and the regularised sum equals the
  singular one bit for bit (the sigma -> 0 limit, reached through the
  regularised code path);
* the singular FMM converges to the singular direct sum as p grows (no
  split-kernel gap: near and far pairs use the same kernel), at particles
  and at target points.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def test_two_point_vortices():
    gam = 0.8
    x, y, g = np.array([0.3, 0.55]), np.array([0.4, 0.47]), np.array([gam, -2.0 * gam])
    u, v = oracle.direct(x, y, g, 0.0)
    dx, dy = x[0] - x[1], y[0] - y[1]
    r = math.hypot(dx, dy)
    speed = g[1] / (2 * math.pi * r)          # induced on particle 0 by particle 1
    assert abs(u[0] + speed * dy / r) < 1e-14 * abs(speed)
    assert abs(v[0] - speed * dx / r) < 1e-14 * abs(speed)
    assert u[1] * g[1] == pytest.approx(-u[0] * g[0], rel=1e-14)   # net force vanishes


@pytest.mark.parametrize("N", [3, 7, 12])
def test_kelvin_polygon(N):
    gam, R, c = 0.37, 0.3, (0.5, 0.5)
    th = 2 * math.pi * np.arange(N) / N + 0.1
    x, y = c[0] + R * np.cos(th), c[1] + R * np.sin(th)
    g = np.full(N, gam)
    speed = (N - 1) * gam / (4 * math.pi * R)
    tu, tv = -np.sin(th), np.cos(th)           # counter-clockwise tangent
    u, v = oracle.direct(x, y, g, 0.0)
    assert np.max(np.abs(u - speed * tu)) < 1e-14 and np.max(np.abs(v - speed * tv)) < 1e-14
    uf, vf = oracle.fmm(x, y, g, 0.0, 40, 3)
    assert np.max(np.abs(uf - speed * tu)) < 1e-13 and np.max(np.abs(vf - speed * tv)) < 1e-13


def test_gaussian_limit_equals_singular():
    x, y, g = workloads.uniform_square(300, 61)
    d2 = (x[:, None] - x[None, :]) ** 2 + (y[:, None] - y[None, :]) ** 2
    dmin = math.sqrt(d2[~np.eye(300, dtype=bool)].min())
    sigma = dmin / 10.0                        # r^2 / 2 sigma^2 >= 50 for every pair
    ur, vr = oracle.direct(x, y, g, sigma)
    us, vs = oracle.direct(x, y, g, 0.0)
    assert np.array_equal(ur, us) and np.array_equal(vr, vs)


def test_singular_fmm_converges_to_the_direct_sum():
    x, y, g = workloads.uniform_square(2000, 62)
    ud, vd = oracle.direct(x, y, g, 0.0)
    err = [oracle.rel_l2(*oracle.fmm(x, y, g, 0.0, p, 4), ud, vd) for p in (6, 12, 24, 40)]
    assert err[0] > err[1] > err[2] > err[3] and err[3] < 1e-13, err
    rng = np.random.default_rng(63)
    tx, ty = rng.random(300), rng.random(300)
    ua, va = oracle.direct_at(x, y, g, 0.0, tx, ty)
    u40, v40, _ = oracle.fmm_at(x, y, g, 0.0, 40, 4, tx, ty)
    assert oracle.rel_l2(u40, v40, ua, va) < 1e-13
    # the split sum with the singular kernel is the singular sum
    us, vs = oracle.direct_split(x, y, g, 0.0, 4)
    assert np.array_equal(us, ud) and np.array_equal(vs, vd)


def test_polygon_rotates_rigidly_under_time_stepping():
    """Kelvin's polygon turns with angular velocity (N - 1) gamma / (4 pi R^2);
    the midpoint rule's position error falls fourfold when dt halves."""
    N, gam, R, T = 6, 0.37, 0.3, 1.0
    omega = (N - 1) * gam / (4 * math.pi * R * R)
    th = 2 * math.pi * np.arange(N) / N + 0.1
    errs = []
    for steps in (25, 50):
        x, y = oracle.advance_rk2(0.5 + R * np.cos(th), 0.5 + R * np.sin(th), np.full(N, gam), 0.0, T / steps,
                                  steps, p=32, L=3, velocity="fmm")
        errs.append(float(np.max(np.hypot(x - 0.5 - R * np.cos(th + omega * T),
                                          y - 0.5 - R * np.sin(th + omega * T)))))
    assert errs[0] < 1e-3 and 3.8 < errs[0] / errs[1] < 4.2, errs
