"""Pins of the oracle's vortex-method time stepping (Section 3, eq. 6: the
particles move with their velocity and keep their circulation), against what
the mathematics fixes rather than against the oracle itself:

* two equal vortices rotate rigidly about their midpoint with the angular
  velocity of the regularised kernel (eq. 8), Omega = g (1 - exp(-d^2 / 2
  sigma^2)) / (pi d^2); the midpoint rule converges to that motion at second
  order in dt;
* the vorticity centroid sum(g x) / sum(g) is an exact invariant of any
  Runge-Kutta step whenever sum(g u) = 0, which holds to rounding for the
  direct sum (the kernel is odd) and for the FMM (its far field is
  antisymmetric), so it is conserved to rounding;
* the angular impulse I = sum(g |z|^2) has dI/dt = 2 sum(g (x u + y v)),
  a double sum whose terms cancel pairwise (the kernel is odd and radial),
  so the direct sum's rate is zero to rounding and the FMM's to its
  truncation error; the midpoint rule's drift of I over a fixed time falls
  at least at second order in dt.
"""
import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _pair_error(dt, T=0.2, d=0.2, sigma=0.02, g=1.0):
    x = np.array([0.5 - d / 2, 0.5 + d / 2])
    y = np.array([0.5, 0.5])
    steps = int(round(T / dt))
    xn, yn = oracle.advance_rk2(x, y, np.array([g, g]), sigma, dt, steps, velocity="direct")
    omega = g * (1.0 - math.exp(-d * d / (2 * sigma * sigma))) / (math.pi * d * d)
    ang = omega * steps * dt                          # counter-clockwise for g > 0
    ex = 0.5 + (x - 0.5) * math.cos(ang) - (y - 0.5) * math.sin(ang)
    ey = 0.5 + (x - 0.5) * math.sin(ang) + (y - 0.5) * math.cos(ang)
    return float(np.max(np.hypot(xn - ex, yn - ey)))


def test_two_vortices_rotate_at_second_order():
    e1 = _pair_error(0.01)
    e2 = _pair_error(0.005)
    e3 = _pair_error(0.0025)
    assert e1 < 1e-3
    for a, b in ((e1, e2), (e2, e3)):
        assert 3.5 < a / b < 4.5, (e1, e2, e3)


@pytest.mark.parametrize("velocity", ["direct", "fmm"])
def test_vorticity_centroid_is_conserved(velocity):
    rng = np.random.default_rng(31)
    n = 400
    x = 0.2 + 0.6 * rng.random(n)
    y = 0.2 + 0.6 * rng.random(n)
    g = rng.uniform(0.2, 1.0, n)                      # one sign: the centroid is well defined
    cx0, cy0 = np.sum(g * x) / np.sum(g), np.sum(g * y) / np.sum(g)
    xn, yn = oracle.advance_rk2(x, y, g, 0.01, 2e-3, 5, p=16, L=3, velocity=velocity)
    cx1, cy1 = np.sum(g * xn) / np.sum(g), np.sum(g * yn) / np.sum(g)
    moved = float(np.max(np.hypot(xn - x, yn - y)))
    assert moved > 1e-4                               # the particles did move
    assert abs(cx1 - cx0) < 1e-14 and abs(cy1 - cy0) < 1e-14, (cx1 - cx0, cy1 - cy0)


def test_fmm_stepping_follows_direct_stepping():
    """With leaves much wider than sigma the split kernel equals the
    regularised one to rounding, so FMM-driven steps follow direct-sum steps
    to the expansion's truncation error."""
    rng = np.random.default_rng(32)
    n = 500
    x, y = rng.random(n), rng.random(n)
    g = rng.uniform(-1, 1, n)
    xa, ya = oracle.advance_rk2(x, y, g, 0.004, 1e-3, 3, p=24, L=3, velocity="fmm")
    xb, yb = oracle.advance_rk2(x, y, g, 0.004, 1e-3, 3, velocity="direct")
    assert float(np.max(np.hypot(xa - xb, ya - yb))) < 1e-10


def _angular_set():
    rng = np.random.default_rng(7)
    n = 40
    x = 0.4 + 0.2 * rng.random(n)
    y = 0.4 + 0.2 * rng.random(n)
    g = 0.01 * rng.uniform(-1.0, 1.0, n)
    return x, y, g


def test_angular_impulse_rate_vanishes():
    x, y, g = _angular_set()
    u, v = oracle.direct(x, y, g, 0.01)
    scale = np.sum(np.abs(g) * (np.abs(x * u) + np.abs(y * v)))
    assert abs(np.sum(g * (x * u + y * v))) < 1e-14 * scale
    uf, vf = oracle.fmm(x, y, g, 0.01, 20, 2, *oracle.bounding_square(x, y))
    assert abs(np.sum(g * (x * uf + y * vf))) < 1e-9 * scale


def test_angular_impulse_drift_falls_with_dt():
    x, y, g = _angular_set()
    i0 = np.sum(g * (x * x + y * y))
    scale = np.sum(np.abs(g) * (x * x + y * y))
    drift = []
    for dt in (4e-3, 2e-3, 1e-3):
        xn, yn = oracle.advance_rk2(x, y, g, 0.01, dt, int(round(0.4 / dt)), velocity="direct")
        assert float(np.max(np.hypot(xn - x, yn - y))) > 0.05       # a real rotation of the set
        drift.append(abs(np.sum(g * (xn * xn + yn * yn)) - i0) / scale)
    assert drift[0] < 1e-8, drift
    assert drift[0] / drift[1] > 3.5 and drift[1] / drift[2] > 3.5, drift
