"""Pins of the oracle's Lennard-Jones sums (the molecular-dynamics kernel
Section 8 names), against what the potential's definition fixes:

* two particles: no force at the potential's minimum r = 2^(1/6) s, where the
  energy is -eps; repulsion 24 eps / s at r = s; the energy 4 eps (s^12/r^12
  - s^6/r^6) at other separations; nothing beyond the cutoff;
* Newton's third law: the forces sum to zero;
* the force is minus the gradient of the total energy (central differences);
* the centre particle of a symmetric square lattice feels no net force.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def test_pair_closed_forms():
    eps, s, rc = 0.7, 0.01, 0.03
    rmin = 2 ** (1 / 6) * s
    fx, fy = oracle.lj_forces([0.5, 0.5 + rmin], [0.5, 0.5], eps, s, rc)
    assert abs(fx[0]) < 1e-9 * 24 * eps / s and fy[0] == 0.0
    assert oracle.lj_energy([0.5, 0.5 + rmin], [0.5, 0.5], eps, s, rc) == pytest.approx(-eps, rel=1e-14)
    d = s / math.sqrt(2)                        # separation s along the diagonal
    fx, fy = oracle.lj_forces([0.4, 0.4 + d], [0.4, 0.4 + d], eps, s, rc)
    assert fx[0] == pytest.approx(-24 * eps / s / math.sqrt(2), rel=1e-13)      # pushed away from the other
    assert fy[0] == pytest.approx(-24 * eps / s / math.sqrt(2), rel=1e-13)
    assert fx[1] == pytest.approx(24 * eps / s / math.sqrt(2), rel=1e-13)
    r = 1.7 * s
    assert oracle.lj_energy([0.0, r], [0.0, 0.0], eps, s, rc) == pytest.approx(
        4 * eps * ((s / r) ** 12 - (s / r) ** 6), rel=1e-14)
    fx, fy = oracle.lj_forces([0.0, rc * (1 + 1e-12)], [0.0, 0.0], eps, s, rc)
    assert fx[0] == 0.0 and oracle.lj_energy([0.0, rc * (1 + 1e-12)], [0.0, 0.0], eps, s, rc) == 0.0
    fx, fy = oracle.lj_forces([0.0, rc * (1 - 1e-12)], [0.0, 0.0], eps, s, rc)
    assert fx[0] != 0.0


def test_newton_third_law_and_gradient():
    rng = np.random.default_rng(71)
    n, eps, s, rc = 400, 1.0, 0.01, 0.025
    # a jittered lattice keeps every pair beyond 0.8 s
    g = np.arange(20) * 0.012
    X, Y = np.meshgrid(g, g)
    x = X.ravel() + rng.uniform(-0.001, 0.001, n)
    y = Y.ravel() + rng.uniform(-0.001, 0.001, n)
    fx, fy = oracle.lj_forces(x, y, eps, s, rc)
    scale = np.max(np.hypot(fx, fy))
    assert abs(fx.sum()) < 1e-12 * scale * n and abs(fy.sum()) < 1e-12 * scale * n
    h = 1e-7
    for i in (0, 57, 210, 399):
        for arr, f in ((x, fx), (y, fy)):
            a0 = arr[i]
            arr[i] = a0 + h
            ep = oracle.lj_energy(x, y, eps, s, rc)
            arr[i] = a0 - h
            em = oracle.lj_energy(x, y, eps, s, rc)
            arr[i] = a0
            assert (em - ep) / (2 * h) == pytest.approx(f[i], rel=1e-5, abs=1e-6 * scale)


def test_symmetric_lattice_centre_feels_nothing():
    a, m = 0.011, 9
    g = (np.arange(m) - m // 2) * a + 0.5
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    c = (m * m) // 2
    fx, fy = oracle.lj_forces(x, y, 1.0, 0.01, 0.035, targets=[c])
    ex, _ = oracle.lj_forces(x, y, 1.0, 0.01, 0.035, targets=[c + m // 2])   # on the lattice's edge
    assert abs(ex[0]) > 1.0
    assert abs(fx[0]) < 1e-12 * abs(ex[0]) and abs(fy[0]) < 1e-12 * abs(ex[0])
