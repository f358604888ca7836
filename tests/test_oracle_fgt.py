"""Pins of the oracle's Gauss transform (a transform Section 8 names), plain
and fast (Greengard and Strain's Hermite / Taylor algorithm), against what
the mathematics fixes:

* Hermite functions: h_n(t) = H_n(t) exp(-t^2) with the closed-form Hermite
  polynomials H_0..H_4, the generating identity exp(-(t - s)^2) =
  sum_n s^n / n! h_n(t), and h_n' = -h_{n+1};
* the plain sum: one source seen from a target, and the self term;
* the fast form converges to the plain sum as p grows (down to 1e-14), and
  leaving out boxes beyond nc costs no more than the Gaussian's tail
  exp(-(nc w)^2 / delta) allows.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def test_hermite_functions():
    for t in (-1.3, -0.2, 0.0, 0.45, 2.1):
        h = oracle.hermite(5, t)
        e = math.exp(-t * t)
        H = [1.0, 2 * t, 4 * t * t - 2, 8 * t ** 3 - 12 * t, 16 * t ** 4 - 48 * t * t + 12]
        for n in range(5):
            assert h[n] == pytest.approx(H[n] * e, rel=1e-14, abs=1e-15)
        # generating identity, |s| <= 1/2
        for s in (-0.5, 0.17, 0.5):
            hh = oracle.hermite(40, t)
            series = sum(s ** n / math.factorial(n) * hh[n] for n in range(40))
            assert series == pytest.approx(math.exp(-(t - s) ** 2), rel=1e-13, abs=1e-15)
        # h_n' = -h_{n+1} (central differences)
        d = 1e-6
        hp, hm, h2 = oracle.hermite(8, t + d), oracle.hermite(8, t - d), oracle.hermite(9, t)
        for n in range(8):
            assert (hp[n] - hm[n]) / (2 * d) == pytest.approx(-h2[n + 1], rel=1e-7, abs=1e-8)


def test_plain_sum_closed_forms():
    sigma = 0.07
    x, y, q = np.array([0.3, 0.41]), np.array([0.6, 0.52]), np.array([1.5, -0.4])
    G = oracle.gauss_direct(x, y, q, sigma)
    r2 = (0.41 - 0.3) ** 2 + (0.52 - 0.6) ** 2
    e = math.exp(-r2 / (2 * sigma * sigma))
    assert G[0] == pytest.approx(1.5 + (-0.4) * e, rel=1e-15)      # self term included
    assert G[1] == pytest.approx(-0.4 + 1.5 * e, rel=1e-15)


def test_fast_form_converges_to_the_plain_sum():
    x, y, q = workloads.uniform_square(4000, 92)
    sigma, L = 0.05, 5
    Gd = oracle.gauss_direct(x, y, q, sigma)
    sd = math.sqrt(2) * sigma
    nc = math.ceil(math.sqrt(36.8) * sd / 2 ** -L)
    err = []
    for p in (4, 8, 12, 16):
        G, nbad = oracle.fgt(x, y, q, sigma, p, L, nc)
        assert nbad == 0
        err.append(np.linalg.norm(G - Gd) / np.linalg.norm(Gd))
    assert err[0] > err[1] > err[2] > err[3] and err[3] < 1e-14, err


def test_range_truncation_within_the_tail_bound():
    x, y, q = workloads.uniform_square(3000, 93)
    sigma, L, p = 0.04, 5, 14
    w = 2.0 ** -L
    delta = 2 * sigma * sigma
    Gd = oracle.gauss_direct(x, y, q, sigma)
    full, _ = oracle.fgt(x, y, q, sigma, p, L, 14)
    floor = np.max(np.abs(full - Gd))
    for nc in (2, 3, 4):
        G, _ = oracle.fgt(x, y, q, sigma, p, L, nc)
        # every left-out source lies at least nc w away (Chebyshev box distance nc + 1)
        bound = np.sum(np.abs(q)) * math.exp(-(nc * w) ** 2 / delta)
        assert np.max(np.abs(G - Gd)) <= bound + floor
    G2, _ = oracle.fgt(x, y, q, sigma, p, L, 2)
    assert np.max(np.abs(G2 - Gd)) > 10 * floor          # the truncation shows


def test_fast_form_at_points():
    """At points apart from the particles: convergence to the plain sum, and
    points on top of the particles reproduce the particle evaluation bit for
    bit (the same boxes, expansions and Taylor sums)."""
    x, y, q = workloads.uniform_square(3000, 94)
    rng = np.random.default_rng(95)
    tx, ty = rng.random(500), rng.random(500)
    sigma, L, p = 0.05, 5, 16
    nc = math.ceil(math.sqrt(36.8) * math.sqrt(2) * sigma / 2 ** -L)
    G, nbad = oracle.fgt_at(x, y, q, sigma, p, L, nc, tx, ty)
    Gd = oracle.gauss_direct_at(x, y, q, sigma, tx, ty)
    assert nbad == 0 and np.linalg.norm(G - Gd) / np.linalg.norm(Gd) < 1e-14
    G1, _ = oracle.fgt(x, y, q, sigma, 12, L, nc)
    G2, _ = oracle.fgt_at(x, y, q, sigma, 12, L, nc, x, y)
    assert np.array_equal(G1, G2)
    Gp = oracle.gauss_direct(x, y, q, sigma)
    Gpa = oracle.gauss_direct_at(x, y, q, sigma, x, y)
    assert np.allclose(Gp, Gpa, rtol=1e-14, atol=0)
