"""Pins of the oracle's 3D form (Laplace kernel 1/r, Cartesian Taylor
expansions of total degree <= p on a uniform octree; the 3D extension
Section 8 describes: same tree and sweeps, a new kernel and expansions).

Each operator is checked against something other than itself:
* derivatives of 1/r: closed forms up to third order, central differences
  of the next lower order, and the Laplace equation at every order;
* the plain sum: two charges, the eight corners of a cube (closed form),
  Newton's third law, and the target subset;
* P2M / multipole evaluation and M2L / L2P: convergence to the plain sum at
  the rate the separation ratio sets;
* M2M and L2L: exact re-expansions of polynomials (the shift of a truncated
  Taylor series is exact), so they agree with P2M about the new centre and
  with the unshifted local evaluation to rounding;
* the whole FMM: equal to the plain sum when every leaf is near (depth <= 1),
  converging to it as p grows, brute force on a tiny case, and particles
  outside the cube counted and left out;
* Morton keys against a bit-by-bit interleave.
"""
import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _rng(seed):
    return np.random.default_rng(seed)


def test_derivatives_closed_forms():
    for seed in range(5):
        R = _rng(seed).uniform(-2, 2, 3)
        x, y, z = R
        r = np.linalg.norm(R)
        D = oracle.deriv3(3, R)
        assert D[0, 0, 0] == pytest.approx(1 / r, rel=1e-15)
        assert D[1, 0, 0] == pytest.approx(-x / r ** 3, rel=1e-14)
        assert D[0, 0, 1] == pytest.approx(-z / r ** 3, rel=1e-14)
        assert D[2, 0, 0] == pytest.approx((3 * x * x - r * r) / r ** 5, rel=1e-13, abs=1e-14 / r ** 3)
        assert D[1, 1, 0] == pytest.approx(3 * x * y / r ** 5, rel=1e-13)
        assert D[0, 1, 1] == pytest.approx(3 * y * z / r ** 5, rel=1e-13)
        assert D[1, 1, 1] == pytest.approx(-15 * x * y * z / r ** 7, rel=1e-13)
        assert D[3, 0, 0] == pytest.approx(-(15 * x ** 3 - 9 * x * r * r) / r ** 7, rel=1e-12)


def test_derivatives_laplace_and_finite_differences():
    q = 12
    for seed in range(4):
        R = _rng(10 + seed).uniform(0.5, 1.5, 3) * _rng(20 + seed).choice([-1, 1], 3)
        D = oracle.deriv3(q, R)
        # harmonic: sum_i D_(m + 2 e_i) = 0 for every |m| <= q - 2
        for a in range(q - 1):
            for b in range(q - 1 - a):
                for c in range(q - 1 - a - b):
                    lap = D[a + 2, b, c] + D[a, b + 2, c] + D[a, b, c + 2]
                    scale = abs(D[a + 2, b, c]) + abs(D[a, b + 2, c]) + abs(D[a, b, c + 2])
                    assert abs(lap) <= 1e-12 * scale
        # central differences of order |m| give order |m| + 1
        h = 1e-5
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            Dp, Dm = oracle.deriv3(q - 1, R + e), oracle.deriv3(q - 1, R - e)
            for a in range(q - 1):
                for b in range(q - 1 - a):
                    for c in range(q - 1 - a - b):
                        m = [a, b, c]
                        up = list(m)
                        up[i] += 1
                        fd = (Dp[a, b, c] - Dm[a, b, c]) / (2 * h)
                        ex = D[tuple(up)]
                        assert fd == pytest.approx(ex, rel=1e-5, abs=1e-7 * max(1.0, abs(D).max()))


def test_direct_closed_forms():
    # two charges
    x, y, z = np.array([0.1, 0.4]), np.array([0.2, 0.6]), np.array([0.3, 0.3])
    q = np.array([2.0, -1.5])
    phi, gx, gy, gz = oracle.direct3(x, y, z, q)
    d = np.array([0.3, 0.4, 0.0])
    assert phi[0] == pytest.approx(-1.5 / 0.5, rel=1e-15)
    assert phi[1] == pytest.approx(2.0 / 0.5, rel=1e-15)
    # gradient at particle 0 from particle 1: -q1 (x0 - x1) / r^3
    assert gx[0] == pytest.approx(1.5 * (-d[0]) / 0.125, rel=1e-14)
    assert gy[0] == pytest.approx(1.5 * (-d[1]) / 0.125, rel=1e-14)
    assert gz[0] == 0.0
    # eight unit charges on the corners of a cube of side a
    a = 0.25
    cx, cy, cz = (np.array([(i >> k) & 1 for i in range(8)], float) * a for k in range(3))
    phi, gx, gy, gz = oracle.direct3(cx, cy, cz, np.ones(8))
    expect = 3 / a + 3 / (a * math.sqrt(2)) + 1 / (a * math.sqrt(3))
    assert np.allclose(phi, expect, rtol=1e-15)
    # the field at a corner points along the body diagonal, outward
    for i in range(8):
        g = np.array([gx[i], gy[i], gz[i]])
        out = np.array([cx[i], cy[i], cz[i]]) - a / 2
        assert np.allclose(np.cross(g, out), 0, atol=1e-12 * np.linalg.norm(g))
        assert g @ out < 0          # grad phi points inward: phi decreases outward


def test_direct_newton_and_targets():
    rng = _rng(3)
    n = 400
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    q = rng.uniform(-1, 1, n)
    phi, gx, gy, gz = oracle.direct3(x, y, z, q)
    scale = np.abs(q * gx).sum()
    assert abs((q * gx).sum()) < 1e-13 * scale
    assert abs((q * gy).sum()) < 1e-13 * scale
    assert abs((q * gz).sum()) < 1e-13 * scale
    t = np.array([5, 0, 399, 17])
    sub = oracle.direct3(x, y, z, q, targets=t)
    for a, b in zip(sub, (phi, gx, gy, gz)):
        assert np.array_equal(a, b[t])


def _cluster(seed, n, c, rad):
    rng = _rng(seed)
    return (c[0] + rng.uniform(-rad, rad, n), c[1] + rng.uniform(-rad, rad, n),
            c[2] + rng.uniform(-rad, rad, n), rng.uniform(-1, 1, n))


def test_p2m_and_multipole_convergence():
    c = np.array([0.5, 0.5, 0.5])
    x, y, z, q = _cluster(4, 50, c, 0.1)
    M = oracle.p2m3(x, y, z, q, c, 0)
    assert M[0] == pytest.approx(q.sum(), rel=1e-14)
    X = np.array([[1.3, 0.6, 0.2]])
    ex = oracle.direct3(np.r_[x, X[:, 0]], np.r_[y, X[:, 1]], np.r_[z, X[:, 2]], np.r_[q, 0.0],
                        targets=[len(x)])[0][0]
    ratio = 0.1 * math.sqrt(3) / np.linalg.norm(X[0] - c)
    errs = []
    for p in (2, 4, 6, 8, 10):
        M = oracle.p2m3(x, y, z, q, c, p)
        errs.append(abs(oracle.me_eval3(M, p, X[0] - c) - ex))
        assert errs[-1] <= 4 * np.abs(q).sum() / np.linalg.norm(X[0] - c) * ratio ** (p + 1)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_m2m_is_exact():
    p = 8
    c = np.array([0.4, 0.45, 0.5])
    x, y, z, q = _cluster(5, 30, c, 0.05)
    for d in ([0.05, -0.05, 0.05], [-0.125, 0.125, 0.125]):
        M1 = oracle.m2m3(oracle.p2m3(x, y, z, q, c, p), p, d)
        M2 = oracle.p2m3(x, y, z, q, c + np.array(d), p)
        assert np.allclose(M1, M2, rtol=1e-12, atol=1e-14 * np.abs(M2).max())


def test_l2l_is_exact():
    p = 7
    rng = _rng(6)
    Lc = np.zeros((p + 1) ** 3)
    for a in range(p + 1):
        for b in range(p + 1 - a):
            for c in range(p + 1 - a - b):
                Lc[(a * (p + 1) + b) * (p + 1) + c] = rng.uniform(-1, 1)
    d = np.array([0.03, -0.02, 0.05])
    L2 = oracle.l2l3(Lc, p, d)
    for _ in range(5):
        e = rng.uniform(-0.1, 0.1, 3)
        assert np.allclose(oracle.l2p3(Lc, p, e), oracle.l2p3(L2, p, e - d), rtol=1e-12, atol=1e-13)


def test_m2l_l2p_convergence():
    """Source cluster about s, target point near t, |t - s| = 2 box widths (the
    nearest interaction-list separation): the error falls with p."""
    s = np.array([0.25, 0.25, 0.25])
    t = np.array([0.75, 0.25, 0.25])
    w = 0.25
    x, y, z, q = _cluster(7, 40, s, w / 2)
    e = np.array([0.1, -0.1, 0.08])
    X = t + e
    allx, ally, allz = np.r_[x, X[0]], np.r_[y, X[1]], np.r_[z, X[2]]
    ex = np.array([a[0] for a in oracle.direct3(allx, ally, allz, np.r_[q, 0.0], targets=[len(x)])])
    errs = []
    for p in (2, 4, 6, 8, 10, 12):
        Lc = oracle.m2l3(oracle.p2m3(x, y, z, q, s, p), p, t - s)
        got = oracle.l2p3(Lc, p, e)
        errs.append(np.abs(got - ex).max() / np.abs(ex).max())
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


def test_morton3_interleave():
    for a, b, c in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (5, 3, 6), (127, 0, 127), (1023, 1023, 1023)]:
        k = 0
        for i in range(10):
            k |= ((a >> i) & 1) << (3 * i) | ((b >> i) & 1) << (3 * i + 1) | ((c >> i) & 1) << (3 * i + 2)
        assert oracle.morton3(a, b, c) == k


def test_fmm3_depth_le_1_is_direct():
    rng = _rng(8)
    n = 300
    x, y, z, q = rng.random(n), rng.random(n), rng.random(n), rng.uniform(-1, 1, n)
    ex = oracle.direct3(x, y, z, q)
    for L in (0, 1):
        got = oracle.fmm3(x, y, z, q, 4, L)
        assert got[4] == 0
        for a, b in zip(got[:4], ex):
            assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


def _rel(got, ex):
    num = sum(np.sum((a - b) ** 2) for a, b in zip(got[1:4], ex[1:4]))
    den = sum(np.sum(b ** 2) for b in ex[1:4])
    return math.sqrt(num / den), np.linalg.norm(got[0] - ex[0]) / np.linalg.norm(ex[0])


def test_fmm3_converges_to_direct():
    rng = _rng(9)
    n = 3000
    x, y, z, q = rng.random(n), rng.random(n), rng.random(n), rng.uniform(-1, 1, n)
    ex = oracle.direct3(x, y, z, q)
    errs = []
    for p in (1, 3, 5, 7, 9):
        got = oracle.fmm3(x, y, z, q, p, 3)
        errs.append(_rel(got, ex))
    assert all(b[0] < a[0] and b[1] < a[1] for a, b in zip(errs, errs[1:])), errs
    assert errs[-1][0] < 1e-4 and errs[-1][1] < 1e-5, errs


def test_fmm3_brute_force_tiny_and_outside():
    """Depth 2 with four charges: the far part is one M2L per pair, checked
    against the truncated expansions built by hand from the operators."""
    x = np.array([0.1, 0.9, 0.12, 0.6, 1.2, np.nan])
    y = np.array([0.1, 0.9, 0.15, 0.1, 0.5, 0.5])
    z = np.array([0.1, 0.9, 0.11, 0.9, 0.5, 0.5])
    q = np.array([1.0, -2.0, 0.5, 0.7, 3.0, 3.0])
    p, L = 6, 2
    phi, gx, gy, gz, nbad = oracle.fmm3(x, y, z, q, p, L)
    assert nbad == 2
    assert phi[4] == phi[5] == gx[4] == gz[5] == 0.0
    w = 0.25
    box = np.floor(np.c_[x[:4], y[:4], z[:4]] / w).astype(int)
    cen = (box + 0.5) * w
    for i in range(4):
        out = np.zeros(4)
        for j in range(4):
            if j == i:
                continue
            d = box[i] - box[j]
            if np.abs(d).max() <= 1:            # near: plain pair
                r = np.array([x[i] - x[j], y[i] - y[j], z[i] - z[j]])
                rn = np.linalg.norm(r)
                out += [q[j] / rn, *(-q[j] * r / rn ** 3)]
            else:                               # all level-2 pairs here are well separated
                assert np.abs(d // 1).max() >= 2
                M = oracle.p2m3(x[j:j + 1], y[j:j + 1], z[j:j + 1], q[j:j + 1], cen[j], p)
                Lc = oracle.m2l3(M, p, cen[i] - cen[j])
                out += oracle.l2p3(Lc, p, np.array([x[i], y[i], z[i]]) - cen[i])
        assert np.allclose([phi[i], gx[i], gy[i], gz[i]], out, rtol=1e-13, atol=1e-13)


def test_leaf_keys3_order():
    rng = _rng(11)
    n = 500
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    x[7] = 1.0                                   # on the far face: outside [0, 1)
    keys, perm = oracle.leaf_keys3(x, y, z, 3)
    assert keys[7] == 1 << 9
    assert perm[-1] == 7
    assert np.all(np.diff(keys[perm].astype(np.int64)) >= 0)
    a, b, c = (np.floor(v * 8).astype(int) for v in (x, y, z))
    for i in (0, 1, 100):
        assert keys[i] == oracle.morton3(a[i], b[i], c[i])
