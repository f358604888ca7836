"""The fast Gauss transform on the GPU (FMM_KERNEL_GAUSS_TRANSFORM): the
Hermite expansions of the leaf boxes, their Hermite-to-Taylor translation
between boxes within the range nc, and the Taylor evaluation at the
particles.

* FP64 parity with the oracle's fast transform (the same algorithm, p and
  range) within 1e-12, for expansion sizes 8-16 (with and without padding
  of the compiled size), depths 0-5, uniform and clustered particles;
* against the plain sum: 1e-13 where p and the box size allow it;
* at target points apart from the particles (and on top of them, where
  they reproduce the particle evaluation bit for bit);
* one particle (its own term only), no particles, and the unsupported
  combinations.
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


def _range(sigma, L):
    """The library's box range: nc = ceil(sqrt(ln 1e16) sqrt(2) sigma / w),
    at most 2^L - 1."""
    return int(min(math.ceil(math.sqrt(math.log(1e16)) * math.sqrt(2.0) * sigma / math.ldexp(1.0, -L)),
                   max((1 << L) - 1, 0)))


def _gpu(x, y, q, sigma, p, L):
    import torch
    import paper_0905_2637_amd as fm
    plan = fm.Plan(len(x), sigma, p, L, kernel="gauss-transform")
    G, v = plan.evaluate(_dev(x), _dev(y), _dev(q), check=True)
    torch.cuda.synchronize()
    plan.close()
    assert not v.cpu().numpy().any()
    return G.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,sigma,L,p", [
    (5000, 0.05, 5, 12),
    (3000, 0.05, 4, 8),
    (3000, 0.03, 5, 10),      # padded to the compiled size 12
    (2000, 0.06, 4, 16),
    (700, 0.2, 2, 12),
    (500, 0.3, 0, 8),         # one box: nc = 0, tau = 0 only
])
def test_fgt_matches_oracle(n, sigma, L, p):
    x, y, q = workloads.uniform_square(n, 900 + n)
    G = _gpu(x, y, q, sigma, p, L)
    Go, nbad = oracle.fgt(x, y, q, sigma, p, L, _range(sigma, L))
    assert nbad == 0
    err = _rel(G, Go)
    assert err < 1e-12, f"rel L2 vs the oracle's fast transform {err:.3e}"


def test_fgt_clustered_and_against_the_plain_sum():
    x, y, q, _, _ = workloads.gaussian_mixture(6000, 5, 910)
    sigma, L, p = 0.04, 5, 16
    G = _gpu(x, y, q, sigma, p, L)
    Go, _ = oracle.fgt(x, y, q, sigma, p, L, _range(sigma, L))
    assert _rel(G, Go) < 1e-12
    Gd = oracle.gauss_direct(x, y, q, sigma)
    assert _rel(G, Gd) < 1e-13


def test_fgt_at_points():
    """The transform at points apart from the particles: parity with the
    oracle's fast form at the points, accuracy against the plain sum, and
    points on top of the particles reproduce fmm_evaluate bit for bit."""
    import torch
    import paper_0905_2637_amd as fm
    x, y, q = workloads.uniform_square(4000, 930)
    rng = np.random.default_rng(931)
    tx = np.concatenate([rng.random(2501), x[:30], np.arange(9) / 8.0])
    ty = np.concatenate([rng.random(2501), y[:30], rng.random(9)])
    sigma, L, p = 0.05, 5, 16
    plan = fm.Plan(len(x), sigma, p, L, kernel="gauss-transform", m_max=len(x))
    xd, yd, qd = _dev(x), _dev(y), _dev(q)
    G, v = plan.evaluate_at(xd, yd, qd, _dev(tx), _dev(ty), check=True)
    Gp, _ = plan.evaluate(xd, yd, qd)
    Gs, _ = plan.evaluate_at(xd, yd, qd, xd, yd)
    torch.cuda.synchronize()
    plan.close()
    G, v = G.cpu().numpy(), v.cpu().numpy()
    assert not v.any()
    Go, nbad = oracle.fgt_at(x, y, q, sigma, p, L, _range(sigma, L), tx, ty)
    assert nbad == 0 and _rel(G, Go) < 1e-12
    assert _rel(G, oracle.gauss_direct_at(x, y, q, sigma, tx, ty)) < 1e-13
    assert np.array_equal(Gs.cpu().numpy(), Gp.cpu().numpy())


def test_fgt_one_and_no_particle():
    import torch
    import paper_0905_2637_amd as fm
    x, y, q = np.array([0.37]), np.array([0.61]), np.array([2.5])
    G = _gpu(x, y, q, 0.05, 12, 4)
    Go, _ = oracle.fgt(x, y, q, 0.05, 12, 4, _range(0.05, 4))
    assert G[0] == pytest.approx(Go[0], rel=1e-13)
    assert G[0] == pytest.approx(2.5, rel=1e-7)      # its own term, to the expansions' accuracy
    plan = fm.Plan(10, 0.05, 12, 4, kernel="gauss-transform")
    e = _dev(np.zeros(0))
    plan.evaluate(e, e, e)
    torch.cuda.synchronize()
    plan.close()


def test_fgt_unsupported_combinations():
    import ctypes as C
    import paper_0905_2637_amd as fm
    lib = fm.load()
    out = C.c_size_t(0)

    def ws(**kw):
        base = dict(kernel="gauss-transform")
        base.update(kw)
        sigma = base.pop("sigma", 0.05)
        p = base.pop("p", 12)
        L = base.pop("L", 5)
        prm = fm.make_params(1000, sigma, p, L, **base)
        return lib.fmm_workspace_size(C.byref(prm), C.byref(out))

    assert ws() == fm.FMM_OK
    assert ws(domain=None) == fm.FMM_E_UNSUPPORTED
    assert ws(precision="mixed") == fm.FMM_E_UNSUPPORTED
    assert ws(p=17) == fm.FMM_E_UNSUPPORTED
    assert ws(sigma=0.3, L=9) == fm.FMM_E_UNSUPPORTED        # a range beyond 63 boxes
    assert ws(m_max=5) == fm.FMM_OK
    prm = fm.make_params(100, 0.05, 12, 3, kernel="gauss-transform", max_instances=2)
    assert lib.fmm_workspace_size(C.byref(prm), C.byref(out)) == fm.FMM_E_UNSUPPORTED
    x, y, q = (_dev(a) for a in workloads.uniform_square(100, 920))
    plan = fm.Plan(100, 0.05, 12, 3, kernel="gauss-transform")
    with pytest.raises(fm.FmmError) as ei:
        plan.advance_rk2(x, y, q, 1e-3, 1)
    assert ei.value.status == fm.FMM_E_UNSUPPORTED
    plan.close()
