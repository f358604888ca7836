"""The velocity at target points distinct from the particles on the GPU
(fmm_evaluate_at; eq. 1 with targets y_i apart from the sources x_j).

* the points' keys, sort permutation and leaf ranges are bit-exact with the
  oracle's tree of the same points;
* velocities match the oracle FMM at the same points within 1e-12 (relative
  L2, FP64) over depths 0-4, expansion sizes, sparse and dense leaves of
  points and particles, points on top of particles, on leaf edges and a
  ragged count;
* with the bounding-square domain the square covers particles and points;
* points at the particles' own positions reproduce fmm_evaluate;
* points outside an explicit square are counted;
* m = 0, n = 0, capacity, mixed-precision and batched-plan errors.
"""
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


def _gpu_at(x, y, g, tx, ty, sigma, p, L, domain, m_max=None):
    import torch
    import paper_0905_2637_amd as fm
    m = len(tx)
    plan = fm.Plan(len(x), sigma, p, L, domain=domain, m_max=m if m_max is None else m_max)
    u, v = plan.evaluate_at(_dev(x), _dev(y), _dev(g), _dev(tx), _dev(ty), check=False)
    torch.cuda.synchronize()
    out = dict(u=u.cpu().numpy(), v=v.cpu().numpy(), nbad=plan.out_of_domain(),
               tkeys=plan.dump(fm.DUMP_TKEYS), tperm=plan.dump(fm.DUMP_TPERM),
               tls=plan.dump(fm.DUMP_TLEAF_START), dom=plan.dump(fm.DUMP_DOMAIN))
    plan.close()
    return out


def _points(rng, m, lo=0.0, hi=1.0):
    return rng.uniform(lo, hi, m), rng.uniform(lo, hi, m)


def _check(x, y, g, tx, ty, sigma, p, L, domain=(0.0, 0.0, 1.0), tol=1e-12):
    r = _gpu_at(x, y, g, tx, ty, sigma, p, L, domain)
    x0, y0, W = domain if domain is not None else oracle.bounding_square(np.concatenate([x, tx]),
                                                                          np.concatenate([y, ty]))
    if domain is None:
        assert (r["dom"][0], r["dom"][1], r["dom"][2]) == (x0, y0, W)
    key_o, perm_o, ls_o, nbad_t = oracle.tree(tx, ty, L, x0, y0, W)
    assert np.array_equal(r["tkeys"], key_o), "point keys differ from the oracle"
    assert np.array_equal(r["tperm"], perm_o), "point permutation differs from the oracle"
    assert np.array_equal(r["tls"].astype(np.int64), ls_o), "point leaf ranges differ from the oracle"
    uo, vo, nbad = oracle.fmm_at(x, y, g, sigma, p, L, tx, ty, x0, y0, W)
    assert r["nbad"] == nbad
    err = oracle.rel_l2(r["u"], r["v"], uo, vo)
    assert err < tol, f"rel L2 vs the oracle FMM at the points {err:.3e}"
    return r, (uo, vo)


def test_uniform_points_ragged_with_coincident():
    """C1's particles (4096 uniform, depth 4, p = 12); 3001 uniform points
    plus 50 on top of particles and 17 on leaf edges."""
    wl = workloads.make("C1")
    rng = np.random.default_rng(501)
    tx, ty = _points(rng, 3001)
    edge = np.arange(17) / 16.0
    tx = np.concatenate([tx, wl.x[:50], edge])
    ty = np.concatenate([ty, wl.y[:50], rng.random(17)])
    _check(wl.x, wl.y, wl.gamma, tx, ty, wl.sigma, wl.p, wl.depth)


@pytest.mark.parametrize("L,p", [(0, 8), (1, 12), (2, 17), (3, 20)])
def test_shallow_trees(L, p):
    """No far field at depths 0 and 1; few boxes at 2 and 3."""
    x, y, g = workloads.uniform_square(700, 510 + L)
    rng = np.random.default_rng(520 + L)
    tx, ty = _points(rng, 333)
    _check(x, y, g, tx, ty, 0.02, p, L)


def test_dense_leaves_of_particles_and_points():
    """Clustered particles (hundreds per leaf at depth 3) and points packed
    into a few leaves (chunks of 64 points with four per lane), beside
    leaves with one or a handful of points; p = 24."""
    x, y, g, _, _ = workloads.gaussian_mixture(20000, 4, 530)
    rng = np.random.default_rng(531)
    tx = np.concatenate([rng.uniform(0.3, 0.36, 900), rng.uniform(0.0, 1.0, 120), [0.93]])
    ty = np.concatenate([rng.uniform(0.55, 0.62, 900), rng.uniform(0.0, 1.0, 120), [0.07]])
    _check(x, y, g, tx, ty, 0.003, 24, 3)


def test_auto_domain_covers_the_points():
    """Particles in [0.25, 0.75]^2, points across [0, 1.2]^2: the bounding
    square is that of both sets."""
    rng = np.random.default_rng(540)
    x, y = rng.uniform(0.25, 0.75, 2500), rng.uniform(0.25, 0.75, 2500)
    g = rng.uniform(-1.0, 1.0, 2500)
    tx, ty = _points(rng, 1500, 0.0, 1.2)
    r, _ = _check(x, y, g, tx, ty, 0.004, 17, 4, domain=None)
    assert r["dom"][2] > 1.19


def test_points_at_the_particles_reproduce_evaluate():
    import torch
    import paper_0905_2637_amd as fm
    wl = workloads.make("C1")
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth, m_max=wl.n)
    x, y, g = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    u1, v1 = plan.evaluate(x, y, g)
    u2, v2 = plan.evaluate_at(x, y, g, x, y)
    torch.cuda.synchronize()
    plan.close()
    err = oracle.rel_l2(u2.cpu().numpy(), v2.cpu().numpy(), u1.cpu().numpy(), v1.cpu().numpy())
    assert err < 1e-13, f"points at the particles vs fmm_evaluate {err:.3e}"


def test_points_outside_are_counted():
    x, y, g = workloads.uniform_square(400, 550)
    tx = np.array([0.5, 1.5, -0.1, 0.2, 0.31])
    ty = np.array([0.5, 0.5, 0.3, 2.0, 0.77])
    r = _gpu_at(x, y, g, tx, ty, 0.01, 12, 3, (0.0, 0.0, 1.0))
    assert r["nbad"] == 3
    inside = np.array([0, 4])
    uo, vo, _ = oracle.fmm_at(x, y, g, 0.01, 12, 3, tx[inside], ty[inside])
    assert oracle.rel_l2(r["u"][inside], r["v"][inside], uo, vo) < 1e-12


def test_empty_and_error_cases():
    import torch
    import paper_0905_2637_amd as fm
    x, y, g = (_dev(a) for a in workloads.uniform_square(256, 560))
    rng = np.random.default_rng(561)
    tx, ty = (_dev(a) for a in _points(rng, 100))
    plan = fm.Plan(256, 0.01, 12, 3, m_max=100)
    # m = 0: nothing written
    e = _dev(np.zeros(0))
    plan.evaluate_at(x, y, g, e, e, u=_dev(np.zeros(0)), v=_dev(np.zeros(0)))
    # n = 0: the velocity vanishes
    u = _dev(np.full(100, 7.0))
    v = _dev(np.full(100, 7.0))
    plan.evaluate_at(e, e, e, tx, ty, u=u, v=v)
    torch.cuda.synchronize()
    assert not u.cpu().numpy().any() and not v.cpu().numpy().any()
    assert plan.out_of_domain() == 0
    # more points than the plan holds
    t2x, t2y = (_dev(a) for a in _points(rng, 101))
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate_at(x, y, g, t2x, t2y)
    assert ei.value.status == fm.FMM_E_CAPACITY
    plan.close()
    # a plan without target capacity
    plan = fm.Plan(256, 0.01, 12, 3)
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate_at(x, y, g, tx, ty)
    assert ei.value.status == fm.FMM_E_CAPACITY
    plan.close()
    # the mixed form has no point evaluation
    plan = fm.Plan(256, 0.01, 12, 3, precision="mixed", m_max=100)
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate_at(x, y, g, tx, ty)
    assert ei.value.status == fm.FMM_E_UNSUPPORTED
    plan.close()
    # batched plans take no points
    import ctypes as C
    prm = fm.make_params(256, 0.01, 12, 3, m_max=10, max_instances=2)
    lib = fm.load()
    out = C.c_size_t(0)
    assert lib.fmm_workspace_size(C.byref(prm), C.byref(out)) == fm.FMM_E_ARG
    prm.m_max = 0
    assert lib.fmm_workspace_size(C.byref(prm), C.byref(out)) == fm.FMM_OK


@pytest.mark.slow
def test_c2_particles_probe_lattice_full_size():
    """C2's 2^20 particles, the velocity on a 1024 x 1024 vertex lattice of
    points (leaf edges included): sampled points against the oracle FMM at
    those points (1e-12) and the FP64 split-kernel sum (1e-6)."""
    import torch
    import paper_0905_2637_amd as fm
    wl = workloads.make("C2")
    tx, ty = workloads.probe_lattice(1024)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth, domain=(wl.x0, wl.y0, wl.width), m_max=len(tx))
    u, v = plan.evaluate_at(_dev(wl.x), _dev(wl.y), _dev(wl.gamma), _dev(tx), _dev(ty), check=True)
    torch.cuda.synchronize()
    tk, tp, tls = plan.dump(fm.DUMP_TKEYS), plan.dump(fm.DUMP_TPERM), plan.dump(fm.DUMP_TLEAF_START)
    u, v = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    key_o, perm_o, ls_o, _ = oracle.tree(tx, ty, wl.depth, wl.x0, wl.y0, wl.width)
    assert np.array_equal(tk, key_o) and np.array_equal(tp, perm_o)
    assert np.array_equal(tls.astype(np.int64), ls_o)
    s = workloads.sample_targets(len(tx), 2048, 1020)
    uo, vo, nbad = oracle.fmm_at(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, tx[s], ty[s],
                                 wl.x0, wl.y0, wl.width)
    assert nbad == 0
    err = oracle.rel_l2(u[s], v[s], uo, vo)
    assert err < 1e-12, f"rel L2 vs the oracle FMM {err:.3e}"
    s2 = workloads.sample_targets(len(tx), 512, 1021)
    us, vs = oracle.direct_split_at(wl.x, wl.y, wl.gamma, wl.sigma, wl.depth, tx[s2], ty[s2],
                                    wl.x0, wl.y0, wl.width)
    gate = oracle.rel_l2(u[s2], v[s2], us, vs)
    assert gate < 1e-6, f"rel L2 vs the FP64 split direct sum {gate:.3e}"
