"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work (keys, permutation, leaf ranges, interaction lists) must match
bit for bit; FP64 velocities within 1e-12 relative L2 of the oracle FMM; the
mixed-precision form within 1e-6 of the FP64 split-kernel direct sum.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import deinterleave, gpu_coeffs_to_oracle, interleave, level_offset, run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-6


def _fm():
    import paper_0905_2637_amd as fm
    return fm


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _clustered(n, seed, frac=0.4, centre=(0.3, 0.6), spread=0.002):
    """Uniform background plus a tight cluster: empty, sparse and >256-particle leaves."""
    rng = np.random.default_rng(seed)
    m = int(n * frac)
    x = np.concatenate([rng.random(n - m), centre[0] + spread * rng.standard_normal(m)])
    y = np.concatenate([rng.random(n - m), centre[1] + spread * rng.standard_normal(m)])
    x = np.clip(x, 0.0, np.nextafter(1.0, 0.0))
    y = np.clip(y, 0.0, np.nextafter(1.0, 0.0))
    g = rng.uniform(-1, 1, n)
    return x, y, g


# ---------------------------------------------------------------------------
# Tree: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["c1", "clustered", "duplicates", "domain", "auto"])
def test_tree_bit_exact(case):
    fm = _fm()
    dom = (0.0, 0.0, 1.0)
    L = 4
    if case == "c1":
        wl = workloads.make("C1")
        x, y, g = wl.x, wl.y, wl.gamma
    elif case == "clustered":
        x, y, g = _clustered(6000, 3)
        L = 5
    elif case == "duplicates":
        rng = np.random.default_rng(4)
        x = rng.integers(0, 32, 5000) / 32.0     # many points exactly on box edges
        y = rng.integers(0, 32, 5000) / 32.0
        g = rng.uniform(-1, 1, 5000)
    elif case == "domain":
        rng = np.random.default_rng(5)
        dom = (-2.5, 1.25, 3.0)
        x = -2.5 + 3.0 * rng.random(3000)
        y = 1.25 + 3.0 * rng.random(3000)
        g = rng.uniform(-1, 1, 3000)
        L = 6
    else:
        rng = np.random.default_rng(6)
        x = 10.0 + 0.37 * rng.random(2500)
        y = -4.0 + 0.21 * rng.random(2500)
        g = rng.uniform(-1, 1, 2500)
        dom = None
        L = 5
    u, v, plan = run(x, y, g, 0.01, 12, L, domain=dom)
    if dom is None:
        x0, y0, W = oracle.bounding_square(x, y)
        d = plan.dump(fm.DUMP_DOMAIN)
        assert (d[0], d[1], d[2]) == (x0, y0, W)
        assert d[3] == np.ldexp(1.0, L) / W
    else:
        x0, y0, W = dom
    key, perm, ls, nbad = oracle.tree(x, y, L, x0, y0, W)
    assert np.array_equal(plan.dump(fm.DUMP_KEYS), key)
    assert np.array_equal(plan.dump(fm.DUMP_PERM), perm)
    assert np.array_equal(plan.dump(fm.DUMP_LEAF_START).astype(np.int64), ls)
    assert plan.out_of_domain() == nbad == 0
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))


def test_interaction_lists_match_as_sets():
    """Every box's list as the M2L kernel walks it equals the oracle's list
    (box output in any order, compared by global box number)."""
    fm = _fm()
    L = 5
    x, y, g = workloads.uniform_square(2000, 7)
    _, _, plan = run(x, y, g, 0.01, 8, L)
    il = plan.dump(fm.DUMP_ILIST)
    assert il.shape == (level_offset(L + 1), 27)
    for l in range(0, L + 1):
        side = 1 << l
        for m in range(side * side):
            a, b = (int(t[0]) for t in deinterleave(np.array([m])))
            ref = {level_offset(l) + int(interleave([sa], [sb])[0]) for sa, sb in oracle.interaction_list(l, a, b)}
            got = il[level_offset(l) + m]
            got_set = set(int(t) for t in got if t >= 0)
            assert len(got_set) == int(np.sum(got >= 0))      # no duplicates
            assert got_set == ref, (l, a, b)


# ---------------------------------------------------------------------------
# FP64 FMM vs the oracle FMM
# ---------------------------------------------------------------------------

def test_c1_fp64_matches_oracle_and_coefficients():
    fm = _fm()
    wl = workloads.make("C1")
    u, v, plan = run(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth)
    uo, vo, me, le, _ = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth, dump=True)
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL
    gme = gpu_coeffs_to_oracle(plan.dump(fm.DUMP_ME), wl.depth, 1.0, "me")
    gle = gpu_coeffs_to_oracle(plan.dump(fm.DUMP_LE), wl.depth, 1.0, "le")
    for l in range(2, wl.depth + 1):
        sl = slice(level_offset(l), level_offset(l + 1))
        for got, ref in ((gme[sl], me[sl]), (gle[sl], le[sl])):
            err = np.max(np.abs(got - ref), axis=1) / np.maximum(np.max(np.abs(ref), axis=1), 1e-300)
            assert np.max(err) < 1e-11, (l, np.max(err))
    # and the accuracy the 12-term expansion buys against the split direct sum
    us, vs = oracle.direct_split(wl.x, wl.y, wl.gamma, wl.sigma, wl.depth)
    assert oracle.rel_l2(u, v, us, vs) < 3e-6


@pytest.mark.parametrize("n,L,p,sigma,seed", [
    (1, 3, 12, 0.01, 1),
    (2, 2, 4, 0.01, 2),
    (7, 2, 5, 0.02, 3),
    (3000, 3, 8, 0.01, 4),
    (5000, 5, 17, 0.003, 5),
    (20000, 5, 20, 0.002, 6),
    (4000, 4, 13, 0.005, 7),
    (3000, 4, 24, 0.005, 8),
    (3000, 3, 32, 0.005, 9),
    (65, 6, 12, 0.01, 10),
    (900, 3, 1, 0.01, 11),      # a single term: the smallest expansion
    (900, 4, 2, 0.01, 12),
])
def test_fp64_parameter_grid(n, L, p, sigma, seed):
    x, y, g = workloads.uniform_square(n, seed)
    u, v, _ = run(x, y, g, sigma, p, L)
    uo, vo = oracle.fmm(x, y, g, sigma, p, L)
    if n == 1:      # a lone particle induces nothing on itself
        assert u[0] == 0.0 and v[0] == 0.0 and uo[0] == 0.0 and vo[0] == 0.0
        return
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL


@pytest.mark.parametrize("p", [17, 20])
def test_fp64_m2l_register_and_staged_forms(p):
    """Depth 7 has 87 M2L tiles.  Split three ways (the default) they take 261
    workgroups, unsplit 87: the register form of the FP64 M2L runs.  Split up
    to level 5, levels 2-5 take 21 workgroups and run in the form with the
    sources staged in LDS, levels 6-7 in the register form.  All match the
    oracle and each other (the splits only reassociate the sums)."""
    import torch
    fm = _fm()
    x, y, g = workloads.uniform_square(40000, 13)
    uo, vo = oracle.fmm(x, y, g, 0.002, p, 7)
    plan = fm.Plan(len(x), 0.002, p, 7)
    xd, yd, gd = (torch.as_tensor(a, device="cuda") for a in (x, y, g))
    ref = None
    for split in (8, 0, 5):
        plan.set_tuning(4, split, 0)
        u, v = plan.evaluate(xd, yd, gd, check=True)
        torch.cuda.synchronize()
        u, v = u.cpu().numpy(), v.cpu().numpy()
        assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL, split
        if ref is None:
            ref = (u, v)
        else:
            assert oracle.rel_l2(u, v, *ref) < 1e-14, split
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_quad_pairs(precision):
    """The near field inside a 2 x 2 block of sibling leaves is evaluated once
    per pair of particles, for both (quads of 2..64 particles); a lattice
    with exactly 64 per quad, a sparse set with empty leaves in some quads,
    and a set where quads fall on both sides of the 64 limit."""
    rng = np.random.default_rng(31)
    m = 64
    gx, gy = np.meshgrid((np.arange(m) + 0.5) / m, (np.arange(m) + 0.5) / m)
    lattice = (gx.ravel() + 0.3 / m * rng.uniform(-1, 1, m * m), gy.ravel() + 0.3 / m * rng.uniform(-1, 1, m * m))
    cases = [(lattice[0], lattice[1], 4), (*workloads.uniform_square(700, 32)[:2], 5),
             (*workloads.uniform_square(3500, 33)[:2], 4)]
    for x, y, L in cases:
        g = rng.uniform(-1.0, 1.0, len(x))
        u, v, _ = run(x, y, g, 0.01, 17, L, precision=precision)
        uo, vo = oracle.fmm(x, y, g, 0.01, 17, L)
        # mixed: the FP32 parts add at most a few 1e-7 on top of the FP64 result
        assert oracle.rel_l2(u, v, uo, vo) < (FP64_TOL if precision == "fp64" else 5e-7)


def test_dense_and_empty_leaves():
    """Leaves with > 64 and > 256 particles (target chunks, staged source
    chunks) next to empty ones."""
    x, y, g = _clustered(12000, 11, frac=0.5, spread=0.004)
    L = 5
    key, _, ls, _ = oracle.tree(x, y, L)
    counts = np.diff(ls)
    assert counts.max() > 256 and np.sum(counts == 0) > 0
    u, v, _ = run(x, y, g, 0.002, 12, L)
    uo, vo = oracle.fmm(x, y, g, 0.002, 12, L)
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL


@pytest.mark.parametrize("L", [0, 1])
def test_depth_without_far_field_is_direct(L):
    x, y, g = workloads.uniform_square(900, 12)
    u, v, _ = run(x, y, g, 0.02, 12, L)
    ur, vr = oracle.direct(x, y, g, 0.02)
    assert oracle.rel_l2(u, v, ur, vr) < 1e-13


def test_coincident_particles():
    x, y, g = workloads.uniform_square(800, 13)
    x[100:150] = x[0]
    y[100:150] = y[0]
    u, v, _ = run(x, y, g, 0.01, 12, 3)
    uo, vo = oracle.fmm(x, y, g, 0.01, 12, 3)
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL


@pytest.mark.parametrize("sigma", [1e-6, 1e-9])
def test_core_far_below_leaf_width(sigma):
    """The FP64 Gaussian factor is 1 - 2^x with x = -r^2 log2(e) / (2 sigma^2).
    With the core far below the leaf width (depth 4, w = 1/16) x reaches
    about -3e9 (sigma 1e-6: its integer part past the 32-bit range, where
    the conversion must saturate) and -3e15 (sigma 1e-9: past 2^52, where x
    has no fraction); the factor must come out exactly 1 there.  A row of
    particles 0.7 sigma apart keeps the Gaussian itself in play."""
    x, y, g = workloads.uniform_square(3000, 41)
    x[1:20] = x[0] + sigma * 0.7 * np.arange(1, 20)
    y[1:20] = y[0]
    u, v, _ = run(x, y, g, sigma, 12, 4)
    uo, vo = oracle.fmm(x, y, g, sigma, 12, 4)
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL
    assert oracle.rel_l2(u[20:], v[20:], uo[20:], vo[20:]) < FP64_TOL


@pytest.mark.parametrize("ex0,ew", [(130, 93), (-80, -90)])
def test_scaled_copies_of_the_unit_square(ex0, ew):
    """The unit-square problem moved to x, y near +-2^ex0 and scaled by 2^ew
    (all positions exact, on a 2^-15 grid of the square): velocities scale
    by 2^-ew exactly, so the result times 2^ew is compared with the oracle
    on the unit square, where its unscaled expansions are exact enough.
    Near 2^130 with width 2^93 (within the 1e36 limit): the FP64 near field
    takes the reciprocal of a product of four squared separations, and the
    padding it adds (targets past a leaf's count, inert source slots, the
    quad's spare lanes) sits on the leaf's scale, so the product stays in
    range (at 1e10, as distance from a point near 2^130, four squares would
    overflow).  At width 2^-90 (sigma 3.2e-30, just above the 1e-30 limit):
    squared separations near 1e-63, far above the 1e-76 floor.  A few
    coincident particles included."""
    ux, uy, g = workloads.uniform_square(3000, 43)
    ux = np.floor(ux * 2.0 ** 15) / 2.0 ** 15
    uy = np.floor(uy * 2.0 ** 15) / 2.0 ** 15
    ux[200:210] = ux[5]
    uy[200:210] = uy[5]
    x0, y0, w = 2.0 ** ex0, -(2.0 ** ex0), 2.0 ** ew
    x, y = x0 + w * ux, y0 + w * uy
    assert np.array_equal((x - x0) / w, ux) and np.array_equal((y - y0) / w, uy)
    u, v, plan = run(x, y, g, 0.004 * w, 12, 4, domain=(x0, y0, w))
    assert plan.out_of_domain() == 0
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))
    uo, vo = oracle.fmm(ux, uy, g, 0.004, 12, 4)
    assert oracle.rel_l2(u * w, v * w, uo, vo) < FP64_TOL


def test_bounding_square_wider_than_limit_is_flagged():
    """A bounding square wider than 1e36 counts every particle as outside
    the domain; the default call raises FMM_E_DOMAIN."""
    fm = _fm()
    x, y, g = workloads.uniform_square(500, 44)
    x = x.copy()
    x[0] = 2e36
    _, _, plan = run(x, y, g, 0.01, 8, 3, domain=None)
    assert plan.out_of_domain() == 500
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate(_dev(x), _dev(y), _dev(g))
    assert ei.value.status == fm.FMM_E_DOMAIN
    plan.close()


def test_out_of_domain_points_are_counted():
    """Points outside an explicit domain are clamped into the nearest leaf,
    counted, and computed exactly as the oracle computes them."""
    x, y, g = workloads.uniform_square(1000, 14)
    x[3] = -0.1
    y[10] = 1.5
    u, v, plan = run(x, y, g, 0.01, 8, 3)
    _, _, nbad = oracle.quantize(x, y, 3)
    assert nbad == 2 and plan.out_of_domain() == 2
    uo, vo = oracle.fmm(x, y, g, 0.01, 8, 3)
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL


def test_default_call_raises_on_out_of_domain():
    """The binding reads the device status word after every call unless told
    not to: a particle outside the explicit square, or a target point outside
    it, raises FMM_E_DOMAIN."""
    import torch
    fm = _fm()
    x, y, g = workloads.uniform_square(600, 18)
    x[7] = 1.25
    plan = fm.Plan(600, 0.01, 8, 3, m_max=10)
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate(_dev(x), _dev(y), _dev(g))
    assert ei.value.status == fm.FMM_E_DOMAIN
    x[7] = 0.5
    plan.evaluate(_dev(x), _dev(y), _dev(g))      # inside again: no error
    tx = np.full(10, 0.5)
    tx[3] = -2.0
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate_at(_dev(x), _dev(y), _dev(g), _dev(tx), _dev(np.full(10, 0.5)))
    assert ei.value.status == fm.FMM_E_DOMAIN
    torch.cuda.synchronize()
    plan.close()


def test_nan_position_is_counted():
    x, y, g = workloads.uniform_square(500, 17)
    x[20] = np.nan
    _, _, plan = run(x, y, g, 0.01, 8, 3)
    assert plan.out_of_domain() == 1


def test_capacity_and_empty_input():
    import torch
    fm = _fm()
    plan = fm.Plan(100, 0.01, 8, 3)
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    u, v = plan.evaluate(z, z, z)
    assert u.numel() == 0 and plan.out_of_domain() == 0
    big = torch.rand(101, dtype=torch.float64, device="cuda")
    with pytest.raises(fm.FmmError) as ei:
        plan.evaluate(big, big, big)
    assert ei.value.status == fm.FMM_E_CAPACITY
    # a smaller call after a larger one reuses the plan
    x, y, g = workloads.uniform_square(100, 15)
    u1, v1, _ = run(x, y, g, 0.01, 8, 3, n_max=100)
    uo, vo = oracle.fmm(x, y, g, 0.01, 8, 3)
    assert oracle.rel_l2(u1, v1, uo, vo) < FP64_TOL


def test_fp64_bitwise_reproducible():
    import torch
    fm = _fm()
    x, y, g = _clustered(8000, 16)
    plan = fm.Plan(8000, 0.003, 17, 5)
    dev = torch.device("cuda")
    xt, yt, gt = (torch.as_tensor(a, device=dev) for a in (x, y, g))
    u1, v1 = plan.evaluate(xt, yt, gt)
    u1, v1 = u1.clone(), v1.clone()
    u2, v2 = plan.evaluate(xt, yt, gt)
    assert torch.equal(u1, u2) and torch.equal(v1, v2)


# ---------------------------------------------------------------------------
# Mixed precision (FP32 near field and fine-level M2L)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,L,p,sigma,fine,seed", [
    (4096, 4, 17, 0.005, 2, 21),
    (20000, 6, 17, 0.002, 2, 22),
    (20000, 6, 20, 0.0015, 3, 23),
    (6000, 5, 12, 0.003, 0, 24),
])
def test_mixed_within_gate_of_split_direct(n, L, p, sigma, fine, seed):
    x, y, g = workloads.uniform_square(n, seed)
    u, v, _ = run(x, y, g, sigma, p, L, precision="mixed", fine=fine)
    us, vs = oracle.direct_split(x, y, g, sigma, L)
    uo, vo = oracle.fmm(x, y, g, sigma, p, L)
    trunc = oracle.rel_l2(uo, vo, us, vs)
    err = oracle.rel_l2(u, v, us, vs)
    # the FP32 parts add at most a few 1e-7 on top of the FP64 result
    assert oracle.rel_l2(u, v, uo, vo) < 5e-7, (err, trunc)
    assert err < trunc + 5e-7
    if trunc < 5e-7:            # the expansion order can meet the gate at all
        assert err < MIXED_TOL


@pytest.mark.parametrize("mfma", [0, 1])
@pytest.mark.parametrize("n,L,p,sigma,fine,split,seed", [
    (20000, 6, 17, 0.002, 2, 5, 26),    # FP32 level 5 split over wavefronts, level 6 not
    (20000, 6, 20, 0.0015, 3, 5, 27),   # FP32 levels 4-5 split, 6 not
    (6000, 5, 12, 0.003, 2, 8, 28),     # every FP32 level split
    (20000, 6, 12, 0.002, 2, 0, 29),    # no level split
    (3000, 3, 12, 0.01, 2, 8, 30),      # every level FP32 and split: no FP64 split level
    (6000, 5, 8, 0.003, 2, 0, 31),      # the compiled sizes 8, 16 and 24 of the FP32 kernels
    (6000, 5, 15, 0.003, 2, 0, 32),
    (6000, 5, 22, 0.003, 2, 5, 33),
])
def test_mixed_m2l_forms_match_oracle(n, L, p, sigma, fine, split, seed, mfma):
    """The FP32 M2L levels on the matrix cores (mfma = 1) and paired on the
    vector units (mfma = 0, the default), the two launch shapes the
    autotuner chooses between for a mixed plan, against the oracle FMM and
    the FP64 split-kernel direct sum, at the mixed form's tolerances."""
    import torch
    fm = _fm()
    x, y, g = workloads.uniform_square(n, seed)
    plan = fm.Plan(n, sigma, p, L, precision="mixed", fp32_fine_levels=fine)
    plan.set_tuning(4, split, mfma)
    assert plan.tuning()["m2l_mfma"] == mfma
    u, v = plan.evaluate(_dev(x), _dev(y), _dev(g))
    torch.cuda.synchronize()
    u, v = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    uo, vo = oracle.fmm(x, y, g, sigma, p, L)
    us, vs = oracle.direct_split(x, y, g, sigma, L)
    trunc = oracle.rel_l2(uo, vo, us, vs)
    err = oracle.rel_l2(u, v, us, vs)
    assert oracle.rel_l2(u, v, uo, vo) < 5e-7, (err, trunc)
    assert err < trunc + 5e-7
    if trunc < 5e-7:
        assert err < MIXED_TOL


def test_mixed_dense_leaves():
    x, y, g = _clustered(12000, 25, frac=0.5, spread=0.004)
    u, v, _ = run(x, y, g, 0.002, 17, 5, precision="mixed", fine=2)
    us, vs = oracle.direct_split(x, y, g, 0.002, 5)
    assert oracle.rel_l2(u, v, us, vs) < MIXED_TOL
