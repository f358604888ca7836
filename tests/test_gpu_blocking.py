"""Near-field register blocking (the p2p_block tuning knob) against the
oracle: a wavefront takes a leaf's targets in chunks of t <= 64 and lays a
chunk out as R targets per lane, TG lane groups and S source slices, from a
table built when the plan is made.  Policy 0 pads t to a power of two,
policy 1 keeps the most lanes on real pairs (TG and S then need not be
powers of two, and the slices meet through LDS).  The near field is the
paper's direct sum over the 3 x 3 neighbourhood (Section 3, eq. 8), so each
policy must reproduce the oracle's FMM:

* every chunk size t = 1 .. 64 once (a depth-3 tree whose 64 leaves hold 1,
  2, ..., 64 particles) and leaves of up to 300 (several chunks);
* FP64 within 1e-12 of the oracle and within 1e-14 of the other policy;
  mixed within the mixed form's 1e-6 of the oracle;
* the singular kernel (eq. 7), Lennard-Jones forces and target points
  (fmm_evaluate_at) under policy 1.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _by_leaf(L, counts, seed):
    """counts[i] points uniform inside leaf i of the depth-L grid (row major)."""
    rng = np.random.default_rng(seed)
    side = 1 << L
    w = 1.0 / side
    xs, ys = [], []
    for i, c in enumerate(counts):
        a, b = i % side, i // side
        xs.append((a + rng.uniform(0.01, 0.99, c)) * w)
        ys.append((b + rng.uniform(0.01, 0.99, c)) * w)
    x, y = np.concatenate(xs), np.concatenate(ys)
    return x, y, rng.uniform(-1.0, 1.0, len(x))


CASES = {
    "t1to64": (3, lambda rng: rng.permutation(np.arange(1, 65))),
    "multichunk": (4, lambda rng: rng.integers(0, 301, 256)),
}


def _evaluate(x, y, g, sigma, p, L, precision, block, kernel="gaussian", **kw):
    import torch
    import paper_0905_2637_amd as fm
    plan = fm.Plan(len(x), sigma, p, L, precision=precision, kernel=kernel, **kw)
    t = plan.tuning()
    t["p2p_block"] = block
    plan.set_tuning(**t)
    assert plan.tuning()["p2p_block"] == block
    u, v = plan.evaluate(_dev(x), _dev(y), _dev(g))
    torch.cuda.synchronize()
    plan.close()
    return u.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_policies_match_oracle_and_each_other(case):
    L, counts = CASES[case]
    c = counts(np.random.default_rng(61))
    x, y, g = _by_leaf(L, c, 62)
    print(f"{case}: n = {len(x)}, depth {L}", flush=True)
    uo, vo = oracle.fmm(x, y, g, 0.004, 14, L)
    out = []
    for block in (0, 1):
        u, v = _evaluate(x, y, g, 0.004, 14, L, "fp64", block)
        err = oracle.rel_l2(u, v, uo, vo)
        assert err < FP64_TOL, (block, err)
        out.append((u, v))
    assert oracle.rel_l2(*out[1], *out[0]) < 1e-14


@pytest.mark.parametrize("case", sorted(CASES))
def test_mixed_policies_match_oracle(case):
    L, counts = CASES[case]
    c = counts(np.random.default_rng(63))
    x, y, g = _by_leaf(L, c, 64)
    uo, vo = oracle.fmm(x, y, g, 0.004, 14, L)
    for block in (0, 1):
        u, v = _evaluate(x, y, g, 0.004, 14, L, "mixed", block, fp32_fine_levels=1)
        err = oracle.rel_l2(u, v, uo, vo)
        assert err < 1e-6, (block, err)


def test_singular_kernel_policy1():
    L, counts = CASES["t1to64"]
    x, y, g = _by_leaf(L, counts(np.random.default_rng(65)), 66)
    uo, vo = oracle.fmm(x, y, g, 0.0, 14, L)
    u, v = _evaluate(x, y, g, 0.0, 14, L, "fp64", 1, kernel="singular")
    assert oracle.rel_l2(u, v, uo, vo) < FP64_TOL


def test_lennard_jones_policy1():
    """Leaves of 1 .. 64 particles, cutoff one leaf width: every pair within
    the cutoff lies in the 3 x 3 neighbourhood."""
    L, counts = CASES["t1to64"]
    x, y, _ = _by_leaf(L, counts(np.random.default_rng(67)), 68)
    s, eps, rc = 0.004, 0.8, 1.0 / (1 << L)
    fx, fy = _evaluate(x, y, np.zeros(len(x)), s, 8, L, "fp64", 1, kernel="lennard-jones", lj_epsilon=eps,
                       cutoff=rc)
    ox, oy = oracle.lj_forces(x, y, eps, s, rc)
    scale = np.sqrt(np.mean(ox ** 2 + oy ** 2))
    assert np.sqrt(np.mean((fx - ox) ** 2 + (fy - oy) ** 2)) / scale < 1e-12


def test_target_points_policy1():
    import torch
    import paper_0905_2637_amd as fm
    L, counts = CASES["multichunk"]
    x, y, g = _by_leaf(L, counts(np.random.default_rng(69)), 70)
    tx, ty, _ = _by_leaf(L, np.random.default_rng(71).integers(0, 130, 1 << (2 * L)), 72)
    plan = fm.Plan(len(x), 0.004, 14, L, m_max=len(tx))
    t = plan.tuning()
    t["p2p_block"] = 1
    plan.set_tuning(**t)
    u, v = plan.evaluate_at(_dev(x), _dev(y), _dev(g), _dev(tx), _dev(ty))
    torch.cuda.synchronize()
    plan.close()
    uo, vo, nbad = oracle.fmm_at(x, y, g, 0.004, 14, L, tx, ty)
    assert nbad == 0
    assert oracle.rel_l2(u.cpu().numpy(), v.cpu().numpy(), uo, vo) < FP64_TOL
