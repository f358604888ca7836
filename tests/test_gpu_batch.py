"""Batched form and launch-shape tuning, through the C ABI.

A batched evaluation must give every instance exactly what a single
evaluation of that instance gives (same kernels, same arithmetic order), and
therefore what the oracle gives; a replayed graph must match the eager
result on every replay; every launch shape the autotuner may pick must give
the same velocities up to the summation order of the split M2L levels.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _fm():
    import paper_0905_2637_amd as fm
    return fm


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _instances(counts, depths, seed):
    """Uneven instances in the unit square: uniform, clustered and tiny ones."""
    rng = np.random.default_rng(seed)
    xs, ys, gs = [], [], []
    for i, n in enumerate(counts):
        if i % 3 == 1 and n > 10:
            m = n // 2
            x = np.concatenate([rng.random(n - m), 0.4 + 0.01 * rng.standard_normal(m)])
            y = np.concatenate([rng.random(n - m), 0.7 + 0.01 * rng.standard_normal(m)])
        else:
            x = rng.random(n)
            y = rng.random(n)
        xs.append(np.clip(x, 0.0, np.nextafter(1.0, 0.0)))
        ys.append(np.clip(y, 0.0, np.nextafter(1.0, 0.0)))
        gs.append(rng.uniform(-1.0, 1.0, n))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(gs), off


def _batch(counts, depths, x, y, g, sigma, p, precision="fp64", fine=2):
    import torch
    fm = _fm()
    bp = fm.BatchPlan(counts, depths, sigma, p, precision=precision, fp32_fine_levels=fine)
    u, v = bp.evaluate(_dev(x), _dev(y), _dev(g), check=True)
    torch.cuda.synchronize()
    return u.cpu().numpy(), v.cpu().numpy(), bp


COUNTS = [3000, 700, 0, 1, 2, 5000, 64, 1500, 12000]
DEPTHS = [4, 3, 2, 0, 1, 5, 2, 3, 6]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_evaluations(precision):
    """Instance i of a batch == a single evaluation of instance i, bit for bit,
    including the permutation and leaf ranges of its segment."""
    fm = _fm()
    x, y, g, off = _instances(COUNTS, DEPTHS, 11)
    ub, vb, bp = _batch(COUNTS, DEPTHS, x, y, g, 0.004, 12, precision)
    perm_b = bp.dump(fm.DUMP_PERM).astype(np.int64)
    ls_b = bp.dump(fm.DUMP_LEAF_START).astype(np.int64)
    seg = 0
    for i, (n, L) in enumerate(zip(COUNTS, DEPTHS)):
        a, b = off[i], off[i + 1]
        nent = 4 ** L + 1
        if n > 0:
            # a single plan takes at most L-1 FP32 levels; more means the same (all of 2..L)
            us, vs, sp = run(x[a:b], y[a:b], g[a:b], 0.004, 12, L, precision=precision,
                             fine=min(2, max(0, L - 1)))
            assert np.array_equal(ub[a:b], us) and np.array_equal(vb[a:b], vs), f"instance {i}"
            assert np.array_equal(perm_b[a:b] - a, sp.dump(fm.DUMP_PERM).astype(np.int64)), f"perm {i}"
            assert np.array_equal(ls_b[seg:seg + nent] - a, sp.dump(fm.DUMP_LEAF_START)), f"leaf ranges {i}"
            sp.close()
        else:
            assert np.all(ls_b[seg:seg + nent] == a)
        seg += nent
    assert seg == len(ls_b)


def test_batch_matches_oracle_fmm():
    x, y, g, off = _instances(COUNTS, DEPTHS, 12)
    ub, vb, _ = _batch(COUNTS, DEPTHS, x, y, g, 0.004, 12)
    for i, (n, L) in enumerate(zip(COUNTS, DEPTHS)):
        a, b = off[i], off[i + 1]
        if n == 0:
            continue
        uo, vo = oracle.fmm(x[a:b], y[a:b], g[a:b], 0.004, 12, L)
        if n == 1:
            assert ub[a] == 0.0 and vb[a] == 0.0
            continue
        err = oracle.rel_l2(ub[a:b], vb[a:b], uo, vo)
        assert err < FP64_TOL, f"instance {i}: rel L2 {err:.3e}"


def test_graph_replays_match_eager():
    """The captured graph is replayed several times, with other device work and
    synchronisations in between; every replay equals the eager result."""
    import torch
    x, y, g, off = _instances(COUNTS, DEPTHS, 13)
    fm = _fm()
    bp = fm.BatchPlan(COUNTS, DEPTHS, 0.004, 12)
    xt, yt, gt = _dev(x), _dev(y), _dev(g)
    u = torch.empty_like(xt)
    v = torch.empty_like(xt)
    # eager reference: single evaluations instance by instance
    ue = np.zeros(len(x))
    ve = np.zeros(len(x))
    for i, (n, L) in enumerate(zip(COUNTS, DEPTHS)):
        a, b = off[i], off[i + 1]
        if n:
            ue[a:b], ve[a:b], sp = run(x[a:b], y[a:b], g[a:b], 0.004, 12, L)
            sp.close()
    other = fm.Plan(4096, 0.005, 12, 4)
    wl = workloads.make("C1")
    ox, oy, og = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    for rep in range(4):
        u.fill_(np.nan)
        v.fill_(np.nan)
        bp.evaluate(xt, yt, gt, u, v)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ue) and np.array_equal(v.cpu().numpy(), ve), f"replay {rep}"
        # unrelated eager work on the same device between replays
        other.evaluate(ox, oy, og)
        (xt * 2.0).sum().item()
        torch.cuda.synchronize()
    # new output arrays: a fresh capture, same result
    u2, v2 = bp.evaluate(xt, yt, gt)
    torch.cuda.synchronize()
    assert np.array_equal(u2.cpu().numpy(), ue) and np.array_equal(v2.cpu().numpy(), ve)
    # changed inputs through the same pointers: the replay reads the new values
    xt2 = xt.clone()
    yt2 = yt.clone()
    gt2 = (gt * -0.5).contiguous()
    u3, v3 = bp.evaluate(xt2, yt2, gt2)
    gt2.mul_(-2.0)    # now equal to gt again
    u4, v4 = bp.evaluate(xt2, yt2, gt2, u3, v3)
    torch.cuda.synchronize()
    assert np.array_equal(u4.cpu().numpy(), ue) and np.array_equal(v4.cpu().numpy(), ve)
    other.close()
    bp.close()


def test_batch_out_of_domain_counted():
    import torch
    fm = _fm()
    counts = [100, 200]
    x, y, g, off = _instances(counts, [2, 3], 14)
    x[5] = 1.5
    y[150] = -0.25
    bp = fm.BatchPlan(counts, [2, 3], 0.01, 8)
    bp.evaluate(_dev(x), _dev(y), _dev(g), check=False)
    torch.cuda.synchronize()
    assert bp.out_of_domain() == 2
    with pytest.raises(fm.FmmError) as ei:        # the default call reads the status and raises
        bp.evaluate(_dev(x), _dev(y), _dev(g))
    assert ei.value.status == fm.FMM_E_DOMAIN


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_launch_shape_agrees(precision):
    """All tuning candidates give the same velocities (the split M2L levels only
    reassociate the sum) and the split-free shape is reproducible bitwise."""
    import torch
    fm = _fm()
    wl = workloads.make("C1")
    x, y, g = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, 5, precision=precision)
    ref = None
    for mfma in ((0, 1) if precision == "mixed" else (0,)):
        for waves in (2, 4):
            for split in (0, 5, 8):
                for block in (0, 1):
                    plan.set_tuning(waves, split, mfma, 1, block)
                    assert plan.tuning() == {"p2p_waves": waves, "m2l_split_max": split, "m2l_mfma": mfma,
                                             "work_order": 1, "p2p_block": block}
                    u, v = plan.evaluate(x, y, g)
                    torch.cuda.synchronize()
                    u, v = u.cpu().numpy(), v.cpu().numpy()
                    if ref is None:
                        ref = (u, v)
                    else:
                        err = oracle.rel_l2(u, v, *ref)
                        assert err < (1e-14 if precision == "fp64" else 1e-6), (mfma, waves, split, block, err)
    plan.close()


def test_autotune_and_cache(tmp_path, monkeypatch):
    import torch
    fm = _fm()
    wl = workloads.make("C1")
    x, y, g = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FMM_AUTOTUNE_CACHE", str(cache))
    plan = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth)
    t = plan.autotune(x, y, g, reps=2)
    assert t["p2p_waves"] in (2, 4) and t["m2l_split_max"] in (0, 5, 8) and t["m2l_mfma"] in (0, 1)
    assert t["p2p_block"] in (0, 1)
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == 1
    # a planted entry is taken from the cache without a search
    key = lines[0].split()[0]
    cache.write_text(f"{key} 2 0 0 1\n")
    plan2 = fm.Plan(wl.n, wl.sigma, wl.p, wl.depth)
    assert plan2.autotune(x, y, g) == {"p2p_waves": 2, "m2l_split_max": 0, "m2l_mfma": 0, "work_order": 1,
                                       "p2p_block": 1}
    u, v = plan2.evaluate(x, y, g)
    torch.cuda.synchronize()
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth)
    assert oracle.rel_l2(u.cpu().numpy(), v.cpu().numpy(), uo, vo) < FP64_TOL
    plan.close()
    plan2.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_seeded_by_the_work_model(precision, monkeypatch):
    """The work model (eqs. 13-15) orders the search: the part of the
    estimate that dominates is tuned first and a minor part is skipped, so
    the seeded search times fewer candidates than the whole grid (12 in FP64,
    24 in the mixed form) and its choice still gives the oracle's velocities."""
    import torch
    fm = _fm()
    monkeypatch.delenv("FMM_AUTOTUNE_CACHE", raising=False)
    wl = workloads.make("C1")
    x, y, g = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    plan = fm.Plan(wl.n, wl.sigma, wl.p, 5, precision=precision)
    monkeypatch.setenv("FMM_AUTOTUNE_EXHAUSTIVE", "1")
    plan.autotune(x, y, g, reps=1)
    full = plan.autotune_report()
    assert full["candidates_timed"] == (24 if precision == "mixed" else 12)
    monkeypatch.delenv("FMM_AUTOTUNE_EXHAUSTIVE")
    t = plan.autotune(x, y, g, reps=1)
    rep = plan.autotune_report()
    assert 2 <= rep["candidates_timed"] < full["candidates_timed"]
    # N = 4096 on 4^5 leaves (4 per leaf): the far field dominates the estimate
    assert 0.0 < rep["near_share"] < 0.5
    u, v = plan.evaluate(x, y, g)
    torch.cuda.synchronize()
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, 5)
    tol = FP64_TOL if precision == "fp64" else 5e-7
    assert oracle.rel_l2(u.cpu().numpy(), v.cpu().numpy(), uo, vo) < tol, t
    plan.close()


def test_c4_batch_sampled_against_single_and_direct():
    """The 512-instance workload at full size: a batched, autotuned graph
    replay; sampled instances equal their single evaluations bit for bit and
    stay within the mixed-precision gate of the FP64 split-kernel direct sum
    (the gate is loosened to what p = 12 truncation allows)."""
    import torch
    fm = _fm()
    wl = workloads.make("C4")
    counts = np.diff(wl.offsets).tolist()
    depths = wl.depths.tolist()
    bp = fm.BatchPlan(counts, depths, wl.sigma, wl.p, precision=wl.precision,
                      fp32_fine_levels=wl.fp32_fine_levels)
    xt, yt, gt = _dev(wl.x), _dev(wl.y), _dev(wl.gamma)
    bp.autotune(xt, yt, gt, reps=1)
    u, v = bp.evaluate(xt, yt, gt, check=True)
    torch.cuda.synchronize()
    u, v = u.cpu().numpy(), v.cpu().numpy()
    rng = np.random.default_rng(40)
    for i in sorted(rng.choice(len(counts), 6, replace=False)):
        a, b = wl.offsets[i], wl.offsets[i + 1]
        us, vs, sp = run(wl.x[a:b], wl.y[a:b], wl.gamma[a:b], wl.sigma, wl.p, depths[i],
                         precision=wl.precision, fine=wl.fp32_fine_levels)
        sp.set_tuning(**bp.tuning())     # work_order has no effect on a single instance
        us, vs = sp.evaluate(_dev(wl.x[a:b]), _dev(wl.y[a:b]), _dev(wl.gamma[a:b]))
        torch.cuda.synchronize()
        assert np.array_equal(u[a:b], us.cpu().numpy()) and np.array_equal(v[a:b], vs.cpu().numpy()), i
        sp.close()
        t = workloads.sample_targets(int(b - a), 256, 41 + int(i))
        ud, vd = oracle.direct_split(wl.x[a:b], wl.y[a:b], wl.gamma[a:b], wl.sigma, depths[i], targets=t)
        err = oracle.rel_l2(u[a:b][t], v[a:b][t], ud, vd)
        assert err < 1e-5, f"instance {i}: rel L2 vs split direct {err:.3e}"


def test_c4_fp64_batch_every_instance_matches_oracle():
    """The 512-instance workload at full size in FP64: every instance of the
    batched evaluation against the oracle FMM of that instance (1e-12), and
    the pooled error against the oracle over all 10 million particles."""
    import torch
    fm = _fm()
    wl = workloads.make("C4")
    counts = np.diff(wl.offsets).tolist()
    depths = wl.depths.tolist()
    bp = fm.BatchPlan(counts, depths, wl.sigma, wl.p, precision="fp64")
    u, v = bp.evaluate(_dev(wl.x), _dev(wl.y), _dev(wl.gamma), check=True)
    torch.cuda.synchronize()
    u, v = u.cpu().numpy(), v.cpu().numpy()
    bp.close()
    num = den = 0.0
    for i, L in enumerate(depths):
        a, b = int(wl.offsets[i]), int(wl.offsets[i + 1])
        uo, vo = oracle.fmm(wl.x[a:b], wl.y[a:b], wl.gamma[a:b], wl.sigma, wl.p, L)
        err = oracle.rel_l2(u[a:b], v[a:b], uo, vo)
        assert err < FP64_TOL, f"instance {i} (n = {b - a}, depth {L}): rel L2 {err:.3e}"
        num += float(np.sum((u[a:b] - uo) ** 2 + (v[a:b] - vo) ** 2))
        den += float(np.sum(uo ** 2 + vo ** 2))
    assert (num / den) ** 0.5 < FP64_TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_work_order_leaves_results_unchanged(precision):
    """Launching the instances heaviest-first (the paper's work model) only
    reorders workgroups: every instance's arithmetic, and so its result, is
    the same bit for bit."""
    import torch
    fm = _fm()
    x, y, g, off = _instances(COUNTS, DEPTHS, 15)
    bp = fm.BatchPlan(COUNTS, DEPTHS, 0.004, 12, precision=precision)
    xt, yt, gt = _dev(x), _dev(y), _dev(g)
    assert bp.tuning()["work_order"] == 1
    u1, v1 = bp.evaluate(xt, yt, gt)
    t = bp.tuning()
    t["work_order"] = 0
    bp.set_tuning(**t)
    u0, v0 = bp.evaluate(xt, yt, gt)
    torch.cuda.synchronize()
    assert np.array_equal(u1.cpu().numpy(), u0.cpu().numpy()) and np.array_equal(v1.cpu().numpy(), v0.cpu().numpy())
    bp.close()


def test_work_estimate_is_the_papers_model():
    """eqs. 13-15 with n_c = 4, n_IL = 27, n_nd = 9 (computed on the device for
    the call's instances): an empty tree of depth L
    costs (4^L - 1)/3 p^2 (2*4 + 27) + 4^L p^2 27, and particles add
    4^L (2 N_i p + 9 N_i^2) with N_i = N / 4^L."""
    fm = _fm()
    counts = [0, 4096, 0, 16384, 1000]
    depths = [3, 3, 5, 5, 2]
    p = 12
    bp = fm.BatchPlan(counts, depths, 0.004, p)
    x, y, g, _ = _instances(counts, depths, 16)
    bp.evaluate(_dev(x), _dev(y), _dev(g))       # the estimates are made on the device, per call
    w = bp.work_estimate()
    assert w.shape == (5,)
    for n, L, got in zip(counts, depths, w):
        leaves = 4 ** L
        empty = (leaves - 1) / 3 * p * p * 35 + leaves * p * p * 27
        ni = n / leaves
        assert got == pytest.approx(empty + leaves * (2 * ni * p + 9 * ni * ni), rel=1e-12)
    # heavier instances come first in the launch order: the estimate grows
    # with the particle count at a fixed depth
    assert w[1] > w[0] and w[3] > w[2]
    bp.close()
