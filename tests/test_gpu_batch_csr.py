"""The batched call with the instance table on the device: one plan fixes
capacities only (particles, instances, leaves, the deepest tree), and every
fmm_evaluate_batch call brings its own CSR offsets and depths in device
memory (Sections 4 and 5.2: many uneven trees, whose sizes change between
calls).  Through the C ABI:

* one plan, three instance sets in a row (different counts, sizes and
  depths; the same arrays, so the captured graph is reused): every instance
  against the oracle FMM (FP64, 1e-12) and against its own single evaluation
  (bit for bit, FP64 and mixed);
* a set beyond the plan's capacities, or a malformed one, computes nothing
  and is reported by fmm_get_status (FMM_E_CAPACITY, FMM_E_ARG).
"""
import numpy as np
import pytest

import oracle
from gpu_util import run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _fm():
    import paper_0905_2637_amd as fm
    return fm


def _instances(counts, seed):
    rng = np.random.default_rng(seed)
    xs, ys, gs = [], [], []
    for i, n in enumerate(counts):
        if i % 2 == 1 and n > 10:
            m = n // 2
            x = np.concatenate([rng.random(n - m), 0.3 + 0.01 * rng.standard_normal(m)])
            y = np.concatenate([rng.random(n - m), 0.6 + 0.01 * rng.standard_normal(m)])
        else:
            x, y = rng.random(n), rng.random(n)
        xs.append(np.clip(x, 0.0, np.nextafter(1.0, 0.0)))
        ys.append(np.clip(y, 0.0, np.nextafter(1.0, 0.0)))
        gs.append(rng.uniform(-1.0, 1.0, n))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(gs), off


SETS = [
    ([3000, 700, 0, 1, 2, 5000, 64, 1500, 12000], [4, 3, 2, 0, 1, 5, 2, 3, 6]),
    ([9000, 400, 2500], [5, 2, 4]),
    ([100, 14000, 2048, 33, 6000, 777], [2, 6, 3, 1, 5, 4]),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_plan_three_instance_sets(precision):
    import torch
    fm = _fm()
    n_cap = max(sum(c) for c, _ in SETS)
    leaves = max(sum(4 ** L for L in d) for _, d in SETS)
    bp = fm.BatchPlan(SETS[0][0], SETS[0][1], 0.004, 12, precision=precision, n_max=n_cap,
                      max_instances=max(len(c) for c, _ in SETS), max_depth=6, max_leaves=leaves)
    X, Y, G, U, V = (torch.zeros(n_cap, dtype=torch.float64, device="cuda") for _ in range(5))
    for k, (counts, depths) in enumerate(SETS):
        print(f"instance set {k}: {len(counts)} instances, {sum(counts)} particles", flush=True)
        x, y, g, off = _instances(counts, 80 + k)
        n = len(x)
        X[:n] = torch.as_tensor(x, device="cuda")
        Y[:n] = torch.as_tensor(y, device="cuda")
        G[:n] = torch.as_tensor(g, device="cuda")
        bp.evaluate(X[:n], Y[:n], G[:n], U[:n], V[:n], counts=counts, depths=depths)
        torch.cuda.synchronize()
        u, v = U[:n].cpu().numpy(), V[:n].cpu().numpy()
        for i, (c, L) in enumerate(zip(counts, depths)):
            a, b = off[i], off[i + 1]
            if c == 0:
                continue
            us, vs, sp = run(x[a:b], y[a:b], g[a:b], 0.004, 12, L, precision=precision,
                             fine=min(2, max(0, L - 1)))
            sp.close()
            assert np.array_equal(u[a:b], us) and np.array_equal(v[a:b], vs), f"set {k} instance {i}"
            if precision == "fp64" and c > 1:
                uo, vo = oracle.fmm(x[a:b], y[a:b], g[a:b], 0.004, 12, L)
                err = oracle.rel_l2(u[a:b], v[a:b], uo, vo)
                assert err < FP64_TOL, f"set {k} instance {i}: rel L2 {err:.3e}"
    bp.close()


def test_sets_beyond_capacity_or_malformed_are_reported():
    import torch
    fm = _fm()
    counts, depths = [1000, 2000], [3, 4]
    bp = fm.BatchPlan(counts, depths, 0.004, 12, max_instances=3, max_leaves=4 ** 3 + 4 ** 4)
    x, y, g, off = _instances(counts, 90)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    X, Y, G = dev(x), dev(y), dev(g)
    U, V = torch.zeros_like(X), torch.zeros_like(X)
    bp.evaluate(X, Y, G, U, V)                                  # fits: no error
    cases = [
        ([0, 1000, 3000], [4, 4], fm.FMM_E_CAPACITY),            # 2 * 4^4 leaves > the plan's 4^3 + 4^4
        ([0, 1000, 3000], [3, 7], fm.FMM_E_ARG),                 # deeper than the plan's deepest tree
        ([0, 2000, 1000], [3, 4], fm.FMM_E_ARG),                 # offsets decrease
        ([0, 1000, 3001], [3, 4], fm.FMM_E_CAPACITY),            # more particles than the plan holds
    ]
    for offs, deps, want in cases:
        d_off = torch.tensor(offs, dtype=torch.int64, device="cuda")
        d_dep = torch.tensor(deps, dtype=torch.int32, device="cuda")
        bp.evaluate_csr(2, d_off, d_dep, X, Y, G, U, V, check=False)
        with pytest.raises(fm.FmmError) as ei:
            bp.check_status()
        assert ei.value.status == want, (offs, deps)
    bp.evaluate(X, Y, G, U, V)                                  # and a good set works again
    torch.cuda.synchronize()
    u, v = U.cpu().numpy(), V.cpu().numpy()
    for i, L in enumerate(depths):
        a, b = off[i], off[i + 1]
        uo, vo = oracle.fmm(x[a:b], y[a:b], g[a:b], 0.004, 12, L)
        assert oracle.rel_l2(u[a:b], v[a:b], uo, vo) < FP64_TOL
    bp.close()
