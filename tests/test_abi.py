"""The C ABI library loads on a CPU-only host, exports every declared entry
point, and validates host-visible arguments synchronously (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_0905_2637_amd as fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fm.LIB_PATH):
        pytest.fail("libfmm_mi355x.so is not built (run __graft_entry__.build())")
    return fm.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "fmm_plan" in names and "fmm_evaluate" in names and "fmm_destroy" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(fm.EXPORTED)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert fm.status_string(s)
    assert lib.fmm_stage_name(0) == b"tree"
    assert lib.fmm_stage_name(99) is None


def _ws(**kw):
    base = dict(n_max=1000, sigma=0.01, p=12, depth=4)
    base.update(kw)
    prm = fm.make_params(base.pop("n_max"), base.pop("sigma"), base.pop("p"), base.pop("depth"), **base)
    out = C.c_size_t(0)
    return fm.load().fmm_workspace_size(C.byref(prm), C.byref(out)), out.value


def test_workspace_size_grows_with_problem(lib):
    s1, b1 = _ws()
    s2, b2 = _ws(n_max=100000)
    s3, b3 = _ws(depth=6)
    s4, b4 = _ws(precision="mixed")
    assert s1 == s2 == s3 == s4 == fm.FMM_OK
    assert b2 > b1 and b3 > b1 and b4 > b1
    # Lambda * p complex values for both ME and LE dominate a deep tree
    s5, b5 = _ws(depth=10, p=20)
    assert b5 >= 2 * 16 * 20 * ((4 ** 11 - 1) // 3)


@pytest.mark.parametrize("kw,err", [
    (dict(sigma=0.0), fm.FMM_E_ARG),
    (dict(sigma=float("nan")), fm.FMM_E_ARG),
    (dict(p=0), fm.FMM_E_ARG),
    (dict(p=33), fm.FMM_E_ARG),
    (dict(depth=-1), fm.FMM_E_ARG),
    (dict(depth=14), fm.FMM_E_ARG),
    (dict(n_max=-5), fm.FMM_E_ARG),
    (dict(n_max=1 << 31), fm.FMM_E_ARG),
    (dict(p=23, precision="mixed"), fm.FMM_E_UNSUPPORTED),
    (dict(depth=4, precision="mixed", fp32_fine_levels=4), fm.FMM_E_ARG),
    (dict(m_max=-1), fm.FMM_E_ARG),
    (dict(m_max=1 << 31), fm.FMM_E_ARG),
    (dict(sigma=1e-31), fm.FMM_E_ARG),                    # Gaussian core below 1e-30
    (dict(domain=(0.0, 0.0, 2e36)), fm.FMM_E_ARG),        # domain wider than 1e36
])
def test_invalid_parameters_rejected(lib, kw, err):
    s, _ = _ws(**kw)
    assert s == err


def test_parameter_limits_are_inclusive(lib):
    """sigma = 1e-30 and width = 1e36 are the last accepted values; the
    singular kernel ignores sigma."""
    assert _ws(sigma=1e-30)[0] == fm.FMM_OK
    assert _ws(domain=(0.0, 0.0, 1e36))[0] == fm.FMM_OK
    assert _ws(sigma=1e-31, kernel="singular")[0] == fm.FMM_OK


def test_kernel_choice(lib):
    # the singular kernel ignores sigma; the Gaussian one needs sigma > 0
    assert _ws(kernel="singular", sigma=0.0)[0] == fm.FMM_OK
    assert _ws(kernel="singular", sigma=float("nan"))[0] == fm.FMM_OK
    assert _ws(kernel="gaussian", sigma=0.0)[0] == fm.FMM_E_ARG
    prm = fm.make_params(100, 0.01, 12, 3)
    prm.kernel = 2
    out = C.c_size_t(0)
    assert lib.fmm_workspace_size(C.byref(prm), C.byref(out)) == fm.FMM_E_ARG


def test_target_capacity_adds_workspace(lib):
    _, b0 = _ws()
    s1, b1 = _ws(m_max=5000)
    assert s1 == fm.FMM_OK and b1 > b0 + 5000 * 32


def test_null_arguments_rejected(lib):
    prm = fm.make_params(100, 0.01, 12, 3)
    h = C.c_void_p()
    assert lib.fmm_workspace_size(C.byref(prm), None) == fm.FMM_E_ARG
    assert lib.fmm_plan(C.byref(prm), None, 1 << 20, None, C.byref(h)) == fm.FMM_E_ARG
    assert lib.fmm_plan(C.byref(prm), C.c_void_p(256), 1 << 20, None, None) == fm.FMM_E_ARG
    # misaligned workspace pointer
    assert lib.fmm_plan(C.byref(prm), C.c_void_p(257), 1 << 30, None, C.byref(h)) == fm.FMM_E_ARG
    # too small a workspace is reported before any device call
    assert lib.fmm_plan(C.byref(prm), C.c_void_p(1 << 20), 16, None, C.byref(h)) == fm.FMM_E_CAPACITY
    assert lib.fmm_evaluate(None, 10, None, None, None, None, None, None) == fm.FMM_E_ARG
    assert lib.fmm_destroy(None) == fm.FMM_OK
    nb = C.c_int64(0)
    assert lib.fmm_get_status(None, None, C.byref(nb)) == fm.FMM_E_ARG


def test_no_cpu_fallback_without_device():
    """The binding refuses to run without a HIP device instead of computing on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        fm.Plan(100, 0.01, 12, 3)


def _ws_batch(n_max, max_instances, depth, max_leaves=0, **kw):
    base = dict(sigma=0.005, p=12)
    base.update(kw)
    prm = fm.make_params(n_max, base.pop("sigma"), base.pop("p"), depth, max_instances=max_instances,
                         max_leaves=max_leaves, **base)
    out = C.c_size_t(0)
    return fm.load().fmm_workspace_size(C.byref(prm), C.byref(out)), out.value


def test_batch_workspace_follows_the_capacities(lib):
    """A batched plan holds the expansions of max_leaves leaf boxes' trees:
    sum Lambda(L_i) <= 4/3 sum 4^L_i boxes, for ME and LE; the default leaf
    capacity is the worst case max_instances * 4^depth."""
    leaves = 4 ** 3 + 4 ** 4 + 4 ** 2
    s, b = _ws_batch(4000, 3, 4, max_leaves=leaves)
    assert s == fm.FMM_OK
    boxes = sum((4 ** (L + 1) - 1) // 3 for L in (3, 4, 2))
    assert b >= 2 * 16 * 12 * boxes
    s1, b1 = _ws_batch(4000, 3, 4)                  # default: 3 * 4^4 leaves
    assert s1 == fm.FMM_OK and b1 > b
    s2, b2 = _ws_batch(4000, 3, 4, max_leaves=4 ** 3)
    assert s2 == fm.FMM_OK and b2 < b


@pytest.mark.parametrize("n_max,max_inst,depth,kw,err", [
    (100, 2, 14, {}, fm.FMM_E_ARG),                                # depth beyond 13
    (-1, 2, 3, {}, fm.FMM_E_ARG),                                  # negative capacity
    (100, 2, 3, dict(max_leaves=-1), fm.FMM_E_ARG),
    (100, 2, 3, dict(domain=None), fm.FMM_E_UNSUPPORTED),          # no explicit square
    (100, 70000, 2, {}, fm.FMM_E_ARG),                             # more than 65536 instances
    (100, 1024, 12, dict(max_leaves=1 << 20), fm.FMM_E_UNSUPPORTED),   # 10 + 24 key bits
    (100, 4, 2, dict(p=23, precision="mixed"), fm.FMM_E_UNSUPPORTED),
    (100, 4, 2, dict(m_max=10), fm.FMM_E_ARG),                     # target points: single plans only
    (100, 4, 2, dict(kernel="gauss-transform", sigma=0.1), fm.FMM_E_UNSUPPORTED),
    (100, -3, 2, {}, fm.FMM_E_ARG),
])
def test_invalid_batches_rejected(lib, n_max, max_inst, depth, kw, err):
    s, _ = _ws_batch(n_max, max_inst, depth, **kw)
    assert s == err


def test_batch_entry_points_reject_null(lib):
    prm = fm.make_params(20, 0.01, 12, 2, max_instances=2)
    h = C.c_void_p()
    assert lib.fmm_plan(C.byref(prm), None, 1 << 20, None, C.byref(h)) == fm.FMM_E_ARG
    assert lib.fmm_plan(C.byref(prm), C.c_void_p(1 << 20), 16, None, C.byref(h)) == fm.FMM_E_CAPACITY
    assert lib.fmm_evaluate_batch(None, 1, None, None, None, None, None, None, None, None) == fm.FMM_E_ARG
    assert lib.fmm_set_tuning(None, 4, 8, 1, 1, 0, None) == fm.FMM_E_ARG
    assert lib.fmm_work_estimate(None, None, 0, None) == fm.FMM_E_ARG
    assert lib.fmm_autotune(None, 10, None, None, None, None, None, None, 3) == fm.FMM_E_ARG
    w = C.c_int32(0)
    assert lib.fmm_get_tuning(None, C.byref(w), C.byref(w), C.byref(w), C.byref(w), C.byref(w)) == fm.FMM_E_ARG


def test_advance_rejects_bad_arguments(lib):
    assert lib.fmm_advance_rk2(None, 10, None, None, None, 1e-3, 1, None, None) == fm.FMM_E_ARG


def test_params_layout_and_enums_match_the_header(tmp_path):
    """fmm_params as the C compiler lays it out (field offsets and size) and
    the enum values of the header agree with the Python binding's mirror."""
    import subprocess
    fields = [f for f, _ in fm.FmmParams._fields_]
    enums = ["FMM_OK", "FMM_E_ARG", "FMM_E_CAPACITY", "FMM_E_DOMAIN", "FMM_E_NOMEM", "FMM_E_DEVICE",
             "FMM_E_UNSUPPORTED", "FMM_PREC_FP64", "FMM_PREC_MIXED", "FMM_KERNEL_GAUSSIAN", "FMM_KERNEL_SINGULAR",
             "FMM_KERNEL_LENNARD_JONES", "FMM_KERNEL_GAUSS_TRANSFORM", "FMM_DUMP_KEYS", "FMM_DUMP_PERM",
             "FMM_DUMP_LEAF_START", "FMM_DUMP_ME", "FMM_DUMP_LE", "FMM_DUMP_DOMAIN", "FMM_DUMP_ILIST",
             "FMM_DUMP_TKEYS", "FMM_DUMP_TPERM", "FMM_DUMP_TLEAF_START"]
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {",
           '  printf("size %zu\\n", sizeof(fmm_params));']
    src += [f'  printf("{f} %zu\\n", offsetof(fmm_params, {f}));' for f in fields]
    src += [f'  printf("{e} %d\\n", (int){e});' for e in enums]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-o", str(exe), str(c)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["size"]) == C.sizeof(fm.FmmParams)
    for f in fields:
        assert int(out[f]) == getattr(fm.FmmParams, f).offset, f
    py = {"FMM_OK": fm.FMM_OK, "FMM_E_ARG": fm.FMM_E_ARG, "FMM_E_CAPACITY": fm.FMM_E_CAPACITY,
          "FMM_E_DOMAIN": fm.FMM_E_DOMAIN, "FMM_E_NOMEM": fm.FMM_E_NOMEM, "FMM_E_DEVICE": fm.FMM_E_DEVICE,
          "FMM_E_UNSUPPORTED": fm.FMM_E_UNSUPPORTED, "FMM_PREC_FP64": fm.FMM_PREC_FP64,
          "FMM_PREC_MIXED": fm.FMM_PREC_MIXED, "FMM_KERNEL_GAUSSIAN": fm.FMM_KERNEL_GAUSSIAN,
          "FMM_KERNEL_SINGULAR": fm.FMM_KERNEL_SINGULAR, "FMM_KERNEL_LENNARD_JONES": fm.FMM_KERNEL_LENNARD_JONES,
          "FMM_KERNEL_GAUSS_TRANSFORM": fm.FMM_KERNEL_GAUSS_TRANSFORM, "FMM_DUMP_KEYS": fm.DUMP_KEYS,
          "FMM_DUMP_PERM": fm.DUMP_PERM, "FMM_DUMP_LEAF_START": fm.DUMP_LEAF_START, "FMM_DUMP_ME": fm.DUMP_ME,
          "FMM_DUMP_LE": fm.DUMP_LE, "FMM_DUMP_DOMAIN": fm.DUMP_DOMAIN, "FMM_DUMP_ILIST": fm.DUMP_ILIST,
          "FMM_DUMP_TKEYS": fm.DUMP_TKEYS, "FMM_DUMP_TPERM": fm.DUMP_TPERM,
          "FMM_DUMP_TLEAF_START": fm.DUMP_TLEAF_START}
    for e in enums:
        assert int(out[e]) == py[e], e
