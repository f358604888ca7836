"""The 3D entry points on the host: fmm3d_params as the C compiler lays it
out, workspace sizes, parameter and NULL checks, and no CPU path without a
device.  No GPU needed."""
import ctypes as C
import os
import subprocess

import pytest

import paper_0905_2637_amd as fm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fmm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fm.LIB_PATH):
        pytest.fail("libfmm_mi355x.so is not built (run __graft_entry__.build())")
    return fm.load()


def _ws(lib, **kw):
    prm = dict(n_max=1000, p=6, depth=3, x0=0.0, y0=0.0, z0=0.0, width=1.0)
    prm.update(kw)
    out = C.c_size_t(0)
    s = lib.fmm3d_workspace_size(C.byref(fm.Fmm3dParams(**prm)), C.byref(out))
    return s, out.value


def test_params_layout_matches_the_header(tmp_path):
    fields = [f for f, _ in fm.Fmm3dParams._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {",
           '  printf("size %zu\\n", sizeof(fmm3d_params));']
    src += [f'  printf("{f} %zu\\n", offsetof(fmm3d_params, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout3.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout3"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-o", str(exe), str(c)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["size"]) == C.sizeof(fm.Fmm3dParams)
    for f in fields:
        assert int(out[f]) == getattr(fm.Fmm3dParams, f).offset, f


def test_workspace_grows_with_depth_p_and_n(lib):
    s, base = _ws(lib)
    assert s == fm.FMM_OK and base > 0
    assert _ws(lib, depth=4)[1] > base
    # more terms need more room (p >= 1 also holds the derivatives as dense
    # (2p+1)^3 cubes for the lane M2L)
    assert _ws(lib, p=5)[1] < base < _ws(lib, p=8)[1] < _ws(lib, p=9)[1]
    assert _ws(lib, p=0)[1] < _ws(lib, p=1)[1]
    assert _ws(lib, n_max=100000)[1] > base
    # coefficient storage dominates at depth 7, p = 9: 2 * (8^8 - 1) / 7 boxes * 220 terms * 8 B
    s, big = _ws(lib, depth=7, p=9, n_max=1 << 24)
    assert s == fm.FMM_OK and big > 2 * ((8 ** 8 - 1) // 7) * 220 * 8


@pytest.mark.parametrize("kw,err", [
    (dict(p=-1), fm.FMM_E_ARG), (dict(depth=-1), fm.FMM_E_ARG), (dict(n_max=-1), fm.FMM_E_ARG),
    (dict(n_max=1 << 31), fm.FMM_E_ARG), (dict(width=0.0), fm.FMM_E_ARG), (dict(width=float("inf")), fm.FMM_E_ARG),
    (dict(x0=float("nan")), fm.FMM_E_ARG), (dict(z0=float("inf")), fm.FMM_E_ARG),
    (dict(p=10), fm.FMM_E_UNSUPPORTED), (dict(depth=8), fm.FMM_E_UNSUPPORTED),
])
def test_invalid_parameters_rejected(lib, kw, err):
    assert _ws(lib, **kw)[0] == err


def test_null_arguments(lib):
    prm = fm.Fmm3dParams(100, 4, 2, 0.0, 0.0, 0.0, 1.0)
    out = C.c_size_t(0)
    assert lib.fmm3d_workspace_size(None, C.byref(out)) == fm.FMM_E_ARG
    assert lib.fmm3d_workspace_size(C.byref(prm), None) == fm.FMM_E_ARG
    h = C.c_void_p()
    assert lib.fmm3d_plan(C.byref(prm), None, 1 << 20, None, C.byref(h)) == fm.FMM_E_ARG
    assert lib.fmm3d_plan(C.byref(prm), C.c_void_p(256), 1 << 20, None, None) == fm.FMM_E_ARG
    assert lib.fmm3d_plan(C.byref(prm), C.c_void_p(257), 1 << 30, None, C.byref(h)) == fm.FMM_E_ARG
    assert lib.fmm3d_plan(C.byref(prm), C.c_void_p(256), 16, None, C.byref(h)) == fm.FMM_E_CAPACITY
    assert lib.fmm3d_evaluate(None, 0, *([None] * 9)) == fm.FMM_E_ARG
    v = C.c_int64(0)
    assert lib.fmm3d_get_status(None, None, C.byref(v)) == fm.FMM_E_ARG
    assert lib.fmm3d_destroy(None) == fm.FMM_OK


def test_no_cpu_path_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(RuntimeError):
        fm.Plan3D(100, 4, 2)


@pytest.mark.parametrize("p", range(1, 10))
def test_workspace_holds_the_derivative_cubes_of_the_lane_m2l(lib, p):
    """The lane M2L (every p from 1 to 9) reads the derivative cubes
    343 x (2p+1)^3 from the workspace: it must hold them on top of the
    moments, locals and graded derivative table."""
    L = 3
    nbox = (8 ** (L + 1) - 1) // 7
    T, T2, S = (p + 1) * (p + 2) * (p + 3) // 6, (2 * p + 1) * (2 * p + 2) * (2 * p + 3) // 6, 2 * p + 1
    s, size = _ws(lib, p=p, depth=L, n_max=1)
    assert s == fm.FMM_OK
    assert size >= 8 * (2 * nbox * T + 343 * T2 + 343 * S ** 3)
