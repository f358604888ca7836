"""A host program using the C ABI alone (paper_0905_2637_amd/examples/
fmm_eval_file.cpp, built next to the library): device memory, stream,
workspace, plan, evaluation and status all through include/fmm.h, with no
Python binding in between.

* on the GPU: its velocities on C1 match the oracle FMM within 1e-12;
* on any host: invalid parameters are refused before the GPU is touched,
  with the status text on stderr.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_0905_2637_amd", "fmm_eval_file")


def _write_input(path, x, y, g):
    with open(path, "wb") as f:
        np.array([len(x)], dtype=np.int64).tofile(f)
        np.concatenate([x, y, g]).astype(np.float64).tofile(f)


def _exe():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    return EXE


def test_invalid_parameters_refused_on_the_host(tmp_path):
    x, y, g = workloads.uniform_square(50, 990)
    src = tmp_path / "in.bin"
    _write_input(src, x, y, g)
    r = subprocess.run([_exe(), str(src), str(tmp_path / "out.bin"), "0.01", "0", "3"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 1
    assert "fmm_workspace_size" in r.stderr and "(-1)" in r.stderr
    assert not (tmp_path / "out.bin").exists()


@pytest.mark.gpu
def test_program_matches_the_oracle(tmp_path):
    oracle.build()
    wl = workloads.make("C1")
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    _write_input(src, wl.x, wl.y, wl.gamma)
    r = subprocess.run([_exe(), str(src), str(dst), repr(wl.sigma), str(wl.p), str(wl.depth)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(dst, dtype=np.float64)
    assert out.shape[0] == 2 * wl.n
    u, v = out[:wl.n], out[wl.n:]
    uo, vo = oracle.fmm(wl.x, wl.y, wl.gamma, wl.sigma, wl.p, wl.depth)
    assert oracle.rel_l2(u, v, uo, vo) < 1e-12
