"""MI355X 2D vortex-particle FMM: thin ctypes binding over libfmm_mi355x.so.

Every step of an evaluation runs in the library's HIP kernels; this module
only marshals PyTorch device tensors (memory and streams) across the C ABI
declared in ``include/fmm.h``.  There is no CPU fallback: if the library is
not built, or no HIP device is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_mi355x.so")

FMM_OK = 0
FMM_E_ARG = -1
FMM_E_CAPACITY = -2
FMM_E_DOMAIN = -3
FMM_E_NOMEM = -4
FMM_E_DEVICE = -5
FMM_E_UNSUPPORTED = -6
FMM_KERNEL_GAUSSIAN, FMM_KERNEL_SINGULAR, FMM_KERNEL_LENNARD_JONES, FMM_KERNEL_GAUSS_TRANSFORM = 0, 1, 2, 3
KERNELS = {"gaussian": FMM_KERNEL_GAUSSIAN, "singular": FMM_KERNEL_SINGULAR,
           "lennard-jones": FMM_KERNEL_LENNARD_JONES, "gauss-transform": FMM_KERNEL_GAUSS_TRANSFORM}

FMM_PREC_FP64 = 0
FMM_PREC_MIXED = 1

DUMP_KEYS, DUMP_PERM, DUMP_LEAF_START, DUMP_ME, DUMP_LE, DUMP_DOMAIN, DUMP_ILIST = range(7)
DUMP_TKEYS, DUMP_TPERM, DUMP_TLEAF_START = range(7, 10)

EXPORTED = ["fmm_workspace_size", "fmm_plan", "fmm_evaluate", "fmm_evaluate_at", "fmm_evaluate_batch", "fmm_advance_rk2", "fmm_get_status", "fmm_set_timing", "fmm_stats", "fmm_stage_name",
            "fmm_get_tuning", "fmm_set_tuning", "fmm_autotune", "fmm_autotune_report", "fmm_work_estimate", "fmm_debug_dump", "fmm_destroy",
            "fmm_status_string", "fmm3d_workspace_size", "fmm3d_plan", "fmm3d_evaluate", "fmm3d_get_status",
            "fmm3d_debug_dump", "fmm3d_destroy", "fmm_evaluate_static"]

# Inspection aid: when set to a byte value, every new plan's workspace is
# filled with it before the plan is made (results must not depend on what
# the workspace held before).
WORKSPACE_FILL = None

# bytes of the fixed device array behind fmm_evaluate_static (FMM_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 64 << 20


class Fmm3dParams(C.Structure):
    _fields_ = [("n_max", C.c_int64), ("p", C.c_int32), ("depth", C.c_int32), ("x0", C.c_double),
                ("y0", C.c_double), ("z0", C.c_double), ("width", C.c_double)]


class FmmParams(C.Structure):
    _fields_ = [("n_max", C.c_int64), ("sigma", C.c_double), ("p", C.c_int32), ("depth", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("width", C.c_double),
                ("precision", C.c_int32), ("fp32_fine_levels", C.c_int32), ("m_max", C.c_int64),
                ("kernel", C.c_int32), ("lj_epsilon", C.c_double), ("cutoff", C.c_double),
                ("max_instances", C.c_int32), ("max_leaves", C.c_int64)]


class FmmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_0905_2637_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.fmm_workspace_size.argtypes = [C.POINTER(FmmParams), C.POINTER(C.c_size_t)]
    lib.fmm_plan.argtypes = [C.POINTER(FmmParams), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.fmm_evaluate.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp]
    lib.fmm_evaluate_at.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp]
    i32p = C.POINTER(C.c_int32)
    lib.fmm_evaluate_batch.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_advance_rk2.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, C.c_int32, vp, vp]
    lib.fmm_get_tuning.argtypes = [vp, i32p, i32p, i32p, i32p, i32p]
    lib.fmm_set_tuning.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
    lib.fmm_work_estimate.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, i32p]
    lib.fmm_autotune.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_int32]
    lib.fmm_autotune_report.argtypes = [vp, i32p, C.POINTER(C.c_double)]
    lib.fmm_get_status.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    lib.fmm_set_timing.argtypes = [vp, C.c_int32]
    lib.fmm_stats.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int64)]
    lib.fmm_stage_name.argtypes = [C.c_int32]
    lib.fmm_stage_name.restype = C.c_char_p
    lib.fmm_debug_dump.argtypes = [vp, C.c_int32, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.fmm_destroy.argtypes = [vp]
    lib.fmm_status_string.argtypes = [C.c_int]
    lib.fmm_status_string.restype = C.c_char_p
    lib.fmm3d_workspace_size.argtypes = [C.POINTER(Fmm3dParams), C.POINTER(C.c_size_t)]
    lib.fmm3d_plan.argtypes = [C.POINTER(Fmm3dParams), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.fmm3d_evaluate.argtypes = [vp, C.c_int64] + [vp] * 9
    lib.fmm3d_get_status.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    lib.fmm3d_destroy.argtypes = [vp]
    lib.fmm3d_debug_dump.argtypes = [vp, C.c_int32, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.fmm_evaluate_static.argtypes = [C.POINTER(FmmParams), C.c_int64, vp, vp, vp, vp, vp, vp]
    for name in EXPORTED:
        if name in ("fmm_stage_name", "fmm_status_string"):
            continue
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().fmm_status_string(int(s)).decode()


def make_params(n_max, sigma, p, depth, domain=(0.0, 0.0, 1.0), precision="fp64", fp32_fine_levels=2, m_max=0,
                kernel="gaussian", lj_epsilon=0.0, cutoff=0.0, max_instances=0, max_leaves=0):
    if domain is None:
        x0, y0, w = 0.0, 0.0, 0.0
    else:
        x0, y0, w = domain
    prec = {"fp64": FMM_PREC_FP64, "mixed": FMM_PREC_MIXED}[precision]
    return FmmParams(int(n_max), float(sigma), int(p), int(depth), float(x0), float(y0), float(w), prec,
                     int(fp32_fine_levels if precision == "mixed" else 0), int(m_max), KERNELS[kernel],
                     float(lj_epsilon), float(cutoff), int(max_instances), int(max_leaves))


def workspace_size(prm: FmmParams) -> int:
    out = C.c_size_t(0)
    s = load().fmm_workspace_size(C.byref(prm), C.byref(out))
    if s != FMM_OK:
        raise FmmError(s, "fmm_workspace_size")
    return int(out.value)


def _stream_handle(stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


def _check_inputs(n, tensors):
    import torch
    for t in tensors:
        if t.dtype != torch.float64 or t.device.type != "cuda" or not t.is_contiguous() or t.shape[0] != n:
            raise ValueError(f"inputs and outputs must be contiguous float64 CUDA tensors of length {n}")


def evaluate_static(x, y, gamma, sigma, p, depth, domain=(0.0, 0.0, 1.0), precision="fp64", fp32_fine_levels=2,
                    kernel="gaussian", n_max=None, u=None, v=None):
    """One evaluation through fmm_evaluate_static: the library's fixed device
    array serves as the workspace, so nothing is allocated for it (u and v are
    allocated here when not given)."""
    import torch
    n = int(x.shape[0])
    if u is None:
        u = torch.empty(n, dtype=torch.float64, device=x.device)
    if v is None:
        v = torch.empty(n, dtype=torch.float64, device=x.device)
    _check_inputs(n, (x, y, gamma, u, v))
    prm = make_params(n if n_max is None else n_max, sigma, p, depth, domain, precision, fp32_fine_levels,
                      kernel=kernel)
    s = load().fmm_evaluate_static(C.byref(prm), n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                   C.c_void_p(gamma.data_ptr()), C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                   _stream_handle())
    if s != FMM_OK:
        raise FmmError(s, "fmm_evaluate_static")
    return u, v


class _PlanBase:
    """Shared handle management, status, timing, tuning and inspection."""

    _h = None

    def _alloc_workspace(self, nbytes):
        import torch
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if WORKSPACE_FILL is not None:
            self.workspace.fill_(int(WORKSPACE_FILL))
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self._ws_bytes = nbytes

    def out_of_domain(self) -> int:
        out = C.c_int64(0)
        s = load().fmm_get_status(self._h, _stream_handle(), C.byref(out))
        if s not in (FMM_OK, FMM_E_DOMAIN):
            raise FmmError(s, "fmm_get_status")
        return int(out.value)

    def set_timing(self, on=True):
        s = load().fmm_set_timing(self._h, 1 if on else 0)
        if s != FMM_OK:
            raise FmmError(s, "fmm_set_timing")

    def stats(self) -> dict:
        """Average GPU milliseconds per stage over the evaluations timed since set_timing(True)."""
        buf = (C.c_double * 16)()
        nw = C.c_int32(0)
        ne = C.c_int64(0)
        s = load().fmm_stats(self._h, buf, 16, C.byref(nw), C.byref(ne))
        if s != FMM_OK:
            raise FmmError(s, "fmm_stats")
        lib = load()
        out = {lib.fmm_stage_name(i).decode(): float(buf[i]) for i in range(nw.value)}
        out["evaluations"] = int(ne.value)
        return out

    def tuning(self) -> dict:
        w, sm, mf, wo, bk = (C.c_int32(0) for _ in range(5))
        s = load().fmm_get_tuning(self._h, C.byref(w), C.byref(sm), C.byref(mf), C.byref(wo), C.byref(bk))
        if s != FMM_OK:
            raise FmmError(s, "fmm_get_tuning")
        return {"p2p_waves": int(w.value), "m2l_split_max": int(sm.value), "m2l_mfma": int(mf.value),
                "work_order": int(wo.value), "p2p_block": int(bk.value)}

    def set_tuning(self, p2p_waves=None, m2l_split_max=None, m2l_mfma=None, work_order=None, p2p_block=None):
        """Sets the given launch-shape knobs; those left None keep their value."""
        t = self.tuning()
        given = dict(p2p_waves=p2p_waves, m2l_split_max=m2l_split_max, m2l_mfma=m2l_mfma, work_order=work_order,
                     p2p_block=p2p_block)
        t.update({k: int(v) for k, v in given.items() if v is not None})
        s = load().fmm_set_tuning(self._h, t["p2p_waves"], t["m2l_split_max"], t["m2l_mfma"], t["work_order"],
                                  t["p2p_block"], _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm_set_tuning")

    def autotune_report(self) -> dict:
        """Candidates the last autotune timed, and the work model's near-field share."""
        t, sh = C.c_int32(0), C.c_double(0.0)
        s = load().fmm_autotune_report(self._h, C.byref(t), C.byref(sh))
        if s != FMM_OK:
            raise FmmError(s, "fmm_autotune_report")
        return {"candidates_timed": int(t.value), "near_share": float(sh.value)}

    def work_estimate(self) -> np.ndarray:
        """The paper's work model (eqs. 13-15) per instance, in input order."""
        n = len(getattr(self, "counts", [0]))
        out = (C.c_double * n)()
        nw = C.c_int32(0)
        s = load().fmm_work_estimate(self._h, out, n, C.byref(nw))
        if s != FMM_OK:
            raise FmmError(s, "fmm_work_estimate")
        return np.array(out[: nw.value])

    def dump(self, what: int) -> np.ndarray:
        lib = load()
        need = C.c_size_t(0)
        lib.fmm_debug_dump(self._h, what, None, 0, C.byref(need))
        dtype = {DUMP_KEYS: np.uint32, DUMP_PERM: np.uint32, DUMP_LEAF_START: np.int32,
                 DUMP_ME: np.complex128, DUMP_LE: np.complex128, DUMP_DOMAIN: np.float64,
                 DUMP_ILIST: np.int32, DUMP_TKEYS: np.uint32, DUMP_TPERM: np.uint32,
                 DUMP_TLEAF_START: np.int32}[what]
        arr = np.zeros(max(1, need.value // np.dtype(dtype).itemsize), dtype=dtype)
        s = lib.fmm_debug_dump(self._h, what, C.c_void_p(arr.ctypes.data), C.c_size_t(arr.nbytes), C.byref(need))
        if s != FMM_OK:
            raise FmmError(s, "fmm_debug_dump")
        arr = arr[: need.value // np.dtype(dtype).itemsize]
        if what in (DUMP_ME, DUMP_LE):
            arr = arr.reshape(-1, self.p)
        if what == DUMP_ILIST:
            arr = arr.reshape(-1, 27)
        return arr

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().fmm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan(_PlanBase):
    """One FMM configuration bound to a device workspace.

    Parameters follow the paper's problem statement: core size ``sigma``,
    expansion order ``p`` and tree ``depth``; ``domain`` = (x0, y0, width) of
    the square, or None for the particles' bounding square at every call.
    ``m_max`` > 0 reserves room for that many target points (``evaluate_at``).
    ``kernel`` = "gaussian" (eq. 8, core ``sigma``) or "singular" (eq. 7,
    point vortices; ``sigma`` ignored) for the near field, or
    "lennard-jones" (length ``sigma``, energy ``lj_epsilon``, ``cutoff`` at
    most the leaf width): ``evaluate`` then returns the forces; or
    "gauss-transform" (``evaluate`` and ``evaluate_at`` return the Gauss
    transform with width ``sigma`` in u, and zeros in v; p <= 16 Hermite
    terms per axis).
    """

    def __init__(self, n_max, sigma, p, depth, domain=(0.0, 0.0, 1.0), precision="fp64",
                 fp32_fine_levels=2, device="cuda", m_max=0, kernel="gaussian", lj_epsilon=0.0, cutoff=0.0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the FMM runs only on the GPU")
        self.params = make_params(n_max, sigma, p, depth, domain, precision, fp32_fine_levels, m_max, kernel,
                                  lj_epsilon, cutoff)
        self.n_max = int(n_max)
        self.m_max = int(m_max)
        self.depth = int(depth)
        self.p = int(p)
        self.precision = precision
        self.device = torch.device(device)
        self._alloc_workspace(workspace_size(self.params))
        handle = C.c_void_p()
        s = load().fmm_plan(C.byref(self.params), C.c_void_p(self._ws_ptr), C.c_size_t(self._ws_bytes),
                            _stream_handle(), C.byref(handle))
        if s != FMM_OK:
            raise FmmError(s, "fmm_plan")
        self._h = handle
        self.last_n = 0

    def _outputs(self, x, u, v):
        import torch
        n = int(x.shape[0])
        if u is None:
            u = torch.empty(n, dtype=torch.float64, device=x.device)
        if v is None:
            v = torch.empty(n, dtype=torch.float64, device=x.device)
        return u, v

    def evaluate(self, x, y, gamma, u=None, v=None, check=True):
        """Velocity (u, v) of eq. 9 at every particle (with the Lennard-Jones
        kernel: the force); FP64 device tensors."""
        n = int(x.shape[0])
        u, v = self._outputs(x, u, v)
        _check_inputs(n, (x, y, gamma, u, v))
        s = load().fmm_evaluate(self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                C.c_void_p(gamma.data_ptr()), C.c_void_p(u.data_ptr()),
                                C.c_void_p(v.data_ptr()), _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm_evaluate")
        self.last_n = n
        if check:
            nbad = self.out_of_domain()
            if nbad:
                raise FmmError(FMM_E_DOMAIN, f"fmm_evaluate: {nbad} particles outside the domain")
        return u, v

    def evaluate_at(self, x, y, gamma, tx, ty, u=None, v=None, check=True):
        """Velocity (u, v) at the target points (tx, ty) induced by the
        particles (eq. 1 with distinct targets); FP64 device tensors."""
        n, m = int(x.shape[0]), int(tx.shape[0])
        u, v = self._outputs(tx, u, v)
        _check_inputs(n, (x, y, gamma))
        _check_inputs(m, (tx, ty, u, v))
        s = load().fmm_evaluate_at(self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                   C.c_void_p(gamma.data_ptr()), m, C.c_void_p(tx.data_ptr()),
                                   C.c_void_p(ty.data_ptr()), C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                   _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm_evaluate_at")
        self.last_n = n
        if check:
            nbad = self.out_of_domain()
            if nbad:
                raise FmmError(FMM_E_DOMAIN, f"fmm_evaluate_at: {nbad} particles or points outside the domain")
        return u, v

    def advance_rk2(self, x, y, gamma, dt, steps, scratch=None):
        """Move the particles (x, y updated in place) by `steps` explicit
        midpoint steps of the vortex method (Section 3, eq. 6)."""
        import torch
        n = int(x.shape[0])
        if scratch is None:
            scratch = torch.empty(4 * max(n, 1), dtype=torch.float64, device=x.device)
        _check_inputs(n, (x, y, gamma))
        if scratch.dtype != torch.float64 or not scratch.is_contiguous() or scratch.numel() < 4 * n:
            raise ValueError("scratch must be a contiguous float64 tensor of at least 4 n elements")
        s = load().fmm_advance_rk2(self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                   C.c_void_p(gamma.data_ptr()), float(dt), int(steps),
                                   C.c_void_p(scratch.data_ptr()), _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm_advance_rk2")
        self.last_n = n
        return x, y

    def autotune(self, x, y, gamma, u=None, v=None, reps=3) -> dict:
        """Time the launch-shape candidates on these inputs and keep the fastest."""
        n = int(x.shape[0])
        u, v = self._outputs(x, u, v)
        _check_inputs(n, (x, y, gamma, u, v))
        s = load().fmm_autotune(self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                C.c_void_p(gamma.data_ptr()), C.c_void_p(u.data_ptr()),
                                C.c_void_p(v.data_ptr()), _stream_handle(), int(reps))
        if s != FMM_OK:
            raise FmmError(s, "fmm_autotune")
        return self.tuning()


class BatchPlan(_PlanBase):
    """Many independent FMM problems evaluated together (fmm_evaluate_batch:
    the instance table on the device, one table kernel and one graph replay).

    ``counts[i]`` particles of instance i follow those of instances 0..i-1
    in the concatenated input arrays; instance i uses tree depth
    ``depths[i]``.  All instances share ``sigma``, ``p``, the precision, the
    near-field ``kernel`` and the explicit square ``domain`` = (x0, y0, width).
    The plan holds capacities only -- ``n_max`` particles, ``max_instances``
    instances, trees no deeper than ``max_depth``, ``max_leaves`` leaf boxes
    in total (by default those of the first instance set) -- and every
    ``evaluate`` may bring another instance set (``counts``, ``depths``).
    """

    def __init__(self, counts, depths, sigma, p, domain=(0.0, 0.0, 1.0), precision="fp64",
                 fp32_fine_levels=2, device="cuda", kernel="gaussian", lj_epsilon=0.0, cutoff=0.0,
                 n_max=None, max_instances=None, max_depth=None, max_leaves=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the FMM runs only on the GPU")
        if domain is None:
            raise ValueError("a batched plan needs an explicit square domain")
        counts = [int(c) for c in counts]
        depths = [int(d) for d in depths]
        self.p = int(p)
        self.precision = precision
        self.device = torch.device(device)
        self.n_max = int(n_max) if n_max is not None else sum(counts)
        self.max_instances = int(max_instances) if max_instances is not None else len(counts)
        self.max_depth = int(max_depth) if max_depth is not None else max(depths)
        self.max_leaves = int(max_leaves) if max_leaves is not None else sum(4 ** d for d in depths)
        self.params = make_params(self.n_max, sigma, p, self.max_depth, domain, precision, fp32_fine_levels,
                                  kernel=kernel, lj_epsilon=lj_epsilon, cutoff=cutoff,
                                  max_instances=max(2, self.max_instances), max_leaves=self.max_leaves)
        self._alloc_workspace(workspace_size(self.params))
        handle = C.c_void_p()
        s = load().fmm_plan(C.byref(self.params), C.c_void_p(self._ws_ptr), C.c_size_t(self._ws_bytes),
                            _stream_handle(), C.byref(handle))
        if s != FMM_OK:
            raise FmmError(s, "fmm_plan")
        self._h = handle
        self.set_instances(counts, depths)

    def set_instances(self, counts, depths):
        """The instance set of the following evaluations (uploaded to the device)."""
        import torch
        if len(counts) != len(depths) or not 1 <= len(counts) <= max(2, self.max_instances):
            raise ValueError("counts and depths: 1 .. max_instances instances of equal length")
        self.counts = [int(c) for c in counts]
        self.depths = [int(d) for d in depths]
        self.n = sum(self.counts)
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self._d_offsets = torch.as_tensor(self.offsets, device=self.device)
        self._d_depths = torch.as_tensor(np.asarray(self.depths, np.int32), device=self.device)

    def _outputs(self, u, v):
        import torch
        if u is None:
            u = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if v is None:
            v = torch.empty(self.n, dtype=torch.float64, device=self.device)
        return u, v

    def evaluate(self, x, y, gamma, u=None, v=None, check=True, counts=None, depths=None):
        """Velocities of every instance, concatenated like the inputs; with
        counts and depths, of that instance set (kept for later calls)."""
        if counts is not None or depths is not None:
            self.set_instances(counts, depths)
        u, v = self._outputs(u, v)
        _check_inputs(self.n, (x, y, gamma, u, v))
        return self.evaluate_csr(len(self.counts), self._d_offsets, self._d_depths, x, y, gamma, u, v, check)

    def evaluate_csr(self, n_inst, d_offsets, d_depths, x, y, gamma, u, v, check=True):
        """fmm_evaluate_batch with a caller's device instance table: int64
        offsets [n_inst + 1] and int32 depths [n_inst] (device tensors)."""
        import torch
        if d_offsets.dtype != torch.int64 or d_depths.dtype != torch.int32:
            raise ValueError("offsets must be int64 and depths int32 device tensors")
        s = load().fmm_evaluate_batch(self._h, int(n_inst), C.c_void_p(d_offsets.data_ptr()),
                                      C.c_void_p(d_depths.data_ptr()), C.c_void_p(x.data_ptr()),
                                      C.c_void_p(y.data_ptr()), C.c_void_p(gamma.data_ptr()),
                                      C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()), _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm_evaluate_batch")
        if check:
            self.check_status()
        return u, v

    def check_status(self):
        """Raise if the last call's instance set was rejected or had particles
        outside the square (synchronises)."""
        out = C.c_int64(0)
        s = load().fmm_get_status(self._h, _stream_handle(), C.byref(out))
        if s == FMM_E_DOMAIN:
            raise FmmError(s, f"fmm_evaluate_batch: {int(out.value)} particles outside the domain")
        if s != FMM_OK:
            raise FmmError(s, "fmm_evaluate_batch")

    def dump(self, what: int) -> np.ndarray:
        """As for a single plan; KEYS and PERM cut to the current instances'
        particles, LEAF_START to their segments."""
        out = super().dump(what)
        if what in (DUMP_KEYS, DUMP_PERM):
            return out[:self.n]
        if what == DUMP_LEAF_START:
            return out[:sum(4 ** d + 1 for d in self.depths)]
        return out

    def autotune(self, x, y, gamma, u=None, v=None, reps=3) -> dict:
        """Time the launch-shape candidates on the current instance set."""
        u, v = self._outputs(u, v)
        _check_inputs(self.n, (x, y, gamma, u, v))
        self.evaluate(x, y, gamma, u, v, check=False)      # the set the tuner re-times
        s = load().fmm_autotune(self._h, self.n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                C.c_void_p(gamma.data_ptr()), C.c_void_p(u.data_ptr()),
                                C.c_void_p(v.data_ptr()), _stream_handle(), int(reps))
        if s != FMM_OK:
            raise FmmError(s, "fmm_autotune")
        return self.tuning()


class Plan3D:
    """The 3D form (octree, Laplace kernel 1/r, Cartesian Taylor expansions of
    total degree ``p`` <= 9, ``depth`` <= 7) bound to a device workspace.
    ``evaluate`` returns the potential and its gradient at every particle of
    the cube ``origin`` + [0, ``width``)^3."""

    def __init__(self, n_max, p, depth, origin=(0.0, 0.0, 0.0), width=1.0, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the FMM runs only on the GPU")
        self.params = Fmm3dParams(int(n_max), int(p), int(depth), float(origin[0]), float(origin[1]),
                                  float(origin[2]), float(width))
        self.n_max, self.p, self.depth = int(n_max), int(p), int(depth)
        self.device = torch.device(device)
        lib = load()
        nbytes = C.c_size_t(0)
        s = lib.fmm3d_workspace_size(C.byref(self.params), C.byref(nbytes))
        if s != FMM_OK:
            raise FmmError(s, "fmm3d_workspace_size")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = (self.workspace.data_ptr() + 255) & ~255
        handle = C.c_void_p()
        s = lib.fmm3d_plan(C.byref(self.params), C.c_void_p(base), nbytes, _stream_handle(), C.byref(handle))
        if s != FMM_OK:
            raise FmmError(s, "fmm3d_plan")
        self._h = handle

    def evaluate(self, x, y, z, q, out=None, check=True):
        """(phi, dphi/dx, dphi/dy, dphi/dz) at every particle; FP64 device tensors."""
        import torch
        n = int(x.shape[0])
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float64, device=x.device) for _ in range(4))
        _check_inputs(n, (x, y, z, q) + tuple(out))
        s = load().fmm3d_evaluate(self._h, n, *(C.c_void_p(t.data_ptr()) for t in (x, y, z, q) + tuple(out)),
                                  _stream_handle())
        if s != FMM_OK:
            raise FmmError(s, "fmm3d_evaluate")
        if check and self.out_of_domain():
            raise FmmError(FMM_E_DOMAIN, "fmm3d_evaluate")
        return out

    def dump(self, what: int) -> np.ndarray:
        """Keys, permutation or leaf ranges of the last evaluation (DUMP_KEYS,
        DUMP_PERM, DUMP_LEAF_START)."""
        lib = load()
        need = C.c_size_t(0)
        lib.fmm3d_debug_dump(self._h, what, None, 0, C.byref(need))
        dtype = np.int32 if what == DUMP_LEAF_START else np.uint32
        arr = np.zeros(max(1, need.value // 4), dtype=dtype)
        s = lib.fmm3d_debug_dump(self._h, what, C.c_void_p(arr.ctypes.data), C.c_size_t(arr.nbytes), C.byref(need))
        if s != FMM_OK:
            raise FmmError(s, "fmm3d_debug_dump")
        return arr[: need.value // 4]

    def out_of_domain(self) -> int:
        v = C.c_int64(0)
        s = load().fmm3d_get_status(self._h, _stream_handle(), C.byref(v))
        if s not in (FMM_OK, FMM_E_DOMAIN):
            raise FmmError(s, "fmm3d_get_status")
        return int(v.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().fmm3d_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
