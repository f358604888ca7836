"""Plain FP64 CPU oracle for the 2D vortex-particle FMM (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library never does: it shares
no code, header, table or helper with the oracle.

The arithmetic lives in ``fmm_oracle.c`` (see its header for the passages of
the paper each function follows); this module only marshals numpy arrays
through ctypes.  ``build()`` compiles the C file with gcc.

Every sum and FMM takes the Gaussian core size ``sigma``; ``sigma = 0``
selects the singular kernel of eq. 7 (point vortices) for every pair.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_SRC3 = os.path.join(_HERE, "fmm3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build() -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (always rebuilds)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fcx-limited-range",
           "-fPIC", "-shared", "-std=gnu11", "-Wall", "-o", _LIB + ".tmp", _SRC, _SRC3,
           "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    i64 = C.c_int64
    i32p = C.POINTER(C.c_int32)
    u32p = C.POINTER(C.c_uint32)
    i64p = C.POINTER(C.c_int64)
    lib.oracle_init.restype = C.c_int
    lib.oracle_threads.restype = C.c_int
    lib.oracle_bounding_square.argtypes = [i64, dp, dp, dp]
    lib.oracle_quantize.argtypes = [i64, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double, i32p, i32p]
    lib.oracle_quantize.restype = i64
    lib.oracle_morton.argtypes = [C.c_uint32, C.c_uint32]
    lib.oracle_morton.restype = C.c_uint32
    lib.oracle_tree.argtypes = [i64, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double, u32p, u32p, i64p]
    lib.oracle_tree.restype = i64
    lib.oracle_direct.argtypes = [i64, dp, dp, dp, C.c_double, i64, i64p, dp, dp]
    lib.oracle_direct_split.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_double, C.c_double,
                                        C.c_double, i64, i64p, dp, dp]
    lib.oracle_p2m.argtypes = [i64, dp, dp, dp, C.c_double, C.c_double, C.c_int, dp]
    lib.oracle_me_eval.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp]
    lib.oracle_m2m.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp]
    lib.oracle_m2l.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp]
    lib.oracle_l2l.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp]
    lib.oracle_l2p.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp]
    lib.oracle_near_list.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p]
    lib.oracle_near_list.restype = C.c_int
    lib.oracle_interaction_list.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p]
    lib.oracle_interaction_list.restype = C.c_int
    lib.oracle_fmm.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_double, i64, i64p, dp, dp, dp, dp]
    lib.oracle_fmm.restype = i64
    lib.oracle_advance_rk2.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double,
                                       C.c_int]
    lib.oracle_direct_at.argtypes = [i64, dp, dp, dp, C.c_double, i64, dp, dp, dp, dp]
    lib.oracle_direct_split_at.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_double, C.c_double,
                                           C.c_double, i64, dp, dp, dp, dp]
    lib.oracle_fmm_at.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_double, i64, dp, dp, dp, dp]
    lib.oracle_fmm_at.restype = i64
    lib.oracle_lj_forces.argtypes = [i64, dp, dp, C.c_double, C.c_double, C.c_double, i64, i64p, dp, dp]
    lib.oracle_lj_energy.argtypes = [i64, dp, dp, C.c_double, C.c_double, C.c_double]
    lib.oracle_lj_energy.restype = C.c_double
    lib.oracle_hermite.argtypes = [C.c_int, C.c_double, dp]
    lib.oracle_gauss_direct.argtypes = [i64, dp, dp, dp, C.c_double, i64, i64p, dp]
    lib.oracle_fgt.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_double, C.c_int, dp]
    lib.oracle_fgt.restype = i64
    lib.oracle_gauss_direct_at.argtypes = [i64, dp, dp, dp, C.c_double, i64, dp, dp, dp]
    lib.oracle_fgt_at.argtypes = [i64, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_int, i64, dp, dp, dp]
    lib.oracle_fgt_at.restype = i64
    lib.oracle3_deriv.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp]
    lib.oracle3_direct.argtypes = [i64, dp, dp, dp, dp, i64, i64p, dp, dp, dp, dp]
    lib.oracle3_p2m.argtypes = [i64, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int, dp]
    lib.oracle3_me_eval.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double]
    lib.oracle3_me_eval.restype = C.c_double
    for f in (lib.oracle3_m2m, lib.oracle3_m2l, lib.oracle3_l2l, lib.oracle3_l2p):
        f.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, dp]
    lib.oracle3_leaf_coords.argtypes = [i64, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                        C.c_double, i32p, i32p, i32p]
    lib.oracle3_leaf_coords.restype = i64
    lib.oracle3_morton.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
    lib.oracle3_morton.restype = C.c_uint32
    lib.oracle3_fmm.argtypes = [i64, dp, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                C.c_double, dp, dp, dp, dp]
    lib.oracle3_fmm.restype = i64
    lib.oracle_init()
    _lib = lib
    return lib


PMAX = 64


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _targets(tgt, n):
    if tgt is None:
        return None, n, None
    t = np.ascontiguousarray(tgt, dtype=np.int64)
    return t, int(t.shape[0]), t.ctypes.data_as(C.POINTER(C.c_int64))


def bounding_square(x, y):
    """(x0, y0, W): the square the auto-domain mode uses."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    dom = np.zeros(3)
    lib.oracle_bounding_square(x.shape[0], _d(x), _d(y), _d(dom))
    return float(dom[0]), float(dom[1]), float(dom[2])


def quantize(x, y, L, x0=0.0, y0=0.0, W=1.0):
    """Level-L box coordinates (ia, ib) of every particle and the out-of-domain count."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    ia = np.zeros(n, np.int32)
    ib = np.zeros(n, np.int32)
    nbad = lib.oracle_quantize(n, _d(x), _d(y), L, x0, y0, W,
                               ia.ctypes.data_as(C.POINTER(C.c_int32)),
                               ib.ctypes.data_as(C.POINTER(C.c_int32)))
    return ia, ib, int(nbad)


def morton(a, b):
    return int(_load().oracle_morton(int(a), int(b)))


def tree(x, y, L, x0=0.0, y0=0.0, W=1.0):
    """(key[n] u32, perm[n] u32, leaf_start[4^L+1] i64, n_out_of_domain)."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    key = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    ls = np.zeros((1 << (2 * L)) + 1, np.int64)
    nbad = lib.oracle_tree(n, _d(x), _d(y), L, x0, y0, W,
                           key.ctypes.data_as(C.POINTER(C.c_uint32)),
                           perm.ctypes.data_as(C.POINTER(C.c_uint32)),
                           ls.ctypes.data_as(C.POINTER(C.c_int64)))
    return key, perm, ls, int(nbad)


def direct(x, y, g, sigma, targets=None):
    """Regularised direct sum (eq. 9) at all particles or at ``targets``."""
    lib = _load()
    x, y, g = _f64(x), _f64(y), _f64(g)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    u = np.zeros(nt)
    v = np.zeros(nt)
    lib.oracle_direct(n, _d(x), _d(y), _d(g), sigma, nt, tp, _d(u), _d(v))
    return u, v


def direct_split(x, y, g, sigma, L, x0=0.0, y0=0.0, W=1.0, targets=None):
    """Split-kernel direct sum: Gaussian kernel for touching-leaf pairs, singular otherwise."""
    lib = _load()
    x, y, g = _f64(x), _f64(y), _f64(g)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    u = np.zeros(nt)
    v = np.zeros(nt)
    lib.oracle_direct_split(n, _d(x), _d(y), _d(g), sigma, L, x0, y0, W, nt, tp, _d(u), _d(v))
    return u, v


def fmm(x, y, g, sigma, p, L, x0=0.0, y0=0.0, W=1.0, targets=None, dump=False):
    """One FP64 FMM evaluation.  Returns (u, v) or (u, v, me, le, nbad) with dump=True.

    me / le are complex arrays [Lambda, p] in the oracle's own layout: level l
    starts at (4^l - 1)/3 and box (a, b) sits at row-major index b * 2^l + a.
    """
    lib = _load()
    if not (1 <= p <= PMAX):
        raise ValueError("p out of range")
    x, y, g = _f64(x), _f64(y), _f64(g)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    u = np.zeros(nt)
    v = np.zeros(nt)
    nbox = ((1 << (2 * (L + 1))) - 1) // 3
    me = le = None
    mep = lep = None
    if dump:
        me = np.zeros(nbox * p, np.complex128)
        le = np.zeros(nbox * p, np.complex128)
        mep = me.ctypes.data_as(C.POINTER(C.c_double))
        lep = le.ctypes.data_as(C.POINTER(C.c_double))
    nbad = lib.oracle_fmm(n, _d(x), _d(y), _d(g), sigma, p, L, x0, y0, W, nt, tp,
                          _d(u), _d(v), mep, lep)
    if dump:
        return u, v, me.reshape(nbox, p), le.reshape(nbox, p), int(nbad)
    return u, v


# ---- single operators (used by the operator-identity pins) -------------------

def p2m(x, y, g, cx, cy, p):
    lib = _load()
    x, y, g = _f64(x), _f64(y), _f64(g)
    a = np.zeros(p, np.complex128)
    lib.oracle_p2m(x.shape[0], _d(x), _d(y), _d(g), cx, cy, p, a.ctypes.data_as(C.POINTER(C.c_double)))
    return a


def me_eval(a, cx, cy, zx, zy):
    lib = _load()
    a = np.ascontiguousarray(a, np.complex128)
    out = np.zeros(2)
    lib.oracle_me_eval(a.shape[0], a.ctypes.data_as(C.POINTER(C.c_double)), cx, cy, zx, zy, _d(out))
    return complex(out[0], out[1])


def _op(fn, coeffs, dx, dy):
    c = np.ascontiguousarray(coeffs, np.complex128)
    out = np.zeros_like(c)
    fn(c.shape[0], c.ctypes.data_as(C.POINTER(C.c_double)), dx, dy, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def m2m(a_child, dx, dy):
    """Shift a child ME by d = c_child - c_parent."""
    return _op(_load().oracle_m2m, a_child, dx, dy)


def m2l(a_src, tx, ty):
    """ME about the source centre -> LE about the target centre, tau = c_s - c_t."""
    return _op(_load().oracle_m2l, a_src, tx, ty)


def l2l(b_parent, dx, dy):
    """Re-centre an LE by d = c_child - c_parent."""
    return _op(_load().oracle_l2l, b_parent, dx, dy)


def l2p(b, cx, cy, zx, zy):
    lib = _load()
    b = np.ascontiguousarray(b, np.complex128)
    out = np.zeros(2)
    lib.oracle_l2p(b.shape[0], b.ctypes.data_as(C.POINTER(C.c_double)), cx, cy, zx, zy, _d(out))
    return complex(out[0], out[1])


def near_list(L, a, b):
    lib = _load()
    sa = np.zeros(9, np.int32)
    sb = np.zeros(9, np.int32)
    k = lib.oracle_near_list(L, a, b, sa.ctypes.data_as(C.POINTER(C.c_int32)),
                             sb.ctypes.data_as(C.POINTER(C.c_int32)))
    return list(zip(sa[:k].tolist(), sb[:k].tolist()))


def interaction_list(l, a, b):
    lib = _load()
    sa = np.zeros(27, np.int32)
    sb = np.zeros(27, np.int32)
    k = lib.oracle_interaction_list(l, a, b, sa.ctypes.data_as(C.POINTER(C.c_int32)),
                                    sb.ctypes.data_as(C.POINTER(C.c_int32)))
    return list(zip(sa[:k].tolist(), sb[:k].tolist()))


def rel_l2(u, v, uref, vref):
    """sqrt(sum |w - w_ref|^2) / sqrt(sum |w_ref|^2) over 2-vectors w = (u, v)."""
    num = np.sum((np.asarray(u) - uref) ** 2 + (np.asarray(v) - vref) ** 2)
    den = np.sum(np.asarray(uref) ** 2 + np.asarray(vref) ** 2)
    return float(np.sqrt(num / den))


def advance_rk2(x, y, g, sigma, dt, steps, p=12, L=4, velocity="fmm"):
    """Explicit midpoint-rule time stepping of the particles (Section 3, eq. 6).

    velocity="fmm": the oracle FMM on the particles' bounding square at every
    stage; velocity="direct": the regularised direct sum.  Returns new (x, y).
    """
    lib = _load()
    x, y, g = _f64(x).copy(), _f64(y).copy(), _f64(g)
    if velocity not in ("fmm", "direct"):
        raise ValueError(velocity)
    lib.oracle_advance_rk2(x.shape[0], _d(x), _d(y), _d(g), float(sigma), int(p), int(L),
                           1 if velocity == "fmm" else 0, float(dt), int(steps))
    return x, y


def direct_at(x, y, g, sigma, tx, ty):
    """Regularised sum of eq. 1 at target points distinct from the sources."""
    lib = _load()
    x, y, g, tx, ty = _f64(x), _f64(y), _f64(g), _f64(tx), _f64(ty)
    m = tx.shape[0]
    u, v = np.zeros(m), np.zeros(m)
    lib.oracle_direct_at(x.shape[0], _d(x), _d(y), _d(g), sigma, m, _d(tx), _d(ty), _d(u), _d(v))
    return u, v


def direct_split_at(x, y, g, sigma, L, tx, ty, x0=0.0, y0=0.0, W=1.0):
    """Split-kernel sum at target points: Gaussian kernel for sources in touching leaves."""
    lib = _load()
    x, y, g, tx, ty = _f64(x), _f64(y), _f64(g), _f64(tx), _f64(ty)
    m = tx.shape[0]
    u, v = np.zeros(m), np.zeros(m)
    lib.oracle_direct_split_at(x.shape[0], _d(x), _d(y), _d(g), sigma, L, x0, y0, W, m, _d(tx), _d(ty),
                               _d(u), _d(v))
    return u, v


def fmm_at(x, y, g, sigma, p, L, tx, ty, x0=0.0, y0=0.0, W=1.0):
    """FP64 FMM of the particles evaluated at target points; returns (u, v, nbad)."""
    lib = _load()
    x, y, g, tx, ty = _f64(x), _f64(y), _f64(g), _f64(tx), _f64(ty)
    m = tx.shape[0]
    u, v = np.zeros(m), np.zeros(m)
    nbad = lib.oracle_fmm_at(x.shape[0], _d(x), _d(y), _d(g), sigma, p, L, x0, y0, W, m, _d(tx), _d(ty),
                             _d(u), _d(v))
    return u, v, int(nbad)


def lj_forces(x, y, eps, sig, rc, targets=None):
    """Lennard-Jones forces (truncated at rc) on all particles or on ``targets``."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    fx, fy = np.zeros(nt), np.zeros(nt)
    lib.oracle_lj_forces(n, _d(x), _d(y), eps, sig, rc, nt, tp, _d(fx), _d(fy))
    return fx, fy


def lj_energy(x, y, eps, sig, rc):
    """Total Lennard-Jones energy (truncated at rc), each pair once."""
    x, y = _f64(x), _f64(y)
    return float(_load().oracle_lj_energy(x.shape[0], _d(x), _d(y), eps, sig, rc))


def hermite(m, t):
    """Hermite functions h_0 .. h_{m-1} at t (h_n = (-1)^n d^n/dt^n exp(-t^2))."""
    h = np.zeros(max(m, 1))
    _load().oracle_hermite(int(m), float(t), _d(h))
    return h[:m]


def gauss_direct(x, y, q, sigma, targets=None):
    """Plain Gauss transform sum_j q_j exp(-|x_i - x_j|^2 / (2 sigma^2)) at the particles."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    G = np.zeros(nt)
    lib.oracle_gauss_direct(n, _d(x), _d(y), _d(q), sigma, nt, tp, _d(G))
    return G


def fgt(x, y, q, sigma, p, L, nc, x0=0.0, y0=0.0, W=1.0):
    """Fast Gauss transform (Hermite / Taylor on the leaf boxes); returns (G, nbad)."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    G = np.zeros(x.shape[0])
    nbad = lib.oracle_fgt(x.shape[0], _d(x), _d(y), _d(q), sigma, int(p), int(L), x0, y0, W, int(nc), _d(G))
    return G, int(nbad)


def gauss_direct_at(x, y, q, sigma, tx, ty):
    """Plain Gauss transform at points apart from the particles."""
    lib = _load()
    x, y, q, tx, ty = _f64(x), _f64(y), _f64(q), _f64(tx), _f64(ty)
    G = np.zeros(tx.shape[0])
    lib.oracle_gauss_direct_at(x.shape[0], _d(x), _d(y), _d(q), sigma, tx.shape[0], _d(tx), _d(ty), _d(G))
    return G


def fgt_at(x, y, q, sigma, p, L, nc, tx, ty, x0=0.0, y0=0.0, W=1.0):
    """Fast Gauss transform at points apart from the particles; returns (G, nbad)."""
    lib = _load()
    x, y, q, tx, ty = _f64(x), _f64(y), _f64(q), _f64(tx), _f64(ty)
    G = np.zeros(tx.shape[0])
    nbad = lib.oracle_fgt_at(x.shape[0], _d(x), _d(y), _d(q), sigma, int(p), int(L), x0, y0, W, int(nc),
                             tx.shape[0], _d(tx), _d(ty), _d(G))
    return G, int(nbad)



# ---------------------------------------------------------------------------
# 3D form: Laplace kernel 1/r, Cartesian Taylor expansions (fmm3d_oracle.c)
# ---------------------------------------------------------------------------

P3MAX = 12


def _cube(p):
    return np.zeros((p + 1) ** 3)


def deriv3(q, r):
    """D[a, b, c] = d^(a,b,c) (1/|R|) at R = r for a + b + c <= q (else 0)."""
    D = _cube(q)
    _load().oracle3_deriv(q, float(r[0]), float(r[1]), float(r[2]), _d(D))
    return D.reshape(q + 1, q + 1, q + 1)


def direct3(x, y, z, q, targets=None):
    """Potential and its gradient from the plain sum over all other particles."""
    lib = _load()
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = x.shape[0]
    t, nt, tp = _targets(targets, n)
    out = [np.zeros(nt) for _ in range(4)]
    lib.oracle3_direct(n, _d(x), _d(y), _d(z), _d(q), nt, tp, *(_d(a) for a in out))
    return tuple(out)


def p2m3(x, y, z, q, c, p):
    M = _cube(p)
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    _load().oracle3_p2m(x.shape[0], _d(x), _d(y), _d(z), _d(q), float(c[0]), float(c[1]), float(c[2]), p, _d(M))
    return M


def me_eval3(M, p, r):
    M = _f64(M)
    return float(_load().oracle3_me_eval(p, _d(M), float(r[0]), float(r[1]), float(r[2])))


def _op3(fn, p, A, d, n_out=None):
    A = _f64(A)
    out = np.zeros(n_out if n_out else (p + 1) ** 3)
    fn(p, _d(A), float(d[0]), float(d[1]), float(d[2]), _d(out))
    return out


def m2m3(M, p, d):
    """Moments about c' = c + d from moments about c."""
    return _op3(_load().oracle3_m2m, p, M, d)


def m2l3(M, p, r):
    """Local coefficients about t from moments about s, r = t - s."""
    return _op3(_load().oracle3_m2l, p, M, r)


def l2l3(Lc, p, d):
    """Local coefficients about t' = t + d from those about t."""
    return _op3(_load().oracle3_l2l, p, Lc, d)


def l2p3(Lc, p, e):
    """(phi, dphi/dx, dphi/dy, dphi/dz) at t + e."""
    return _op3(_load().oracle3_l2p, p, Lc, e, 4)


def morton3(a, b, c):
    return int(_load().oracle3_morton(a, b, c))


def leaf_keys3(x, y, z, L, origin=(0.0, 0.0, 0.0), W=1.0):
    """Morton leaf key per particle (2^(3L) for one outside the cube) and the
    stable key order: what the GPU tree must reproduce bit for bit."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    ia, ib, ic = (np.zeros(n, np.int32) for _ in range(3))
    ip = C.POINTER(C.c_int32)
    lib.oracle3_leaf_coords(n, _d(x), _d(y), _d(z), L, float(origin[0]), float(origin[1]), float(origin[2]),
                            float(W), ia.ctypes.data_as(ip), ib.ctypes.data_as(ip), ic.ctypes.data_as(ip))
    keys = np.array([morton3(int(a), int(b), int(c)) if a >= 0 else 1 << (3 * L)
                     for a, b, c in zip(ia, ib, ic)], dtype=np.uint32)
    return keys, np.argsort(keys, kind="stable").astype(np.uint32)


def fmm3(x, y, z, q, p, L, origin=(0.0, 0.0, 0.0), W=1.0):
    """One FP64 FMM evaluation of the 3D form: (phi, gx, gy, gz, nbad)."""
    lib = _load()
    if not (0 <= p <= P3MAX) or not (0 <= L <= 7):
        raise ValueError("p or L out of range")
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = x.shape[0]
    out = [np.zeros(n) for _ in range(4)]
    nbad = lib.oracle3_fmm(n, _d(x), _d(y), _d(z), _d(q), p, L, float(origin[0]), float(origin[1]),
                           float(origin[2]), float(W), *(_d(a) for a in out))
    return (*out, int(nbad))
