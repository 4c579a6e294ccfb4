"""FP64 CPU oracle for the all-pairs N-body hot path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports
this package and shares no code with it.

The arithmetic lives in ``nbody_oracle.c`` (plain C, IEEE double, no FMA
contraction, OpenMP over target rows only); this module compiles it with gcc
and wraps it with ctypes over NumPy arrays.  All arrays are float64,
component-major ``(3, n)`` for vectors and ``(n,)`` for masses.

Paper references (arxiv 2203.08263): the problem statement and pseudo-code of
section 2.3, the force loop of the section 3.1-3.3 listings, and the
20-flop-per-interaction convention of section 4.1.  Every function here is
pinned by ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_nbody.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-std=c99"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle_nbody.so``."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, dbl, ptr = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_accel.argtypes = [i64, ptr, ptr, dbl, dbl, ptr]
    lib.oracle_accel_rows.argtypes = [i64, ptr, ptr, dbl, dbl, i64, ptr, ptr]
    lib.oracle_step.argtypes = [i64, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl,
                                ctypes.c_int, ctypes.c_int]
    lib.oracle_energy.argtypes = [i64, ptr, ptr, ptr, dbl, dbl, ptr]
    lib.oracle_momentum.argtypes = [i64, ptr, ptr, ptr]
    lib.oracle_accel_vjp.argtypes = [i64, ptr, ptr, ptr, dbl, dbl, ptr, ptr]
    lib.oracle_accel_vjp_rows.argtypes = [i64, ptr, ptr, ptr, dbl, dbl, i64,
                                          ptr, ptr, ptr]
    lib.oracle_step_adjoint.argtypes = [i64, i64, ptr, ptr, ptr, dbl, dbl, dbl,
                                        ctypes.c_int, ptr, ptr, ptr, ptr]
    lib.oracle_step_adjoint.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _vec(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (3, n):
        raise ValueError("expected shape (3, %d), got %r" % (n, a.shape))
    return a


def _scal(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError("expected shape (%d,), got %r" % (n, a.shape))
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def accel(pos, mass, G, eps):
    """a_i = G sum_j m_j (x_j - x_i) (|x_j - x_i|^2 + eps^2)^(-3/2), all i."""
    n = mass.shape[0]
    pos, mass = _vec(pos, n), _scal(mass, n)
    out = np.empty((3, n))
    _load().oracle_accel(n, _p(pos), _p(mass), G, eps, _p(out))
    return out


def accel_rows(pos, mass, G, eps, rows):
    """Accelerations of the selected target rows only, shape (3, len(rows))."""
    n = mass.shape[0]
    pos, mass = _vec(pos, n), _scal(mass, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    out = np.empty((3, rows.size))
    _load().oracle_accel_rows(n, _p(pos), _p(mass), G, eps, rows.size,
                              _p(rows), _p(out))
    return out


SCHEMES = {"kdk": 0, "half_kick_drift": 1}


def step(pos, vel, mass, G, eps, dt, steps, acc=None, scheme="kdk"):
    """Time integration; returns (pos, vel, acc) after `steps` steps (copies).

    scheme "kdk": kick-drift-kick leapfrog; "half_kick_drift": the update of
    the paper's listings (v += a dt/2; x += v dt per step)."""
    n = mass.shape[0]
    x = _vec(pos, n).copy()
    v = _vec(vel, n).copy()
    mass = _scal(mass, n)
    if acc is None:
        a, valid = np.empty((3, n)), 0
    else:
        a, valid = _vec(acc, n).copy(), 1
    _load().oracle_step(n, int(steps), _p(x), _p(v), _p(a), _p(mass), G, eps,
                        dt, valid, SCHEMES[scheme])
    return x, v, a


def energy(pos, vel, mass, G, eps):
    """(kinetic, potential) of the Plummer-softened system."""
    n = mass.shape[0]
    pos, vel, mass = _vec(pos, n), _vec(vel, n), _scal(mass, n)
    out = np.empty(2)
    _load().oracle_energy(n, _p(pos), _p(vel), _p(mass), G, eps, _p(out))
    return float(out[0]), float(out[1])


def momentum(vel, mass):
    n = mass.shape[0]
    vel, mass = _vec(vel, n), _scal(mass, n)
    out = np.empty(3)
    _load().oracle_momentum(n, _p(vel), _p(mass), _p(out))
    return out


def accel_vjp(pos, mass, gacc, G, eps):
    """(dL/dx (3,n), dL/dm (n,)) given dL/da."""
    n = mass.shape[0]
    pos, mass, gacc = _vec(pos, n), _scal(mass, n), _vec(gacc, n)
    gp, gm = np.empty((3, n)), np.empty(n)
    _load().oracle_accel_vjp(n, _p(pos), _p(mass), _p(gacc), G, eps, _p(gp),
                             _p(gm))
    return gp, gm


def accel_vjp_rows(pos, mass, gacc, G, eps, rows):
    n = mass.shape[0]
    pos, mass, gacc = _vec(pos, n), _scal(mass, n), _vec(gacc, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    gp, gm = np.empty((3, rows.size)), np.empty(rows.size)
    _load().oracle_accel_vjp_rows(n, _p(pos), _p(mass), _p(gacc), G, eps,
                                  rows.size, _p(rows), _p(gp), _p(gm))
    return gp, gm


MORTON_BITS = 10


def morton_order(pos):
    """Permutation that sorts bodies by their Morton (Z-order) code.

    Positions are quantised on a 1024^3 grid over the cube [lo, lo + ext]^3
    (lo the componentwise minimum, ext the largest extent of the bounding
    box): q = min(1023, floor((x - lo) * (1024 / ext))) per axis in FP64, 0
    when ext == 0; the code interleaves the bits of (q_x, q_y, q_z) from the
    most significant down, x first.  Equal codes keep their original order.
    Pure NumPy; the spatial ordering the near / far precision mode relies on
    for speed (the paper's data-locality concern, section 3.3)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    if pos.ndim != 2 or pos.shape[0] != 3:
        raise ValueError("expected shape (3, n)")
    lo = pos.min(axis=1)
    ext = float(np.max(pos.max(axis=1) - lo))
    sc = 1024.0 / ext if ext > 0.0 else 0.0
    q = np.floor((pos - lo[:, None]) * sc)
    q = np.where(q > 0.0, q, 0.0)
    q = np.minimum(q, 1023.0).astype(np.uint64)
    code = np.zeros(pos.shape[1], dtype=np.uint64)
    for b in range(MORTON_BITS):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            code |= ((q[axis] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + shift)
    return np.argsort(code, kind="stable")


def step_adjoint(pos0, vel0, mass, G, eps, dt, steps, gpos_T, gvel_T,
                 gacc_T=None, scheme="kdk"):
    """Exact reverse sweep of `step` from (pos0, vel0) (acc recomputed).

    Returns (dL/dx_0, dL/dv_0, dL/dm) for upstream (dL/dx_S, dL/dv_S[, dL/da_S]).
    """
    n = mass.shape[0]
    x0, v0, mass = _vec(pos0, n), _vec(vel0, n), _scal(mass, n)
    gx = _vec(gpos_T, n).copy()
    gv = _vec(gvel_T, n).copy()
    ga = None if gacc_T is None else _vec(gacc_T, n)
    gm = np.empty(n)
    rc = _load().oracle_step_adjoint(n, int(steps), _p(x0), _p(v0), _p(mass),
                                     G, eps, dt, SCHEMES[scheme], _p(gx), _p(gv),
                                     None if ga is None else _p(ga), _p(gm))
    if rc != 0:
        raise MemoryError("oracle_step_adjoint: allocation failed")
    return gx, gv, gm
