"""ctypes binding of libnbody_hip.so (C ABI in include/nbody.h).

Argument marshalling only: every function checks torch tensors (float64,
contiguous, on the current HIP device, component-major ``(3, n)`` vectors
and ``(n,)`` masses), allocates the workspace the library asks for from
torch's caching allocator, and passes raw device pointers plus the current
torch stream.  All arithmetic happens in the library's gfx950 kernels.  The
names mirror the C entry points.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libnbody_hip.so")

NBODY_FP64 = 0
NBODY_MIXED = 1
NBODY_MIXED_D64 = 2
NBODY_MIXED_NF = 3
NBODY_MIXED_NF64 = 4
NBODY_MIXED_DS = 5
PRECISIONS = {"fp64": NBODY_FP64, "mixed": NBODY_MIXED,
              "mixed_d64": NBODY_MIXED_D64, "mixed_nf": NBODY_MIXED_NF,
              "mixed_nf64": NBODY_MIXED_NF64, "mixed_ds": NBODY_MIXED_DS}

NBODY_OK = 0
NBODY_ACC_VALID = 1
NBODY_HALF_KICK_DRIFT = 2
INTEGRATORS = {"kdk": 0, "half_kick_drift": NBODY_HALF_KICK_DRIFT}
NBODY_OP_ACCEL, NBODY_OP_STEP, NBODY_OP_VJP, NBODY_OP_STEP_ADJOINT = 0, 1, 2, 3
NBODY_OP_DIAGNOSTICS = 4
NBODY_OP_MORTON_SORT = 5
NBODY_MAX_N = 1 << 28
NBODY_NOALLOC_SCRATCH_BYTES = 64 << 20
# smallest eps of the FP32-pair precisions: every call / the VJP calls
NBODY_MIN_EPS_FP32 = 2.0 ** -42
NBODY_MIN_EPS_FP32_VJP = 2.0 ** -32

SYMBOLS = ("nbody_workspace_bytes", "nbody_checkpoint_bytes", "nbody_accel",
           "nbody_step", "nbody_accel_vjp", "nbody_step_adjoint",
           "nbody_diagnostics", "nbody_rows_workspace_bytes",
           "nbody_accel_rows", "nbody_accel_vjp_rows", "nbody_morton_sort",
           "nbody_f32_workspace_bytes", "nbody_accel_f32", "nbody_step_f32",
           "nbody_accel_noalloc", "nbody_error_string", "nbody_last_error")

_INVALID = ctypes.c_size_t(-1).value


class NBodyError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("nbody error %d: %s" % (code, message))
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("eps", ctypes.c_double),
                ("dt", ctypes.c_double)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            "libnbody_hip.so is not built (%s); run "
            "`python -m paper_2203_08263_amd.build` -- there is no CPU "
            "fallback" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, sz, vp, ci = ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
    pp = ctypes.POINTER(_Params)
    lib.nbody_workspace_bytes.argtypes = [ci, i64, i64, i64, ci]
    lib.nbody_workspace_bytes.restype = sz
    lib.nbody_checkpoint_bytes.argtypes = [i64, i64, i64]
    lib.nbody_checkpoint_bytes.restype = sz
    lib.nbody_accel.argtypes = [i64, vp, vp, vp, pp, ci, vp, sz, vp]
    lib.nbody_accel_noalloc.argtypes = [i64, vp, vp, vp, pp, ci, vp]
    lib.nbody_step.argtypes = [i64, i64, vp, vp, vp, vp, pp, ci, ctypes.c_uint,
                               vp, i64, vp, sz, vp]
    lib.nbody_accel_vjp.argtypes = [i64, vp, vp, vp, vp, vp, pp, ci, vp, sz, vp]
    lib.nbody_step_adjoint.argtypes = [i64, i64, i64, vp, vp, pp, ci,
                                       ctypes.c_uint, vp, vp, vp, vp, vp, sz, vp]
    lib.nbody_diagnostics.argtypes = [i64, vp, vp, vp, pp, ci, vp, vp, sz, vp]
    lib.nbody_rows_workspace_bytes.argtypes = [ci, i64, i64, ci]
    lib.nbody_rows_workspace_bytes.restype = sz
    lib.nbody_accel_rows.argtypes = [i64, i64, i64, vp, vp, vp, pp, ci, vp, sz, vp]
    lib.nbody_accel_vjp_rows.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, pp, ci,
                                         vp, sz, vp]
    lib.nbody_morton_sort.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.nbody_f32_workspace_bytes.argtypes = [ci, i64]
    lib.nbody_f32_workspace_bytes.restype = sz
    lib.nbody_accel_f32.argtypes = [i64, vp, vp, vp, pp, vp, sz, vp]
    lib.nbody_step_f32.argtypes = [i64, i64, vp, vp, vp, vp, pp, ctypes.c_uint, vp,
                                   sz, vp]
    for f in ("nbody_accel", "nbody_accel_noalloc", "nbody_step", "nbody_accel_vjp",
              "nbody_step_adjoint", "nbody_diagnostics", "nbody_accel_rows",
              "nbody_accel_vjp_rows", "nbody_morton_sort", "nbody_accel_f32",
              "nbody_step_f32"):
        getattr(lib, f).restype = ci
    lib.nbody_error_string.argtypes = [ci]
    lib.nbody_error_string.restype = ctypes.c_char_p
    lib.nbody_last_error.argtypes = []
    lib.nbody_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != NBODY_OK:
        lib = load_library()
        raise NBodyError(rc, lib.nbody_last_error().decode() or
                         lib.nbody_error_string(rc).decode())


def _run(dev, fn, *args):
    """Call a library entry point with the tensors' device current (the
    library launches on the current HIP device) and check its status."""
    with torch.cuda.device(dev):
        _check(fn(*args))


def _precision(p) -> int:
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError("unknown precision %r" % p)
        return PRECISIONS[p]
    return int(p)


def _vec(t, n, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64 or t.shape != (3, n) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 (3, %d) tensor, got "
                         "%s %s" % (name, n, t.dtype, tuple(t.shape)))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError("%s must be on the GPU device %s" % (name, device))
    return t


def _f32(t, shape, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float32 or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 %s tensor, got %s %s"
                         % (name, shape, t.dtype, tuple(t.shape)))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError("%s must be on the GPU device %s" % (name, device))
    return t


def _scal(t, n, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64 or t.shape != (n,) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 (%d,) tensor" % (name, n))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError("%s must be on the GPU device %s" % (name, device))
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes, device, workspace=None):
    if nbytes == _INVALID:
        raise NBodyError(1, "invalid arguments for the workspace size")
    if nbytes == 0:
        return None, 0
    if workspace is not None:
        if workspace.device != device or not workspace.is_contiguous():
            raise ValueError("workspace must be contiguous on %s" % device)
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace smaller than the %d bytes needed" % nbytes)
        return workspace, workspace.numel() * workspace.element_size()
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return ws, nbytes


def nbody_workspace_bytes(op: int, n: int, steps: int = 0, ckpt_every: int = 1,
                          precision=NBODY_FP64) -> int:
    return int(load_library().nbody_workspace_bytes(op, n, steps, ckpt_every,
                                                    _precision(precision)))


def nbody_rows_workspace_bytes(op: int, n: int, row_count: int,
                               precision=NBODY_FP64) -> int:
    return int(load_library().nbody_rows_workspace_bytes(op, n, row_count,
                                                         _precision(precision)))


def nbody_checkpoint_bytes(n: int, steps: int, ckpt_every: int) -> int:
    return int(load_library().nbody_checkpoint_bytes(n, steps, ckpt_every))


def nbody_accel(pos, mass, G=1.0, eps=1e-3, precision=NBODY_FP64, out=None,
                workspace=None):
    """Accelerations (3, n) of all bodies (all-pairs, softened)."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    prec = _precision(precision)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev) if out is None \
        else _vec(out, n, "out", dev)
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_ACCEL, n, 0, 1, prec),
                         dev, workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel, n, _ptr(pos), _ptr(mass), _ptr(acc), ctypes.byref(prm),
         prec, _ptr(ws), wsb, _stream(dev))
    return acc


def nbody_accel_noalloc(pos, mass, G=1.0, eps=1e-3, precision=NBODY_FP64, out=None):
    """nbody_accel without a workspace: the library's static device scratch
    holds the partial sums (the call allocates nothing; `out` must be given
    by callers that cannot allocate)."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    prec = _precision(precision)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev) if out is None \
        else _vec(out, n, "out", dev)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel_noalloc, n, _ptr(pos), _ptr(mass), _ptr(acc),
         ctypes.byref(prm), prec, _stream(dev))
    return acc


def _integrator(name) -> int:
    if name not in INTEGRATORS:
        raise ValueError("unknown integrator %r (kdk or half_kick_drift)" % (name,))
    return INTEGRATORS[name]


def nbody_step(pos, vel, acc, mass, G=1.0, eps=1e-3, dt=1e-3, steps=1,
               precision=NBODY_FP64, acc_valid=False, ckpt=None, ckpt_every=0,
               workspace=None, integrator="kdk"):
    """`steps` time steps in place on pos, vel, acc.  integrator "kdk"
    (kick-drift-kick leapfrog) or "half_kick_drift" (the paper's listings)."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    _vec(vel, n, "vel", dev)
    _vec(acc, n, "acc", dev)
    prec = _precision(precision)
    if ckpt is not None:
        need = lib.nbody_checkpoint_bytes(n, steps, ckpt_every)
        if need == _INVALID:
            raise NBodyError(1, "invalid checkpoint arguments")
        if (ckpt.dtype != torch.float64 or not ckpt.is_contiguous()
                or ckpt.device != dev or ckpt.numel() * 8 < need):
            raise ValueError("ckpt must be contiguous float64 on %s with at "
                             "least %d bytes" % (dev, need))
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_STEP, n, steps, 1, prec),
                         dev, workspace)
    prm = _Params(G, eps, dt)
    flags = (NBODY_ACC_VALID if acc_valid else 0) | _integrator(integrator)
    _run(dev, lib.nbody_step, n, int(steps), _ptr(pos), _ptr(vel), _ptr(acc),
         _ptr(mass), ctypes.byref(prm), prec, flags, _ptr(ckpt),
         int(ckpt_every), _ptr(ws), wsb, _stream(dev))
    return pos, vel, acc


def nbody_accel_vjp(pos, mass, gacc, G=1.0, eps=1e-3, precision=NBODY_FP64,
                    gpos=None, gmass=None, workspace=None):
    """(dL/dx (3, n), dL/dm (n,)) for upstream gacc = dL/da."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    _vec(gacc, n, "gacc", dev)
    prec = _precision(precision)
    gpos = torch.empty((3, n), dtype=torch.float64, device=dev) if gpos is None \
        else _vec(gpos, n, "gpos", dev)
    gmass = torch.empty(n, dtype=torch.float64, device=dev) if gmass is None \
        else _scal(gmass, n, "gmass", dev)
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_VJP, n, 0, 1, prec),
                         dev, workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel_vjp, n, _ptr(pos), _ptr(mass), _ptr(gacc), _ptr(gpos),
         _ptr(gmass), ctypes.byref(prm), prec, _ptr(ws),
         wsb, _stream(dev))
    return gpos, gmass


def nbody_step_adjoint(ckpt, mass, gpos, gvel, G=1.0, eps=1e-3, dt=1e-3,
                       steps=1, ckpt_every=1, precision=NBODY_FP64,
                       gacc_T=None, gmass=None, workspace=None, integrator="kdk"):
    """Reverse sweep: gpos/gvel (in: dL/dx_S, dL/dv_S) become dL/dx_0, dL/dv_0
    in place; returns (gpos, gvel, gmass)."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(gpos, n, "gpos", dev)
    _vec(gvel, n, "gvel", dev)
    if gacc_T is not None:
        _vec(gacc_T, n, "gacc_T", dev)
    prec = _precision(precision)
    need = lib.nbody_checkpoint_bytes(n, steps, ckpt_every)
    if need == _INVALID:
        raise NBodyError(1, "invalid checkpoint arguments")
    if (ckpt.dtype != torch.float64 or not ckpt.is_contiguous()
            or ckpt.device != dev or ckpt.numel() * 8 < need):
        raise ValueError("ckpt must be contiguous float64 on %s with at least "
                         "%d bytes" % (dev, need))
    gmass = torch.empty(n, dtype=torch.float64, device=dev) if gmass is None \
        else _scal(gmass, n, "gmass", dev)
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_STEP_ADJOINT, n, steps,
                                                   ckpt_every, prec), dev, workspace)
    prm = _Params(G, eps, dt)
    _run(dev, lib.nbody_step_adjoint, n, int(steps), int(ckpt_every), _ptr(ckpt),
         _ptr(mass), ctypes.byref(prm), prec,
         _integrator(integrator), _ptr(gpos),
         _ptr(gvel), _ptr(gacc_T), _ptr(gmass), _ptr(ws),
         wsb, _stream(dev))
    return gpos, gvel, gmass


def nbody_diagnostics(pos, vel, mass, G=1.0, eps=1e-3, precision=NBODY_FP64,
                      out=None, workspace=None):
    """Device tensor (9,): kinetic energy, softened potential energy,
    momentum (3), mass-weighted position sum (3), total mass."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    _vec(vel, n, "vel", dev)
    prec = _precision(precision)
    if out is None:
        out = torch.empty(9, dtype=torch.float64, device=dev)
    elif out.dtype != torch.float64 or out.numel() < 9 or not out.is_contiguous() \
            or out.device != dev:
        raise ValueError("out must be a contiguous float64 tensor of >= 9 on %s" % dev)
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_DIAGNOSTICS, n, 0, 1, prec),
                         dev, workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_diagnostics, n, _ptr(pos), _ptr(vel), _ptr(mass), ctypes.byref(prm),
         prec, _ptr(out), _ptr(ws), wsb, _stream(dev))
    return out


def _rows_out(t, rows, shape, name, dev):
    if t is None:
        return torch.empty(shape, dtype=torch.float64, device=dev)
    return _vec(t, rows, name, dev) if len(shape) == 2 else _scal(t, rows, name, dev)


def nbody_accel_rows(pos, mass, row_begin, row_count, G=1.0, eps=1e-3,
                     precision=NBODY_FP64, out=None, workspace=None):
    """Accelerations (3, row_count) of bodies row_begin .. row_begin +
    row_count - 1 against all n sources."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    prec = _precision(precision)
    rows = int(row_count)
    acc = _rows_out(out, rows, (3, rows), "out", dev)
    ws, wsb = _workspace(lib.nbody_rows_workspace_bytes(NBODY_OP_ACCEL, n, rows,
                                                        prec), dev, workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel_rows, n, int(row_begin), rows, _ptr(pos), _ptr(mass),
         _ptr(acc), ctypes.byref(prm), prec, _ptr(ws), wsb,
         _stream(dev))
    return acc


def nbody_accel_vjp_rows(pos, mass, gacc, row_begin, row_count, G=1.0, eps=1e-3,
                         precision=NBODY_FP64, gpos=None, gmass=None,
                         workspace=None):
    """(dL/dx (3, row_count), dL/dm (row_count,)) of bodies row_begin ..
    row_begin + row_count - 1, for upstream gacc = dL/da of all n bodies."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    _vec(gacc, n, "gacc", dev)
    prec = _precision(precision)
    rows = int(row_count)
    gpos = _rows_out(gpos, rows, (3, rows), "gpos", dev)
    gmass = _rows_out(gmass, rows, (rows,), "gmass", dev)
    ws, wsb = _workspace(lib.nbody_rows_workspace_bytes(NBODY_OP_VJP, n, rows,
                                                        prec), dev, workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel_vjp_rows, n, int(row_begin), rows, _ptr(pos), _ptr(mass),
         _ptr(gacc), _ptr(gpos), _ptr(gmass),
         ctypes.byref(prm), prec, _ptr(ws), wsb,
         _stream(dev))
    return gpos, gmass


def nbody_morton_sort(pos, mass, vel=None, workspace=None, perm=None,
                      pos_out=None, vel_out=None, mass_out=None):
    """Bodies in Morton (Z) order of their positions: returns (perm, pos_out,
    vel_out or None, mass_out) with pos_out[:, r] = pos[:, perm[r]].  `vel`
    may be any (3, n) per-body vector carried along with the bodies (e.g.
    dL/da).  Outputs are allocated unless given."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _scal(mass, n, "mass")
    _vec(pos, n, "pos", dev)
    if vel is not None:
        _vec(vel, n, "vel", dev)
    if perm is None:
        perm = torch.empty(n, dtype=torch.int64, device=dev)
    elif (perm.dtype != torch.int64 or tuple(perm.shape) != (n,)
          or not perm.is_contiguous() or perm.device != dev):
        raise ValueError("perm must be a contiguous int64 (%d,) tensor on %s" % (n, dev))
    pos_out = torch.empty((3, n), dtype=torch.float64, device=dev) if pos_out is None \
        else _vec(pos_out, n, "pos_out", dev)
    if vel is None:
        if vel_out is not None:
            raise ValueError("vel_out given without vel")
    else:
        vel_out = torch.empty((3, n), dtype=torch.float64, device=dev) \
            if vel_out is None else _vec(vel_out, n, "vel_out", dev)
    mass_out = torch.empty(n, dtype=torch.float64, device=dev) if mass_out is None \
        else _scal(mass_out, n, "mass_out", dev)
    ws, wsb = _workspace(lib.nbody_workspace_bytes(NBODY_OP_MORTON_SORT, n, 0, 1, 0),
                         dev, workspace)
    _run(dev, lib.nbody_morton_sort, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(perm),
         _ptr(pos_out), _ptr(vel_out), _ptr(mass_out),
         _ptr(ws), wsb, _stream(dev))
    return perm, pos_out, vel_out, mass_out


def nbody_f32_workspace_bytes(op: int, n: int) -> int:
    return int(load_library().nbody_f32_workspace_bytes(op, n))


def nbody_accel_f32(pos, mass, G=1.0, eps=1e-3, out=None, workspace=None):
    """Accelerations (3, n) float32 of float32 state, all arithmetic FP32."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _f32(mass, (n,), "mass")
    _f32(pos, (3, n), "pos", dev)
    acc = torch.empty((3, n), dtype=torch.float32, device=dev) if out is None \
        else _f32(out, (3, n), "out", dev)
    ws, wsb = _workspace(lib.nbody_f32_workspace_bytes(NBODY_OP_ACCEL, n), dev,
                         workspace)
    prm = _Params(G, eps, 0.0)
    _run(dev, lib.nbody_accel_f32, n, _ptr(pos), _ptr(mass), _ptr(acc),
         ctypes.byref(prm), _ptr(ws), wsb, _stream(dev))
    return acc


def nbody_step_f32(pos, vel, acc, mass, G=1.0, eps=1e-3, dt=1e-3, steps=1,
                   acc_valid=False, workspace=None, integrator="kdk"):
    """`steps` FP32 time steps in place on float32 pos, vel, acc."""
    lib = load_library()
    n = mass.shape[0]
    dev = mass.device
    _f32(mass, (n,), "mass")
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
        _f32(t, (3, n), name, dev)
    ws, wsb = _workspace(lib.nbody_f32_workspace_bytes(NBODY_OP_STEP, n), dev,
                         workspace)
    prm = _Params(G, eps, dt)
    flags = (NBODY_ACC_VALID if acc_valid else 0) | _integrator(integrator)
    _run(dev, lib.nbody_step_f32, n, int(steps), _ptr(pos), _ptr(vel), _ptr(acc),
         _ptr(mass), ctypes.byref(prm), flags, _ptr(ws), wsb,
         _stream(dev))
    return pos, vel, acc
