"""MI355X-native all-pairs gravitational N-body hot path (arxiv 2203.08263).

The compute path is the HIP library ``libnbody_hip.so`` built from ``csrc/``
for gfx950, reached through its C ABI (``include/nbody.h``).  This package is
the thin Python binding: argument marshalling over torch device tensors and
``torch.autograd.Function`` wrappers.  The library is loaded on first use and
a missing build raises immediately; there is no CPU fallback.

Submodules load lazily so that ``paper_2203_08263_amd.inputs`` (the seeded
input generators) can be imported without torch or the HIP library.
"""
import importlib

_BINDING = (
    "NBODY_FP64", "NBODY_MIXED", "NBODY_MIXED_D64", "NBODY_MIXED_NF",
    "NBODY_MIXED_NF64", "NBODY_MIXED_DS", "PRECISIONS",
    "NBodyError", "nbody_morton_sort", "nbody_accel_f32", "nbody_step_f32",
    "nbody_f32_workspace_bytes",
    "nbody_accel", "nbody_accel_noalloc", "nbody_accel_vjp", "nbody_step",
    "nbody_step_adjoint",
    "nbody_diagnostics", "nbody_accel_rows", "nbody_accel_vjp_rows",
    "nbody_workspace_bytes", "nbody_rows_workspace_bytes",
    "nbody_checkpoint_bytes", "library_path",
    "load_library",
)
_AUTOGRAD = ("NBodyAccel", "NBodyRollout", "accel", "rollout", "auto_ckpt_every")

__all__ = list(_BINDING + _AUTOGRAD)


def __getattr__(name):
    if name in _BINDING:
        return getattr(importlib.import_module(".binding", __name__), name)
    if name in _AUTOGRAD:
        return getattr(importlib.import_module(".autograd", __name__), name)
    raise AttributeError(name)
