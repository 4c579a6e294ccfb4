"""Error and throughput figures used to state results (no method arithmetic).

Per-body relative acceleration error E_i = |a_i - a_i^ref| / |a_i^ref|
(Euclidean norms over the three components), summarised as

* ``E_max``  = max_i E_i (the "max relative acceleration error");
* ``E_norm`` = |a - a^ref|_F / |a^ref|_F;
* ``E_inf``  = max_i |a_i - a_i^ref| / max_i |a_i^ref|;
* ``E_med``  = median_i E_i.

Interaction counts follow the paper's convention (section 4.1): N^2 body
pairs per force evaluation, self pairs included, 20 flops per pair.
"""
from __future__ import annotations

import numpy as np

FLOPS_PER_INTERACTION = 20


def rel_errors(a, ref) -> dict:
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if a.shape != ref.shape:
        raise ValueError("shape mismatch %r vs %r" % (a.shape, ref.shape))
    d = np.sqrt(((a - ref) ** 2).sum(axis=0))
    r = np.sqrt((ref ** 2).sum(axis=0))
    with np.errstate(divide="ignore", invalid="ignore"):
        ei = np.where(r > 0, d / r, np.where(d > 0, np.inf, 0.0))
    return {
        "E_max": float(ei.max()) if ei.size else 0.0,
        "E_norm": float(np.sqrt((d ** 2).sum()) / max(np.sqrt((r ** 2).sum()), 1e-300)),
        "E_inf": float(d.max() / max(r.max(), 1e-300)) if d.size else 0.0,
        "E_med": float(np.median(ei)) if ei.size else 0.0,
    }


def normwise(a, ref) -> float:
    """|a - ref|_F / |ref|_F."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def interactions(n: int, evals: int) -> int:
    return int(n) * int(n) * int(evals)
