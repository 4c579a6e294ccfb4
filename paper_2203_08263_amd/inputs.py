"""Seeded synthetic initial conditions and upstream gradients.

This module generates inputs only; it holds none of the force, integrator or
adjoint arithmetic.  Both the HIP path (tests, benchmark) and the FP64 oracle
take their inputs from here, so they see identical float64 arrays.

The paper (arxiv 2203.08263, section 4.1) benchmarks synthetic systems of N
bodies but states neither its initial conditions nor G, the softening or the
time step; the workloads below fix them:

* ``uniform_cube``: positions U(-1, 1)^3, velocities N(0, 0.1^2) per
  component, masses U(0.5, 1.0) / N, drawn in that order from one PCG64
  stream.
* ``plummer``: a Plummer sphere of scale radius ``a`` and total mass ``M``
  with equal masses, sampled by the method of Aarseth, Henon & Wielen (1974):
  radius from the inverse cumulative mass profile, isotropic directions, and
  speeds from the isotropic distribution function by von Neumann rejection.
  The cumulative mass fraction is cut at 0.999 (r <= 38.7 a) and the centre
  of mass position and velocity are removed.

All generators use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_cube(n: int, seed: int):
    """(pos (3,n), vel (3,n), mass (n,)) for the uniform-cube workloads."""
    rng = _rng(seed)
    pos = rng.uniform(-1.0, 1.0, size=(3, n))
    vel = rng.normal(0.0, 0.1, size=(3, n))
    mass = rng.uniform(0.5, 1.0, size=n) / n
    return pos, vel, mass


def _isotropic(rng: np.random.Generator, length: np.ndarray) -> np.ndarray:
    cos_t = rng.uniform(-1.0, 1.0, size=length.shape)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=length.shape)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    return np.stack([length * sin_t * np.cos(phi),
                     length * sin_t * np.sin(phi),
                     length * cos_t])


def plummer(n: int, seed: int, a: float = 1.0, M: float = 1.0, G: float = 1.0,
            mass_cut: float = 0.999):
    """(pos, vel, mass) of an equal-mass Plummer sphere (AHW 1974 sampling)."""
    rng = _rng(seed)
    X = rng.uniform(0.0, mass_cut, size=n)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, r)
    # Speed: v = q v_esc(r), with q distributed as q^2 (1 - q^2)^(7/2) on [0, 1]
    # (max 0.0920 at q^2 = 2/9); von Neumann rejection against 0.1.
    q = np.empty(n)
    filled = 0
    while filled < n:
        k = max(2 * (n - filled), 64)
        qq = rng.uniform(0.0, 1.0, size=k)
        yy = rng.uniform(0.0, 0.1, size=k)
        ok = qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]
        take = min(ok.size, n - filled)
        q[filled:filled + take] = ok[:take]
        filled += take
    v_esc = np.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    vel = _isotropic(rng, q * v_esc)
    mass = np.full(n, M / n)
    pos -= pos.mean(axis=1, keepdims=True)
    vel -= vel.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


def upstream_normal(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """An upstream gradient dL/d(.) ~ N(0, scale^2), shape (3, n)."""
    return _rng(seed).normal(0.0, scale, size=(3, n))


def subset_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct seeded row indices in [0, n), sorted."""
    k = min(k, n)
    return np.sort(_rng(seed).choice(n, size=k, replace=False)).astype(np.int64)


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: size, initial conditions and constants."""
    name: str
    n: int
    steps: int
    ic: str            # "cube" or "plummer"
    eps: float
    dt: float
    seed: int
    plummer_a: float = 1.0
    G: float = 1.0
    ckpt_every: int = 0

    def initial_state(self):
        if self.ic == "cube":
            return uniform_cube(self.n, self.seed)
        return plummer(self.n, self.seed, a=self.plummer_a, M=1.0, G=self.G)

    def rows(self, k: int) -> np.ndarray:
        return subset_rows(self.n, k, self.seed + 100)


# The five workloads: a small FP64 rollout; FP64 vs mixed at 16384 bodies;
# a mixed Plummer rollout at 65536; a forward + adjoint rollout at 8192 with
# checkpoints every 10 steps; and one acceleration + VJP at 262144 on a
# clustered (a = 0.1) Plummer sphere.
WORKLOADS = {
    "cube1024_fp64": Workload("cube1024_fp64", 1024, 100, "cube", 1e-3, 1e-3, 1001),
    "cube16384": Workload("cube16384", 16384, 10, "cube", 1e-3, 1e-3, 1002),
    "plummer65536": Workload("plummer65536", 65536, 10, "plummer", 1e-2, 1e-3, 1003),
    "cube8192_adjoint": Workload("cube8192_adjoint", 8192, 50, "cube", 1e-3, 1e-3,
                                 1004, ckpt_every=10),
    "plummer262144_vjp": Workload("plummer262144_vjp", 262144, 0, "plummer", 1e-3,
                                  1e-3, 1005, plummer_a=0.1),
}
