"""torch.autograd wrappers over the C ABI (no arithmetic of their own).

* ``NBodyAccel``: a = A(x, m); backward calls ``nbody_accel_vjp``.
* ``NBodyRollout``: (x_S, v_S, a_S) from S steps (kick-drift-kick, or the
  paper's half-kick + drift) of (x_0, v_0, m); forward calls ``nbody_step``
  with a checkpoint every K steps,
  backward calls ``nbody_step_adjoint`` (segment recomputation from the
  checkpoints, then the reverse sweep).

Gradients flow to positions, velocities and masses; G, eps and dt are
constants.
"""
from __future__ import annotations

import torch

from . import binding as B


def _zeros_like(ref, g):
    return torch.zeros_like(ref) if g is None else g.contiguous()


class NBodyAccel(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, G, eps, precision):
        pos, mass = pos.contiguous(), mass.contiguous()
        acc = B.nbody_accel(pos, mass, G, eps, precision)
        ctx.save_for_backward(pos, mass)
        ctx.consts = (G, eps, precision)
        return acc

    @staticmethod
    def backward(ctx, gacc):
        pos, mass = ctx.saved_tensors
        G, eps, precision = ctx.consts
        if gacc is None:
            return None, None, None, None, None
        gpos, gmass = B.nbody_accel_vjp(pos, mass, gacc.contiguous(), G, eps,
                                        precision)
        return gpos, gmass, None, None, None


class NBodyRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos0, vel0, mass, G, eps, dt, steps, ckpt_every, precision,
                integrator="kdk"):
        mass = mass.contiguous()
        n = mass.shape[0]
        pos = pos0.detach().clone().contiguous()
        vel = vel0.detach().clone().contiguous()
        acc = torch.empty_like(pos)
        K = max(1, int(ckpt_every))
        ckpt = torch.empty(B.nbody_checkpoint_bytes(n, steps, K) // 8,
                           dtype=torch.float64, device=mass.device)
        B.nbody_step(pos, vel, acc, mass, G, eps, dt, steps, precision,
                     acc_valid=False, ckpt=ckpt, ckpt_every=K, integrator=integrator)
        ctx.save_for_backward(ckpt, mass)
        ctx.consts = (G, eps, dt, int(steps), K, precision, integrator)
        return pos, vel, acc

    @staticmethod
    def backward(ctx, gpos, gvel, gacc):
        ckpt, mass = ctx.saved_tensors
        G, eps, dt, steps, K, precision, integrator = ctx.consts
        n = mass.shape[0]
        ref = torch.empty((3, n), dtype=torch.float64, device=mass.device)
        gx = _zeros_like(ref, gpos).clone()
        gv = _zeros_like(ref, gvel).clone()
        ga = None if gacc is None else gacc.contiguous()
        gx, gv, gm = B.nbody_step_adjoint(ckpt, mass, gx, gv, G, eps, dt, steps,
                                          K, precision, gacc_T=ga,
                                          integrator=integrator)
        return gx, gv, gm, None, None, None, None, None, None, None


def accel(pos, mass, G=1.0, eps=1e-3, precision="fp64"):
    return NBodyAccel.apply(pos, mass, G, eps, B._precision(precision))


def auto_ckpt_every(n, steps, precision="fp64", budget_bytes=1 << 30):
    """The smallest checkpoint interval K whose checkpoint buffer plus the
    adjoint's workspace (which holds K segment positions) fits in
    budget_bytes; K = 1 stores every state and needs no recomputation in the
    reverse sweep (one VJP per step), larger K recompute K - 1 forward
    evaluations per K steps.  Sizes come from the library."""
    steps = int(steps)
    prec = B._precision(precision)
    best = None
    for K in range(1, max(1, steps) + 1):
        need = (B.nbody_checkpoint_bytes(n, steps, K)
                + B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, steps, K, prec))
        if need <= budget_bytes:
            return K
        if best is None or need < best[0]:
            best = (need, K)
    return best[1]


def rollout(pos0, vel0, mass, G=1.0, eps=1e-3, dt=1e-3, steps=1, ckpt_every=10,
            precision="fp64", integrator="kdk", memory_budget=1 << 30):
    """(x_S, v_S, a_S) with a checkpointed adjoint.  ckpt_every="auto" picks
    the smallest interval whose checkpoints and adjoint workspace fit in
    memory_budget bytes (auto_ckpt_every)."""
    if ckpt_every == "auto":
        ckpt_every = auto_ckpt_every(mass.shape[0], steps, precision, memory_budget)
    return NBodyRollout.apply(pos0, vel0, mass, G, eps, dt, steps, ckpt_every,
                              B._precision(precision), integrator)
