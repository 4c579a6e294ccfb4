#!/usr/bin/env python3
"""Benchmark of the all-pairs N-body hot path on one MI355X.

Headline workload (plummer262144_vjp): 262144 bodies of a clustered Plummer
sphere (scale radius 0.1, total mass 1, equal masses), G = 1, Plummer
softening eps = 1e-3, and an upstream gradient dL/da ~ N(0, 1) -- the largest
configuration that runs on one GPU.  One benchmark step is one pass of the
force + adjoint hot path over that input:

  * near / far precisions only: nbody_morton_sort puts the bodies (and their
    dL/da, carried as the sort's optional vector) in Morton order;
  * nbody_accel: the accelerations of all bodies (N^2 pairs);
  * nbody_accel_vjp: dL/dx and dL/dm for the upstream dL/da (N^2 pairs).

`value` = N^2 / (step time) in G body-pair interactions/s: the paper's
convention (section 4.1: N^2 pairs per evaluation, self pairs included), with
the forward and its adjoint counted together as one pass over the pairs
(forward + adjoint rate = N^2 S / (t_fwd + t_bwd), S = 1 here).  Inputs are
resident in HBM before the timed region starts.

The default precision is NBODY_MIXED_NF, the fastest FP32-pair mode whose
largest per-body relative acceleration error on this workload stays within
the stated 1e-6 (checked against the FP64 oracle on the 1024 seeded rows plus
the 256 bodies nearest the centre of mass, and reported as `error`).

Also on the same JSON line: every precision's step at the headline workload
with its errors (`legs`); the roofline position of the dominant kernel (the
VJP) and of the forward, each timed with HIP events on the stream it runs on;
kernel-level rates at N = 65536 (Plummer a = 1, eps = 1e-2: forward, energy
diagnostics, FP32-state forward) and one eighth of the N = 262144 target
rows; the N = 16384 forward + checkpointed-adjoint rollouts; the N = 1024
FP64 rollout; the N = 8192 50-step forward + adjoint; and the FP64 oracle
timed on the host cores (cpu_baseline, cpu_oracle_by_workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("G body-pair interactions/s (FP64 vs mixed, fwd and fwd+adjoint) "
          "at stated error")
WORKLOAD = "plummer262144_vjp"
DEFAULT_PRECISION = "mixed_nf"
ERROR_TARGET = 1e-6          # largest per-body relative acceleration error
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32, published
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64, published
# Flops per body pair, counting add/sub/mul as 1, FMA as 2 and the reciprocal
# square root as 2: the force pair (3 sub, 3 FMA, rsqrt, 3 mul, 3 FMA) is the
# paper's 20.  The VJP pair, in the split form the kernels run (3 sub, 3 FMA,
# rsqrt, 2 mul for y^2 and y^3, 1 mul + 2 FMA for gbar_j.e and again for
# gbar_k.e, 1 mul + 1 FMA for e.h, 1 FMA for the mass term, 2 mul, 3 + 1 + 3
# FMA into the sums) is 44 (48 with h formed per pair: 3 sub, 3 FMA, rsqrt,
# 2 mul, 3 mul + 3 FMA for h, 1 mul + 2 FMA twice for e.h and gbar.e, 1 FMA,
# 2 mul, 6 FMA).
# The potential pair (diagnostics) is 3 sub, 3 FMA, rsqrt, 1 FMA = 13.
FLOPS_PER_PAIR = {"accel": 20, "vjp": 44, "diag": 13}
DTYPE = {"fp64": "f64", "mixed": "f32-pair/f64-acc",
         "mixed_d64": "f32-pair(f64-diff)/f64-acc",
         "mixed_nf": "f32-pair(near f64-diff, far recentred)/f64-acc",
         "mixed_nf64": "near f64-pair, far f32-pair(recentred)/f64-acc",
         "mixed_ds": "f32-pair(two-float diff)/f64-acc"}
PRECS = ("fp64", "mixed", "mixed_d64", "mixed_nf", "mixed_nf64", "mixed_ds")
SORTED = ("mixed_nf", "mixed_nf64")   # run on the bodies in Morton order
KERNEL_KIND = {"accel": "accel_kernel", "vjp": "vjp_kernel"}
# HBM bytes per launch of a roofline kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, each scaled by what the counter reads for a
# 64 MiB device copy), keyed by (kind, precision, N).  Each record names the
# kernel sources it was taken on (first 16 hex digits of their SHA-256) and
# is reported as null for any other source.
MEASURED_TRAFFIC = {
    # profiles/vjp_nf_kernel_plummer262144_counters.md: 555.5 MB fetched +
    # 134.2 MB written by the second vjp_nf_kernel launch
    ("vjp", "mixed_nf", 262144): {"bytes": 689700238, "src_sha256": "426be688f1d855fe"},
    # same file: 212.4 MB + 50.3 MB, accel_nf_kernel
    ("accel", "mixed_nf", 262144): {"bytes": 262738440, "src_sha256": "426be688f1d855fe"},
    # profiles/accel_kernel_plummer65536_mixed.md: 16.8 MB + 50.3 MB
    ("accel", "mixed", 65536): {"bytes": 67169572, "src_sha256": "426be688f1d855fe"},
}
# the kernels and the launch plans (nbody_api.hip), which set the split
# partials' bytes
KERNEL_SRC = [os.path.join(ROOT, "paper_2203_08263_amd", "csrc", f)
              for f in ("nbody_kernels.hip", "nbody_nearfar.hip", "nbody_device.h",
                        "nbody_api.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def warm(torch, fn, seconds=0.1):
    """Run fn untimed for about `seconds` so the GPU clock has ramped up
    (after host-side work the first launches run up to ~12 % slower)."""
    t0 = time.perf_counter()
    while True:
        fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return


def event_ms(torch, fn, reps, warmup=1):
    """Average duration of fn in ms, HIP events on torch's current stream
    (the stream every library call of the binding is enqueued on)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_src_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Headline:
    """The headline workload resident on the GPU, one precision's step."""

    def __init__(self, torch, B, inputs, w):
        self.torch, self.B, self.w = torch, B, w
        dev = torch.device("cuda:0")
        self.dev = dev
        T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
        pos, _, mass = w.initial_state()
        self.g = inputs.upstream_normal(w.n, w.seed + 400)
        self.np_state = (pos, mass)
        self.P0, self.M0, self.G0 = T(pos), T(mass), T(self.g)
        n = w.n
        self.A = torch.empty_like(self.P0)
        self.GX = torch.empty_like(self.P0)
        self.GM = torch.empty_like(self.M0)
        self.perm = torch.empty(n, dtype=torch.int64, device=dev)
        self.Ps, self.Gs = torch.empty_like(self.P0), torch.empty_like(self.P0)
        self.Ms = torch.empty_like(self.M0)
        nb = max([B.nbody_workspace_bytes(op, n, 0, 1, p)
                  for p in PRECS for op in (B.NBODY_OP_ACCEL, B.NBODY_OP_VJP)] +
                 [B.nbody_workspace_bytes(B.NBODY_OP_MORTON_SORT, n, 0, 1, 0), 256])
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)

    def sort(self):
        """Bodies and their dL/da in Morton order (into Ps, Gs, Ms, perm)."""
        self.B.nbody_morton_sort(self.P0, self.M0, self.G0, workspace=self.ws,
                                 perm=self.perm, pos_out=self.Ps, vel_out=self.Gs,
                                 mass_out=self.Ms)

    def inputs(self, p):
        if p in SORTED:
            return self.Ps, self.Ms, self.Gs
        return self.P0, self.M0, self.G0

    def accel(self, p):
        w = self.w
        P, M, _ = self.inputs(p)
        self.B.nbody_accel(P, M, w.G, w.eps, p, out=self.A, workspace=self.ws)

    def vjp(self, p):
        w = self.w
        P, M, Gt = self.inputs(p)
        self.B.nbody_accel_vjp(P, M, Gt, w.G, w.eps, p, gpos=self.GX, gmass=self.GM,
                               workspace=self.ws)

    def step(self, p):
        if p in SORTED:
            self.sort()
        self.accel(p)
        self.vjp(p)

    def results(self, p):
        """(a, dL/dx, dL/dm) as NumPy arrays in the generated body order."""
        import numpy as np
        self.torch.cuda.synchronize()
        a, gx, gm = (t.cpu().numpy() for t in (self.A, self.GX, self.GM))
        if p in SORTED:
            perm = self.perm.cpu().numpy()
            out = []
            for t in (a, gx, gm):
                back = np.empty_like(t)
                back[..., perm] = t
                out.append(back)
            a, gx, gm = out
        return a, gx, gm


def error_rows(w, pos, mass):
    """The 1024 seeded rows plus the 256 bodies nearest the centre of mass
    (where the net acceleration almost cancels and relative errors peak)."""
    import numpy as np
    com = (mass * pos).sum(axis=1) / mass.sum()
    central = np.argsort(np.linalg.norm(pos - com[:, None], axis=0), kind="stable")[:256]
    return np.union1d(w.rows(1024), central)


def roofline(torch, fn, n, kind, p, launches):
    """Average launch duration of the all-pairs kernel of `kind` at N = n
    (HIP events on the stream the call launches on, after a clock ramp), and
    its position against the vector peak of its arithmetic type.  A call is
    the all-pairs kernel plus the O(N) split reduction (and, for the near /
    far modes, the O(N) bounding-box pass and, at 2^32 pairs or more, the
    dispatch-order pass)."""
    warm(torch, fn)
    ms = event_ms(torch, fn, launches)
    flops = FLOPS_PER_PAIR[kind] * float(n) * n
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
    rec = MEASURED_TRAFFIC.get((kind, p, n))
    traffic = None
    if rec is not None and kernel_src_hash() == rec["src_sha256"]:
        traffic = rec["bytes"]
    name = KERNEL_KIND[kind] if p not in SORTED else KERNEL_KIND[kind].replace("_kernel",
                                                                              "_nf_kernel")
    return {"kernel": "%s (%s), N=%d" % (name, p, n), "bound": "alu",
            "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "traffic_unit": "HBM bytes per launch", "avg_launch_ms": round(ms, 4),
            "flops_per_pair": FLOPS_PER_PAIR[kind],
            "algorithmic_flops_per_launch": flops}


def headline_legs(torch, hd, oracle_ref):
    """Every precision's step at the headline workload, with its errors."""
    import numpy as np
    from paper_2203_08263_amd import metrics
    w = hd.w
    n2 = float(w.n) * w.n
    rows, ra, rx, rm = oracle_ref
    legs = {}
    for p in PRECS:
        warm(torch, lambda: hd.step(p))
        step_ms = event_ms(torch, lambda: hd.step(p), 3)
        acc_ms = event_ms(torch, lambda: hd.accel(p), 3)
        vjp_ms = event_ms(torch, lambda: hd.vjp(p), 3)
        leg = {"step_ms": round(step_ms, 4), "G_int_s": round(n2 / (step_ms * 1e-3) / 1e9, 1),
               "accel_ms": round(acc_ms, 4), "vjp_ms": round(vjp_ms, 4),
               "accel_G_int_s": round(n2 / (acc_ms * 1e-3) / 1e9, 1),
               "vjp_G_int_s": round(n2 / (vjp_ms * 1e-3) / 1e9, 1),
               "vjp_over_fwd": round(vjp_ms / acc_ms, 3)}
        if p in SORTED:
            leg["sort_ms"] = round(event_ms(torch, hd.sort, 3), 4)
        hd.step(p)
        a, gx, gm = hd.results(p)
        e = metrics.rel_errors(a[:, rows], ra)
        leg["accel_error"] = {k: float("%.3e" % v) for k, v in e.items()}
        leg["vjp_error_normwise"] = {"dL/dx": float("%.3e" % metrics.normwise(gx[:, rows], rx)),
                                     "dL/dm": float("%.3e" % metrics.normwise(gm[rows], rm))}
        leg["meets_error_target"] = bool(e["E_max"] <= ERROR_TARGET)
        legs[p] = leg
        log("bench: leg %s %s" % (p, leg))
    _ = np
    return legs


def shape_legs(torch, B, inputs):
    """Kernel-level throughput: the forward and energy diagnostics at
    N = 65536 (Plummer, a = 1, eps = 1e-2; also the FP32-state forward and the
    Morton sort), and one device's share when the N = 262144 target rows are
    split eight ways (rows 3/8 .. 4/8 against all sources, through the
    row-range entry points), each timed with HIP events over back-to-back
    calls (kernel + split reduce)."""
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    out = {}
    for name, precs, kinds in (("plummer65536", PRECS, ("accel", "diag")),
                               ("plummer262144_vjp", PRECS, ("accel_share8", "vjp_share8"))):
        w = inputs.WORKLOADS[name]
        pos, vel, mass = w.initial_state()
        P0, M0, V0 = T(pos), T(mass), T(vel)
        D = torch.empty(9, dtype=torch.float64, device=dev)
        G0 = T(inputs.upstream_normal(w.n, w.seed + 400))
        sort_fn = lambda: B.nbody_morton_sort(P0, M0, V0)  # noqa
        warm(torch, sort_fn)
        sort_ms = event_ms(torch, sort_fn, 5, warmup=0)
        perm, Ps, Vs, Ms = sort_fn()
        Gs = G0[:, perm].contiguous()
        A = torch.empty_like(P0)
        share = w.n // 8
        r0 = 3 * share
        As = torch.empty((3, share), dtype=torch.float64, device=dev)
        GXs = torch.empty((3, share), dtype=torch.float64, device=dev)
        GMs = torch.empty(share, dtype=torch.float64, device=dev)
        res = {"morton_sort_ms": round(sort_ms, 4)}
        if name == "plummer65536":
            # FP32 state (the paper's single-precision variant): forward only
            Pf, Mf = P0.float(), M0.float()
            Af = torch.empty_like(Pf)
            wsf = torch.empty(max(B.nbody_f32_workspace_bytes(B.NBODY_OP_ACCEL, w.n), 256),
                              dtype=torch.uint8, device=dev)
            fnf = lambda: B.nbody_accel_f32(Pf, Mf, w.G, w.eps, out=Af, workspace=wsf)  # noqa
            warm(torch, fnf)
            fms = event_ms(torch, fnf, 20, warmup=0)
            fips = float(w.n) * w.n / (fms * 1e-3)
            res["accel_f32_state"] = {
                "ms": round(fms, 4), "G_int_s": round(fips / 1e9, 1),
                "TFLOP_s": round(fips * 20 / 1e12, 2),
                "frac_of_vector_peak": round(fips * 20 / 1e12 / PEAK_FP32_TFLOPS, 4)}
        for p in precs:
            if p in SORTED:
                P, M, Vt, Gt = Ps, Ms, Vs, Gs
            else:
                P, M, Vt, Gt = P0, M0, V0, G0
            ws = torch.empty(max(B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, w.n, 0, 1, p),
                                 B.nbody_workspace_bytes(B.NBODY_OP_DIAGNOSTICS, w.n, 0, 1,
                                                         p),
                                 B.nbody_rows_workspace_bytes(B.NBODY_OP_ACCEL, w.n, share, p),
                                 B.nbody_rows_workspace_bytes(B.NBODY_OP_VJP, w.n, share, p),
                                 256),
                             dtype=torch.uint8, device=dev)
            for kind in kinds:
                if kind == "accel":
                    fn = lambda: B.nbody_accel(P, M, w.G, w.eps, p, out=A, workspace=ws)  # noqa
                elif kind == "accel_share8":
                    fn = lambda: B.nbody_accel_rows(P, M, r0, share, w.G, w.eps, p,  # noqa
                                                    out=As, workspace=ws)
                elif kind == "vjp_share8":
                    fn = lambda: B.nbody_accel_vjp_rows(  # noqa
                        P, M, Gt, r0, share, w.G, w.eps, p, gpos=GXs, gmass=GMs,
                        workspace=ws)
                else:
                    fn = lambda: B.nbody_diagnostics(P, Vt, M, w.G, w.eps, p, out=D,  # noqa
                                                     workspace=ws)
                rows = share if kind.endswith("_share8") else w.n
                warm(torch, fn)
                ms = event_ms(torch, fn, 20 if w.n <= 65536 else 8, warmup=0)
                ips = float(rows) * w.n / (ms * 1e-3)
                peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
                fl = FLOPS_PER_PAIR[kind.replace("_share8", "")]
                res["%s_%s" % (kind, p)] = {
                    "ms": round(ms, 4), "G_int_s": round(ips / 1e9, 1),
                    "TFLOP_s": round(ips * fl / 1e12, 2),
                    "frac_of_vector_peak": round(ips * fl / 1e12 / peak, 4)}
        out[name] = res
    return out


class Rollout16384:
    """The N = 16384 uniform cube (eps = 1e-3, dt = 1e-3): 10 KDK steps
    forward with a checkpoint every 5, then the adjoint for a seeded
    upstream dL/dx_10 ~ N(0, 1) (segment recomputation plus 11 VJPs)."""
    CKPT_EVERY = 5

    def __init__(self, torch, B, inputs):
        self.torch, self.B = torch, B
        w = self.w = inputs.WORKLOADS["cube16384"]
        dev = self.dev = torch.device("cuda:0")
        T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
        pos, vel, mass = w.initial_state()
        self.np_state = (pos, vel, mass)
        self.gx_T = inputs.upstream_normal(w.n, w.seed + 500)
        self.P0, self.V0, self.M, self.GX0 = T(pos), T(vel), T(mass), T(self.gx_T)
        n = w.n
        self.P, self.V = torch.empty_like(self.P0), torch.empty_like(self.V0)
        self.A = torch.empty_like(self.P0)
        self.GX, self.GV = torch.empty_like(self.P0), torch.empty_like(self.P0)
        self.GM = torch.empty_like(self.M)
        self.CK = torch.empty(B.nbody_checkpoint_bytes(n, w.steps, self.CKPT_EVERY) // 8,
                              dtype=torch.float64, device=dev)
        self.perm, self.P0s, self.V0s, self.Ms = B.nbody_morton_sort(self.P0, self.M,
                                                                     self.V0)
        self.GX0s = self.GX0[:, self.perm].contiguous()
        self.P0f, self.V0f, self.Mf = (t.float() for t in (self.P0, self.V0, self.M))
        self.Pf, self.Vf = torch.empty_like(self.P0f), torch.empty_like(self.V0f)
        self.Af0 = B.nbody_accel_f32(self.P0f, self.Mf, w.G, w.eps)
        self.Af = torch.empty_like(self.Af0)
        self.wsf = torch.empty(max(B.nbody_f32_workspace_bytes(B.NBODY_OP_STEP, n), 256),
                               dtype=torch.uint8, device=dev)
        self.A0, self.ws = {}, {}
        for p in PRECS:
            P0, _, M, _ = self.state0(p)
            self.A0[p] = B.nbody_accel(P0, M, w.G, w.eps, p)
            nb = max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, w.steps, self.CKPT_EVERY, p),
                     B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, w.steps,
                                             self.CKPT_EVERY, p), 256)
            self.ws[p] = torch.empty(nb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()

    def state0(self, p):
        if p in SORTED:
            return self.P0s, self.V0s, self.Ms, self.GX0s
        return self.P0, self.V0, self.M, self.GX0

    def forward(self, p, ck=None, K=None, ws=None):
        w, B = self.w, self.B
        P0, V0, M, _ = self.state0(p)
        self.P.copy_(P0)
        self.V.copy_(V0)
        self.A.copy_(self.A0[p])
        B.nbody_step(self.P, self.V, self.A, M, w.G, w.eps, w.dt, w.steps, p,
                     acc_valid=True, ckpt=self.CK if ck is None else ck,
                     ckpt_every=K or self.CKPT_EVERY,
                     workspace=self.ws[p] if ws is None else ws)

    def adjoint(self, p, ck=None, K=None, ws=None):
        w, B = self.w, self.B
        _, _, M, GX0 = self.state0(p)
        self.GX.copy_(GX0)
        self.GV.zero_()
        B.nbody_step_adjoint(self.CK if ck is None else ck, M, self.GX, self.GV, w.G,
                             w.eps, w.dt, w.steps, K or self.CKPT_EVERY, p,
                             gmass=self.GM, workspace=self.ws[p] if ws is None else ws)

    def forward_f32(self):
        w, B = self.w, self.B
        self.Pf.copy_(self.P0f)
        self.Vf.copy_(self.V0f)
        self.Af.copy_(self.Af0)
        B.nbody_step_f32(self.Pf, self.Vf, self.Af, self.Mf, w.G, w.eps, w.dt, w.steps,
                         acc_valid=True, workspace=self.wsf)

    def legs(self, main_p):
        torch, w = self.torch, self.w
        n2s = float(w.n) * w.n * w.steps
        out = {"workload": "cube16384: N=16384 uniform cube, %d KDK steps forward "
                           "(checkpoint every %d) + adjoint for dL/dx_%d ~ N(0,1)"
                           % (w.steps, self.CKPT_EVERY, w.steps)}
        finals = {}
        for q in PRECS:
            warm(torch, lambda: self.forward(q))
            fms = event_ms(torch, lambda: self.forward(q), 10)
            sms = event_ms(torch, lambda: (self.forward(q), self.adjoint(q)), 5)
            out[q] = {"fwd_G_int_s": round(n2s / (fms * 1e-3) / 1e9, 1),
                      "fwd_ms": round(fms, 4),
                      "fwd_adj_G_int_s": round(n2s / (sms * 1e-3) / 1e9, 1),
                      "fwd_adj_ms": round(sms, 4),
                      "bwd_over_fwd": round((sms - fms) / fms, 3)}
            self.forward(q)
            torch.cuda.synchronize()
            finals[q] = (self.P.cpu().numpy(), self.V.cpu().numpy(),
                         self.state0(q)[2].cpu().numpy())
            log("bench: cube16384 leg %s %s" % (q, out[q]))
        sweep = {}
        for K in (1, self.CKPT_EVERY, w.steps):
            ck = torch.empty(self.B.nbody_checkpoint_bytes(w.n, w.steps, K) // 8,
                             dtype=torch.float64, device=self.dev)
            wsk = torch.empty(max(self.B.nbody_workspace_bytes(self.B.NBODY_OP_STEP, w.n,
                                                               w.steps, K, main_p),
                                  self.B.nbody_workspace_bytes(
                                      self.B.NBODY_OP_STEP_ADJOINT, w.n, w.steps, K,
                                      main_p)),
                              dtype=torch.uint8, device=self.dev)
            fn = lambda: (self.forward(main_p, ck, K, wsk),  # noqa
                          self.adjoint(main_p, ck, K, wsk))
            warm(torch, fn)
            kms = event_ms(torch, fn, 5)
            sweep["K%d" % K] = {"fwd_adj_G_int_s": round(n2s / (kms * 1e-3) / 1e9, 1),
                                "fwd_adj_ms": round(kms, 4),
                                "checkpoint_MB": round(ck.numel() * 8 / 1e6, 2)}
        out["%s_ckpt_every" % main_p] = sweep
        warm(torch, self.forward_f32)
        fms = event_ms(torch, self.forward_f32, 10)
        out["f32_state"] = {"fwd_G_int_s": round(n2s / (fms * 1e-3) / 1e9, 1),
                            "fwd_ms": round(fms, 4)}
        return out, finals


def adjoint_leg(torch, B, inputs):
    """The forward + adjoint configuration: N = 8192 uniform cube, 50 KDK
    steps with a checkpoint every 10, then the reverse sweep (which
    recomputes each segment).  Step-level t_bwd / t_fwd per precision; and,
    as `mixed_auto_K`, the same with the interval rollout(ckpt_every="auto")
    picks for a 1 GiB budget (every state stored: no recomputation)."""
    from paper_2203_08263_amd import auto_ckpt_every
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS["cube8192_adjoint"]
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    pos, vel, mass = w.initial_state()
    P0, V0, M = T(pos), T(vel), T(mass)
    GX0 = T(inputs.upstream_normal(w.n, w.seed + 500))
    P, V, A = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(P0)
    GX, GV, GM = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(M)
    out = {"workload": "cube8192_adjoint: N=%d, %d KDK steps, checkpoint every %d"
                       % (w.n, w.steps, w.ckpt_every)}
    for p, K, key in (("mixed", w.ckpt_every, "mixed"), ("fp64", w.ckpt_every, "fp64"),
                      ("mixed", auto_ckpt_every(w.n, w.steps, "mixed"), "mixed_auto_K")):
        CK = torch.empty(B.nbody_checkpoint_bytes(w.n, w.steps, K) // 8,
                         dtype=torch.float64, device=dev)
        ws = torch.empty(max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, w.n, w.steps, K, p),
                             B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, w.n,
                                                     w.steps, K, p)),
                         dtype=torch.uint8, device=dev)

        def fwd():
            P.copy_(P0)
            V.copy_(V0)
            B.nbody_step(P, V, A, M, w.G, w.eps, w.dt, w.steps, p, ckpt=CK,
                         ckpt_every=K, workspace=ws)

        def bwd():
            GX.copy_(GX0)
            GV.zero_()
            B.nbody_step_adjoint(CK, M, GX, GV, w.G, w.eps, w.dt, w.steps, K, p,
                                 gmass=GM, workspace=ws)
        warm(torch, lambda: (fwd(), bwd()))
        tf = event_ms(torch, fwd, 3)
        fwd()   # the adjoint reads this forward's checkpoints
        tb = event_ms(torch, bwd, 3, warmup=0)
        out[key] = {"ckpt_every": K, "fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                    "bwd_over_fwd": round(tb / tf, 3),
                    "fwd_adj_G_int_s": round(float(w.n) * w.n * w.steps
                                             / ((tf + tb) * 1e-3) / 1e9, 1)}
    return out


def small_rollout_leg(torch, B, inputs):
    """The launch-bound configuration: N = 1024, 100 FP64 KDK steps.  Timed
    eagerly and as a replayed HIP graph of the same nbody_step call (state
    restored by device copies before each run)."""
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS["cube1024_fp64"]
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    pos, vel, mass = w.initial_state()
    P0, V0, M = T(pos), T(vel), T(mass)
    A0 = B.nbody_accel(P0, M, w.G, w.eps, "fp64")
    P, V, A = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(P0)
    ws = torch.empty(max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, w.n, w.steps, 1, "fp64"),
                         256), dtype=torch.uint8, device=dev)

    def run():
        P.copy_(P0)
        V.copy_(V0)
        A.copy_(A0)
        B.nbody_step(P, V, A, M, w.G, w.eps, w.dt, w.steps, "fp64", acc_valid=True,
                     workspace=ws)

    warm(torch, run)
    eager = event_ms(torch, run, 20)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    warm(torch, g.replay)
    graph = event_ms(torch, g.replay, 20)
    pairs = float(w.n) * w.n * w.steps
    return {"workload": "%s: N=%d, %d FP64 KDK steps" % (w.name, w.n, w.steps),
            "eager_ms": round(eager, 4), "graph_ms": round(graph, 4),
            "eager_G_int_s": round(pairs / (eager * 1e-3) / 1e9, 1),
            "graph_G_int_s": round(pairs / (graph * 1e-3) / 1e9, 1)}


def cpu_baseline(hd, target_s=12.0):
    """The FP64 oracle on the host cores over a bounded sample of the
    headline workload: the accelerations and the VJP rows of R seeded bodies
    against all N sources (the same per-row work as the GPU's pass),
    counted like `value`: R * N pairs / (t_accel_rows + t_vjp_rows).  R is
    grown from a short probe until the sample takes about target_s."""
    import oracle
    w = hd.w
    pos, mass = hd.np_state
    g = hd.g

    def run(k):
        rows = w.rows(k)
        t0 = time.perf_counter()
        oracle.accel_rows(pos, mass, w.G, w.eps, rows)
        oracle.accel_vjp_rows(pos, mass, g, w.G, w.eps, rows)
        return time.perf_counter() - t0

    k = 512
    t = run(k)
    k = int(min(w.n, max(k, k * target_s / max(t, 1e-3))))
    k = max(512, k // 512 * 512)
    t = run(k)
    return {"value": round(float(k) * w.n / t / 1e9, 4), "unit": "G interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle: accelerations and VJP (dL/dx, dL/dm) of %d seeded "
                      "bodies against all %d sources of the headline workload, "
                      "%.2f s; %d x %d pairs counted once for both, as value counts "
                      "N^2 per forward + VJP" % (k, w.n, t, k, w.n)}


def cpu_by_workload(inputs, r16):
    """The FP64 oracle on a bounded sample of each other workload (a few
    seconds in all), for the per-workload GPU legs beside it."""
    import numpy as np
    import oracle
    out = {}

    def rate(pairs, fn):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        return round(pairs / dt / 1e9, 3), round(dt, 3)

    w = inputs.WORKLOADS["cube1024_fp64"]
    pos, vel, mass = w.initial_state()
    out["cube1024_fp64"] = dict(zip(("G_int_s", "s"), rate(
        float(w.n) ** 2 * w.steps,
        lambda: oracle.step(pos, vel, mass, w.G, w.eps, w.dt, w.steps))),
        sample="the whole 100-step rollout")
    w = inputs.WORKLOADS["plummer65536"]
    pos, vel, mass = w.initial_state()
    rows = w.rows(4096)
    out["plummer65536"] = dict(zip(("G_int_s", "s"), rate(
        float(len(rows)) * w.n,
        lambda: oracle.accel_rows(pos, mass, w.G, w.eps, rows))),
        sample="forces on the 4096 seeded rows")
    w = inputs.WORKLOADS["cube8192_adjoint"]
    pos, vel, mass = w.initial_state()
    out["cube8192_adjoint"] = dict(zip(("G_int_s", "s"), rate(
        float(w.n) ** 2 * w.steps,
        lambda: oracle.step(pos, vel, mass, w.G, w.eps, w.dt, w.steps))),
        sample="the 50-step forward rollout")
    w = r16.w
    pos, vel, mass = r16.np_state
    out["cube16384"] = dict(zip(("G_int_s", "s"), rate(
        float(w.n) ** 2 * w.steps,
        lambda: oracle.step_adjoint(pos, vel, mass, w.G, w.eps, w.dt, w.steps,
                                    r16.gx_T, np.zeros((3, w.n))))),
        sample="the 10-step forward + exact reverse sweep (all positions stored), "
               "counted like the GPU's forward + adjoint legs")
    return out


def rollout_errors(r16, finals, main_p):
    """Energy drift of every precision's 10-step cube16384 rollout (FP64
    oracle energy; bodies in Morton order for the near / far modes: the
    energy does not depend on the order)."""
    import oracle
    w = r16.w
    pos, vel, mass = r16.np_state
    e0 = sum(oracle.energy(pos, vel, mass, w.G, w.eps))
    out = {}
    for q, (xq, vq, mq) in finals.items():
        eq = sum(oracle.energy(xq, vq, mq, w.G, w.eps))
        out["energy_drift_cube16384_%s_%dsteps" % (q, w.steps)] = float(
            "%.3e" % (abs(eq - e0) / abs(e0)))
    return out


def profile_mode(torch, B, inputs, args):
    """Counter-collection mode: a 64 MiB device copy (the traffic
    calibration) then --steps calls of one all-pairs kernel on one workload
    (bodies Morton-ordered first for the near / far modes); no JSON line."""
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    w = inputs.WORKLOADS[args.profile_workload]
    pos, _, mass = w.initial_state()
    P, M = T(pos), T(mass)
    G = T(inputs.upstream_normal(w.n, w.seed + 400))
    p = args.precision
    if p in SORTED:
        perm, P, G, M = B.nbody_morton_sort(P, M, G)
    A, GX, GM = torch.empty_like(P), torch.empty_like(P), torch.empty_like(M)
    src = torch.ones(8 << 20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)                       # calibration: 64 MiB read + write
    torch.cuda.synchronize()
    for _ in range(args.steps):
        if args.profile == "accel":
            B.nbody_accel(P, M, w.G, w.eps, p, out=A)
        else:
            B.nbody_accel_vjp(P, M, G, w.G, w.eps, p, gpos=GX, gmass=GM)
    torch.cuda.synchronize()
    log("bench: profile mode done (%s, %s, %s, %d calls)" % (args.profile, p, w.name,
                                                            args.steps))
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default=DEFAULT_PRECISION, choices=PRECS)
    ap.add_argument("--no-legs", action="store_true",
                    help="time only the headline step and its roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads' legs")
    ap.add_argument("--profile", choices=["accel", "vjp"], default=None,
                    help="counter-collection mode (see profile_mode)")
    ap.add_argument("--profile-workload", default=WORKLOAD,
                    help="workload of --profile (default: the headline's)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2203_08263_amd import binding as B
    from paper_2203_08263_amd import inputs, metrics

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    B.load_library()
    if args.profile:
        return profile_mode(torch, B, inputs, args)

    w = inputs.WORKLOADS[WORKLOAD]
    p = args.precision
    hd = Headline(torch, B, inputs, w)
    n2 = float(w.n) * w.n

    # main timed region: K whole steps of the hot path
    log("bench: %s, precision %s, %d warmup + %d timed steps" % (w.name, p, args.warmup,
                                                                args.steps))
    for _ in range(args.warmup):
        hd.step(p)
    torch.cuda.synchronize()   # one process, one GPU: no barrier to take
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        hd.step(p)
    e1.record()
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    ms = e0.elapsed_time(e1) / args.steps
    value = n2 / (ms * 1e-3) / 1e9
    log("bench: %.3f ms/step (events), %.3f ms/step (wall), %.1f G int/s"
        % (ms, wall_ms, value))

    # stated error of the timed step's results against the FP64 oracle
    import oracle
    pos, mass = hd.np_state
    rows = error_rows(w, pos, mass)
    ra = oracle.accel_rows(pos, mass, w.G, w.eps, rows)
    rx, rm = oracle.accel_vjp_rows(pos, mass, hd.g, w.G, w.eps, rows)
    a, gx, gm = hd.results(p)
    e = metrics.rel_errors(a[:, rows], ra)
    error = {"rows": "the 1024 seeded rows + the 256 bodies nearest the centre of "
                     "mass (%d rows), FP64 oracle" % len(rows),
             "accel": {k: float("%.3e" % v) for k, v in e.items()},
             "vjp_normwise": {"dL/dx": float("%.3e" % metrics.normwise(gx[:, rows], rx)),
                              "dL/dm": float("%.3e" % metrics.normwise(gm[rows], rm))},
             "E_max_target": ERROR_TARGET,
             "meets_error_target": bool(e["E_max"] <= ERROR_TARGET)}
    log("bench: error %s" % error)

    # roofline of the dominant kernel (the VJP: about twice the forward) and
    # of the forward, at the headline size, on the headline's inputs
    if p in SORTED:
        hd.sort()
    roof = roofline(torch, lambda: hd.vjp(p), w.n, "vjp", p, 8)
    roof_fwd = roofline(torch, lambda: hd.accel(p), w.n, "accel", p, 8)
    log("bench: roofline vjp %s" % roof)
    log("bench: roofline accel %s" % roof_fwd)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "G interactions/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[p],
           "data": "synthetic",
           "config": {"workload": "%s: N=%d Plummer sphere (scale radius %g, total mass "
                                  "1, equal masses), eps=%g, G=%g, dL/da ~ N(0,1); one "
                                  "step = %snbody_accel + nbody_accel_vjp, precision %s"
                                  % (w.name, w.n, w.plummer_a, w.eps, w.G,
                                     "nbody_morton_sort + " if p in SORTED else "", p),
                      "n": w.n, "precision": p, "parallelism": "single GPU"},
           "error": error, "roofline": roof, "roofline_forward": roof_fwd,
           "vjp_over_fwd_kernel": round(roof["avg_launch_ms"] / roof_fwd["avg_launch_ms"], 3)}
    if not args.no_legs:
        log("bench: every precision at the headline workload")
        out["legs"] = headline_legs(torch, hd, (rows, ra, rx, rm))
    if not args.no_extras:
        log("bench: other workloads")
        extras = {}
        # the N = 65536 mixed forward (60 %-of-peak target) on its own workload
        w3 = inputs.WORKLOADS["plummer65536"]
        pos3, _, mass3 = w3.initial_state()
        P3 = torch.tensor(pos3, dtype=torch.float64, device=hd.dev)
        M3 = torch.tensor(mass3, dtype=torch.float64, device=hd.dev)
        A3 = torch.empty_like(P3)
        out["roofline_forward_plummer65536"] = roofline(
            torch, lambda: B.nbody_accel(P3, M3, w3.G, w3.eps, "mixed", out=A3),
            w3.n, "accel", "mixed", 20)
        extras["shapes"] = shape_legs(torch, B, inputs)
        r16 = Rollout16384(torch, B, inputs)
        extras["cube16384"], finals = r16.legs("mixed")
        extras["cube1024_fp64_rollout"] = small_rollout_leg(torch, B, inputs)
        extras["cube8192_adjoint"] = adjoint_leg(torch, B, inputs)
        out["extras"] = extras
        out["error"].update(rollout_errors(r16, finals, "mixed"))
        log("bench: extras %s" % extras)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (FP64 oracle on the host cores)")
        out["cpu_baseline"] = cpu_baseline(hd)
        if not args.no_extras:
            out["cpu_oracle_by_workload"] = cpu_by_workload(inputs, r16)
    else:
        out["cpu_baseline"] = None
    _ = np
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
