#!/usr/bin/env python3
"""Benchmark of the all-pairs N-body hot path on one MI355X.

Workload: 16384 bodies in a uniform cube (positions U(-1,1)^3, velocities
N(0, 0.1^2), masses U(0.5,1)/N), G = 1, Plummer softening eps = 1e-3,
dt = 1e-3, 10 kick-drift-kick steps -- the FP64-vs-mixed configuration.
One benchmark step is one pass of the whole hot path over that input:

  * forward: 10 KDK steps (nbody_step, acceleration of x_0 already cached)
    writing a checkpoint every 5 steps;
  * reverse: nbody_step_adjoint for a seeded upstream dL/dx_10 ~ N(0,1)
    (segment recomputation from the checkpoints plus 11 VJPs).

`value` = N^2 * 10 / (forward + adjoint time) in G body-pair interactions/s
(the paper's convention, section 4.1: N^2 pairs per force evaluation, self
pairs included, 20 flops per pair).  Inputs are resident in HBM before the
timed region; every step restores the initial state with device copies.

Also reported on the same line: forward-only and forward + adjoint legs of
every precision (the near / far ones on the bodies in Morton order), the
checkpoint-interval sweep and the FP32-state forward; kernel-level rates at
N = 65536 and 262144 (whole system and one eighth of the target rows); the
roofline position of the dominant kernel and of the forward (timed with HIP
events on the stream they run on); the stated errors against the FP64
oracle; and the oracle itself timed on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("G body-pair interactions/s (FP64 vs mixed, fwd and fwd+adjoint) "
          "at stated error")
WORKLOAD = "cube16384"
CKPT_EVERY = 5
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32, published
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64, published
# Flops per body pair, counting add/sub/mul as 1, FMA as 2 and the reciprocal
# square root as 2: the force pair (3 sub, 3 FMA, rsqrt, 3 mul, 3 FMA) is the
# paper's 20; the VJP pair (3 sub, 3 FMA, rsqrt, 2 mul, 3 mul + 3 FMA for h,
# 1 mul + 2 FMA twice for e.h and gbar.e, 1 FMA, 2 mul, 6 FMA) is 48.
# The potential pair (diagnostics) is 3 sub, 3 FMA, rsqrt, 1 FMA = 13.
FLOPS_PER_PAIR = {"accel": 20, "vjp": 48, "diag": 13}
# HBM bytes per launch of the roofline kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, each scaled by what the counter reads for a
# 64 MiB device copy; profiles/vjp_kernel_cube16384_mixed_traffic.md).  They
# describe the kernel source they were taken on (first 16 hex digits of its
# SHA-256) and are reported as null for any other source.
MEASURED_TRAFFIC = {("vjp", "mixed"): {"bytes": 24.2e6, "src_sha256": "26b351e90e1d50b8"}}
# the sources that define the all-pairs VJP / forward kernels of the roofline
KERNEL_SRC = [os.path.join(ROOT, "paper_2203_08263_amd", "csrc", f)
              for f in ("nbody_kernels.hip", "nbody_device.h")]
DTYPE = {"fp64": "f64", "mixed": "f32-pair/f64-acc",
         "mixed_d64": "f32-pair(f64-diff)/f64-acc",
         "mixed_nf": "f32-pair(near f64-diff, far recentred)/f64-acc",
         "mixed_nf64": "near f64-pair, far f32-pair(recentred)/f64-acc"}
PRECS = ("fp64", "mixed", "mixed_d64", "mixed_nf", "mixed_nf64")
SORTED = ("mixed_nf", "mixed_nf64")   # run on the bodies in Morton order


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


class Bench:
    def __init__(self, torch, B, inputs, w):
        self.torch, self.B, self.w = torch, B, w
        dev = torch.device("cuda:0")
        self.dev = dev
        T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
        pos, vel, mass = w.initial_state()
        self.np_state = (pos, vel, mass)
        self.gx_T = inputs.upstream_normal(w.n, w.seed + 500)
        self.P0, self.V0, self.M = T(pos), T(vel), T(mass)
        self.GX0 = T(self.gx_T)
        n = w.n
        self.P, self.V = torch.empty_like(self.P0), torch.empty_like(self.V0)
        self.A = torch.empty_like(self.P0)
        self.GX, self.GV = torch.empty_like(self.P0), torch.empty_like(self.P0)
        self.GM = torch.empty_like(self.M)
        self.CK = torch.empty(B.nbody_checkpoint_bytes(n, w.steps, CKPT_EVERY) // 8,
                              dtype=torch.float64, device=dev)
        # the near / far mode runs on the same bodies in Morton order (sorted
        # once here on the GPU; perm maps its results back)
        self.perm, self.P0s, self.V0s, self.Ms = B.nbody_morton_sort(self.P0, self.M,
                                                                     self.V0)
        self.GX0s = self.GX0[:, self.perm].contiguous()
        # the paper's single-precision variant: FP32 copies of the state
        self.P0f, self.V0f, self.Mf = (t.float() for t in (self.P0, self.V0, self.M))
        self.Pf, self.Vf = torch.empty_like(self.P0f), torch.empty_like(self.V0f)
        self.Af0 = B.nbody_accel_f32(self.P0f, self.Mf, w.G, w.eps)
        self.Af = torch.empty_like(self.Af0)
        self.wsf = torch.empty(max(B.nbody_f32_workspace_bytes(B.NBODY_OP_STEP, n), 256),
                               dtype=torch.uint8, device=dev)
        self.A0 = {}
        self.ws = {}
        for p in PRECS:
            P0, M = self.state0(p)[0], self.state0(p)[2]
            self.A0[p] = B.nbody_accel(P0, M, w.G, w.eps, p)
            nb = max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, w.steps, CKPT_EVERY, p),
                     B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, w.steps,
                                             CKPT_EVERY, p), 256)
            self.ws[p] = torch.empty(nb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()

    def state0(self, p):
        """(x_0, v_0, m, dL/dx_S) in the body order precision p runs in."""
        if p in SORTED:
            return self.P0s, self.V0s, self.Ms, self.GX0s
        return self.P0, self.V0, self.M, self.GX0

    def forward(self, p):
        w, B = self.w, self.B
        P0, V0, M, _ = self.state0(p)
        self.P.copy_(P0)
        self.V.copy_(V0)
        self.A.copy_(self.A0[p])
        B.nbody_step(self.P, self.V, self.A, M, w.G, w.eps, w.dt, w.steps, p,
                     acc_valid=True, ckpt=self.CK, ckpt_every=CKPT_EVERY,
                     workspace=self.ws[p])

    def forward_f32(self):
        w, B = self.w, self.B
        self.Pf.copy_(self.P0f)
        self.Vf.copy_(self.V0f)
        self.Af.copy_(self.Af0)
        B.nbody_step_f32(self.Pf, self.Vf, self.Af, self.Mf, w.G, w.eps, w.dt, w.steps,
                         acc_valid=True, workspace=self.wsf)

    def fwd_adj_every(self, p, K, ck, ws):
        """Forward with a checkpoint every K steps, then the adjoint."""
        w, B = self.w, self.B
        P0, V0, M, GX0 = self.state0(p)
        self.P.copy_(P0)
        self.V.copy_(V0)
        self.A.copy_(self.A0[p])
        B.nbody_step(self.P, self.V, self.A, M, w.G, w.eps, w.dt, w.steps, p,
                     acc_valid=True, ckpt=ck, ckpt_every=K, workspace=ws)
        self.GX.copy_(GX0)
        self.GV.zero_()
        B.nbody_step_adjoint(ck, M, self.GX, self.GV, w.G, w.eps, w.dt, w.steps, K,
                             p, gmass=self.GM, workspace=ws)

    def adjoint(self, p):
        w, B = self.w, self.B
        _, _, M, GX0 = self.state0(p)
        self.GX.copy_(GX0)
        self.GV.zero_()
        B.nbody_step_adjoint(self.CK, M, self.GX, self.GV, w.G, w.eps, w.dt,
                             w.steps, CKPT_EVERY, p, gmass=self.GM,
                             workspace=self.ws[p])

    def step(self, p):
        self.forward(p)
        self.adjoint(p)

    def timed(self, fn, reps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / reps, 1e3 * wall / reps


def kernel_src_hash():
    """sha256 prefix of the kernel sources (concatenated in KERNEL_SRC order)."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def roofline(bench, p, kind):
    """Average launch duration (HIP events on the launch stream) of the
    all-pairs kernel of `kind` at the workload's size, and its position
    against the vector peak of its arithmetic type."""
    torch, B, w = bench.torch, bench.B, bench.w
    n = w.n
    P0, _, M, GX0 = bench.state0(p)
    if kind == "accel":
        fn = lambda: B.nbody_accel(P0, M, w.G, w.eps, p, out=bench.A)  # noqa
    else:
        fn = lambda: B.nbody_accel_vjp(P0, M, GX0, w.G, w.eps, p,  # noqa
                                       gpos=bench.GX, gmass=bench.GM)
    warm(bench.torch, fn)
    ms, _ = bench.timed(fn, reps=50, warmup=3)
    flops = FLOPS_PER_PAIR[kind] * n * n
    traffic = None
    rec = MEASURED_TRAFFIC.get((kind, p))
    if rec is not None:
        if kernel_src_hash() == rec["src_sha256"]:
            traffic = rec["bytes"]
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
    return {"kernel": "%s (%s), N=%d" % ({"accel": "accel_kernel", "vjp": "vjp_kernel"}[kind],
                                         p, n),
            "bound": "alu", "achieved": round(achieved, 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "avg_launch_ms": round(ms, 4),
            "flops_per_pair": FLOPS_PER_PAIR[kind]}


def shape_legs(torch, B, inputs):
    """Kernel-level throughput at the two large target shapes: the forward
    and the energy diagnostics at N = 65536 (Plummer, a = 1, eps = 1e-2) and
    the forward and VJP at N = 262144 (clustered Plummer, a = 0.1,
    eps = 1e-3), each timed with HIP events over back-to-back calls (kernel +
    split reduce).  At N = 262144 also one device's share when the target rows
    are split eight ways (rows 3/8 .. 4/8 against all sources, the row-range
    entry points), the per-device kernel shape of that partition."""
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    out = {}
    for name, precs, kinds in (("plummer65536", ("mixed", "mixed_d64", "fp64", "mixed_nf",
                                                 "mixed_nf64"),
                                ("accel", "diag")),
                               ("plummer262144_vjp", ("mixed", "mixed_d64", "fp64",
                                                      "mixed_nf", "mixed_nf64"),
                                ("accel", "vjp", "accel_share8", "vjp_share8"))):
        w = inputs.WORKLOADS[name]
        pos, vel, mass = w.initial_state()
        P0, M0, V0 = T(pos), T(mass), T(vel)
        D = torch.empty(9, dtype=torch.float64, device=dev)
        G0 = T(inputs.upstream_normal(w.n, w.seed + 400))
        # Morton order for the near / far mode; the sort itself is timed too
        sort_fn = lambda: B.nbody_morton_sort(P0, M0, V0)  # noqa
        warm(torch, sort_fn)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(5):
            perm, Ps, Vs, Ms = sort_fn()
        s1.record()
        torch.cuda.synchronize()
        sort_ms = s0.elapsed_time(s1) / 5
        Gs = G0[:, perm].contiguous()
        A, GX, GM = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(M0)
        share = w.n // 8
        r0 = 3 * share
        As = torch.empty((3, share), dtype=torch.float64, device=dev)
        GXs = torch.empty((3, share), dtype=torch.float64, device=dev)
        GMs = torch.empty(share, dtype=torch.float64, device=dev)
        res = {"morton_sort_ms": round(sort_ms, 4)}
        # FP32 state (the paper's single-precision variant): forward only
        Pf, Mf = P0.float(), M0.float()
        Af = torch.empty_like(Pf)
        wsf = torch.empty(max(B.nbody_f32_workspace_bytes(B.NBODY_OP_ACCEL, w.n), 256),
                          dtype=torch.uint8, device=dev)
        fnf = lambda: B.nbody_accel_f32(Pf, Mf, w.G, w.eps, out=Af, workspace=wsf)  # noqa
        warm(torch, fnf)
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20 if w.n <= 65536 else 4
        f0.record()
        for _ in range(reps):
            fnf()
        f1.record()
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / reps
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
                                 B.nbody_workspace_bytes(B.NBODY_OP_VJP, w.n, 0, 1, p),
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
                elif kind == "diag":
                    fn = lambda: B.nbody_diagnostics(P, Vt, M, w.G, w.eps, p, out=D,  # noqa
                                                     workspace=ws)
                else:
                    fn = lambda: B.nbody_accel_vjp(P, M, Gt, w.G, w.eps, p, gpos=GX,  # noqa
                                                   gmass=GM, workspace=ws)
                rows = share if kind.endswith("_share8") else w.n
                reps = 20 if w.n <= 65536 else (16 if rows < w.n else 4)
                warm(torch, fn)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                ips = float(rows) * w.n / (ms * 1e-3)
                peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
                fl = FLOPS_PER_PAIR[kind.replace("_share8", "")]
                res["%s_%s" % (kind, p)] = {
                    "ms": round(ms, 4), "G_int_s": round(ips / 1e9, 1),
                    "TFLOP_s": round(ips * fl / 1e12, 2),
                    "frac_of_vector_peak": round(ips * fl / 1e12 / peak, 4)}
        if "vjp_mixed" in res:
            for p in precs:
                if "vjp_%s" % p not in res:
                    continue
                res["vjp_over_fwd_%s" % p] = round(res["vjp_%s" % p]["ms"] /
                                                   res["accel_%s" % p]["ms"], 3)
        out[name] = res
    return out


def adjoint_leg(torch, B, inputs):
    """The forward + adjoint configuration: N = 8192 uniform cube, 50 KDK
    steps with a checkpoint every 10, then the reverse sweep (which
    recomputes each segment).  Step-level t_bwd / t_fwd per precision."""
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS["cube8192_adjoint"]
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa
    pos, vel, mass = w.initial_state()
    P0, V0, M = T(pos), T(vel), T(mass)
    GX0 = T(inputs.upstream_normal(w.n, w.seed + 500))
    P, V, A = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(P0)
    GX, GV, GM = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(M)
    K = w.ckpt_every
    CK = torch.empty(B.nbody_checkpoint_bytes(w.n, w.steps, K) // 8, dtype=torch.float64,
                     device=dev)
    out = {"workload": "cube8192_adjoint: N=%d, %d KDK steps, checkpoint every %d"
                       % (w.n, w.steps, K)}
    for p in ("mixed", "fp64"):
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
        times = []
        for fn in (fwd, bwd):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fwd()   # the adjoint reads this forward's checkpoints
            torch.cuda.synchronize()
            e0.record()
            for _ in range(3):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 3)
        tf, tb = times
        out[p] = {"fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                  "bwd_over_fwd": round(tb / tf, 3),
                  "fwd_adj_G_int_s": round(float(w.n) * w.n * w.steps / ((tf + tb) * 1e-3) / 1e9, 1)}
    return out


def small_rollout_leg(torch, B, inputs):
    """The launch-bound configuration: N = 1024, 100 FP64 KDK steps (one
    launch per step at this size).  Timed eagerly and as a replayed HIP graph
    of the same nbody_step call (state restored by device copies before each
    run)."""
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

    def timed(fn, reps=20):
        warm(torch, fn)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    eager = timed(run)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    graph = timed(g.replay)
    pairs = float(w.n) * w.n * w.steps
    return {"workload": "%s: N=%d, %d FP64 KDK steps" % (w.name, w.n, w.steps),
            "eager_ms": round(eager, 4), "graph_ms": round(graph, 4),
            "eager_G_int_s": round(pairs / (eager * 1e-3) / 1e9, 1),
            "graph_G_int_s": round(pairs / (graph * 1e-3) / 1e9, 1)}


def cpu_baseline(bench, p, gx_gpu, gv_gpu, gm_gpu, x_end, v_end, finals=None):
    """The FP64 oracle on the host cores over the same workload (forward plus
    exact reverse sweep), and the stated errors of the GPU results."""
    import numpy as np

    import oracle
    from paper_2203_08263_amd import metrics

    w = bench.w
    pos, vel, mass = bench.np_state
    n = w.n
    # the whole workload, repeated until about 10 s of CPU work; median rate
    times = []
    t_all = time.perf_counter()
    while not times or (time.perf_counter() - t_all < 10.0 and len(times) < 9):
        t0 = time.perf_counter()
        rx, rv, rm = oracle.step_adjoint(pos, vel, mass, w.G, w.eps, w.dt, w.steps,
                                         bench.gx_T, np.zeros((3, n)))
        times.append(time.perf_counter() - t0)
    t_cpu = float(np.median(times))
    base = {"value": round(n * n * w.steps / t_cpu / 1e9, 4),
            "unit": "G interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "the whole workload: N=%d, %d KDK steps forward + exact "
                      "reverse sweep (FP64, all positions stored), median of %d "
                      "runs of %.2f s" % (n, w.steps, len(times), t_cpu)}
    # stated errors: gradients of this run vs the oracle's; accelerations at
    # x_0 on 2048 seeded rows for every precision
    err = {"grad_vs_oracle_normwise_%s" % p: {
        "dL/dx0": metrics.normwise(gx_gpu, rx), "dL/dv0": metrics.normwise(gv_gpu, rv),
        "dL/dm": metrics.normwise(gm_gpu, rm)}}
    # energy drift of this run's forward rollout (FP64 oracle energy)
    e0 = sum(oracle.energy(pos, vel, mass, w.G, w.eps))
    e1 = sum(oracle.energy(x_end, v_end, mass, w.G, w.eps))
    err["energy_drift_%s_%dsteps" % (p, w.steps)] = float("%.3e" % (abs(e1 - e0) / abs(e0)))
    # and of every precision's rollout (final states of the legs; bodies in
    # Morton order for the near / far modes: the energy is order-independent)
    for q, (xq, vq, mq) in (finals or {}).items():
        eq = sum(oracle.energy(xq, vq, mq, w.G, w.eps))
        err["energy_drift_%s_%dsteps" % (q, w.steps)] = float("%.3e" % (abs(eq - e0) / abs(e0)))
    rows = w.rows(2048)
    ref = oracle.accel_rows(pos, mass, w.G, w.eps, rows)
    for q in PRECS:
        a = bench.A0[q].cpu().numpy()
        if q in SORTED:                  # back from Morton order
            back = np.empty_like(a)
            back[:, bench.perm.cpu().numpy()] = a
            a = back
        a = a[:, rows]
        err["accel_x0_2048rows_%s" % q] = {k: float("%.3e" % v) for k, v in
                                          metrics.rel_errors(a, ref).items()}
    return base, err


def cpu_by_workload(inputs):
    """The FP64 oracle's rate on a bounded sample of each other workload
    (about 3 s in all), for the per-workload GPU legs beside it."""
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
    w = inputs.WORKLOADS["plummer262144_vjp"]
    pos, _, mass = w.initial_state()
    rows = w.rows(1024)
    g = inputs.upstream_normal(w.n, w.seed + 400)

    def both():
        oracle.accel_rows(pos, mass, w.G, w.eps, rows)
        oracle.accel_vjp_rows(pos, mass, g, w.G, w.eps, rows)
    out["plummer262144_vjp"] = dict(zip(("G_int_s", "s"), rate(
        2.0 * len(rows) * w.n, both)),
        sample="force and VJP rows of the 1024 seeded bodies")
    _ = np
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", default="mixed", choices=PRECS)
    ap.add_argument("--no-legs", action="store_true",
                    help="time only the main precision's forward + adjoint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the kernel legs at N = 65536 and 262144")
    ap.add_argument("--profile", choices=["accel", "vjp"], default=None,
                    help="counter-collection mode: a 64 MiB device copy (the "
                         "traffic calibration) then --steps launches of one "
                         "all-pairs kernel at the workload size; no JSON line")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2203_08263_amd import binding as B
    from paper_2203_08263_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    B.load_library()
    w = inputs.WORKLOADS[WORKLOAD]
    bench = Bench(torch, B, inputs, w)
    p = args.precision
    n2s = float(w.n) * w.n * w.steps

    if args.profile:
        src = torch.ones(8 << 20, dtype=torch.float64, device=bench.dev)
        dst = torch.empty_like(src)
        dst.copy_(src)                       # calibration: 64 MiB read + write
        torch.cuda.synchronize()
        P0, _, M, GX0 = bench.state0(p)
        for _ in range(args.steps):
            if args.profile == "accel":
                B.nbody_accel(P0, M, w.G, w.eps, p, out=bench.A)
            else:
                B.nbody_accel_vjp(P0, M, GX0, w.G, w.eps, p, gpos=bench.GX,
                                  gmass=bench.GM)
        torch.cuda.synchronize()
        log("bench: profile mode done (%s, %s, %d launches)" % (args.profile, p,
                                                                 args.steps))
        return 0

    # main timed region: K whole steps of the hot path
    log("bench: %s, precision %s, %d warmup + %d timed steps" % (w.name, p,
                                                                args.warmup, args.steps))
    torch.cuda.synchronize()   # one process, one GPU: no barrier to take
    ms, wall_ms = bench.timed(lambda: bench.step(p), args.steps, args.warmup)
    value = n2s / (ms * 1e-3) / 1e9
    log("bench: %.3f ms/step (events), %.3f ms/step (wall), %.1f G int/s"
        % (ms, wall_ms, value))
    gx, gv, gm = (bench.GX.cpu().numpy(), bench.GV.cpu().numpy(),
                  bench.GM.cpu().numpy())
    x_end, v_end = bench.P.cpu().numpy(), bench.V.cpu().numpy()

    legs = {}
    finals = {}
    if not args.no_legs:
        for q in PRECS:
            warm(torch, lambda: bench.forward(q))
            fms, _ = bench.timed(lambda: bench.forward(q), 10, 2)
            sms, _ = bench.timed(lambda: bench.step(q), 5, 1)
            legs[q] = {"fwd_G_int_s": round(n2s / (fms * 1e-3) / 1e9, 1),
                       "fwd_ms": round(fms, 4),
                       "fwd_adj_G_int_s": round(n2s / (sms * 1e-3) / 1e9, 1),
                       "fwd_adj_ms": round(sms, 4),
                       "bwd_over_fwd": round((sms - fms) / fms, 3)}
            # the forward of the last timed step left this precision's final state
            finals[q] = (bench.P.cpu().numpy(), bench.V.cpu().numpy(),
                         bench.state0(q)[2].cpu().numpy())
            log("bench: leg %s %s" % (q, legs[q]))
        # checkpoint interval: K = 1 stores every state (no recomputation),
        # K = steps keeps one record and recomputes the whole rollout
        sweep = {}
        for K in (1, CKPT_EVERY, w.steps):
            ck = torch.empty(B.nbody_checkpoint_bytes(w.n, w.steps, K) // 8,
                             dtype=torch.float64, device=bench.dev)
            wsk = torch.empty(max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, w.n, w.steps, K, p),
                                  B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, w.n,
                                                          w.steps, K, p)),
                              dtype=torch.uint8, device=bench.dev)
            fn = lambda: bench.fwd_adj_every(p, K, ck, wsk)  # noqa
            warm(torch, fn)
            kms, _ = bench.timed(fn, 5, 1)
            sweep["K%d" % K] = {"fwd_adj_G_int_s": round(n2s / (kms * 1e-3) / 1e9, 1),
                                "fwd_adj_ms": round(kms, 4),
                                "checkpoint_MB": round(ck.numel() * 8 / 1e6, 2)}
        legs["%s_ckpt_every" % p] = sweep
        log("bench: checkpoint sweep %s" % sweep)
        # FP32 state (forward only: this variant has no adjoint)
        warm(torch, bench.forward_f32)
        fms, _ = bench.timed(bench.forward_f32, 10, 2)
        legs["f32_state"] = {"fwd_G_int_s": round(n2s / (fms * 1e-3) / 1e9, 1),
                             "fwd_ms": round(fms, 4)}
        log("bench: leg f32_state %s" % legs["f32_state"])

    # roofline of the dominant kernel of the step (the VJP: 11 launches of
    # ~2x the cost of each of the 18 force evaluations), plus the forward's
    roof = roofline(bench, p, "vjp")
    roof_fwd = roofline(bench, p, "accel")
    log("bench: roofline vjp %s" % roof)
    log("bench: roofline accel %s" % roof_fwd)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "G interactions/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[p],
           "data": "synthetic",
           "config": {"workload": "%s: N=%d uniform cube, %d KDK steps forward + "
                                  "checkpointed adjoint (every %d), eps=%g, dt=%g, "
                                  "G=%g, precision %s"
                                  % (w.name, w.n, w.steps, CKPT_EVERY, w.eps, w.dt,
                                     w.G, p),
                      "n": w.n, "sim_steps": w.steps, "ckpt_every": CKPT_EVERY,
                      "precision": p, "parallelism": "single GPU"},
           "roofline": roof, "roofline_forward": roof_fwd, "legs": legs,
           "vjp_over_fwd_kernel": round(roof["avg_launch_ms"] / roof_fwd["avg_launch_ms"], 3)}
    if not args.no_shapes:
        log("bench: kernel legs at N = 65536 and 262144")
        out["shapes"] = shape_legs(torch, B, inputs)
        out["shapes"]["cube1024_fp64_rollout"] = small_rollout_leg(torch, B, inputs)
        out["shapes"]["cube8192_adjoint"] = adjoint_leg(torch, B, inputs)
        log("bench: shapes %s" % out["shapes"])
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (FP64 oracle on the host cores)")
        base, err = cpu_baseline(bench, p, gx, gv, gm, x_end, v_end, finals)
        out["cpu_baseline"] = base
        out["error"] = err
        if not args.no_shapes:
            out["cpu_oracle_by_workload"] = cpu_by_workload(inputs)
            log("bench: oracle by workload %s" % out["cpu_oracle_by_workload"])
    else:
        out["cpu_baseline"] = None
    _ = np
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
