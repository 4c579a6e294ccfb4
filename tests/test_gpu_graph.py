"""The C-ABI calls are capturable into a HIP graph (torch.cuda.graph).

The library allocates nothing, issues no memsets and never synchronises, so
a caller can capture a whole rollout and its adjoint once and replay it --
the way to remove per-launch overhead from small, launch-bound systems.
Each replay is checked bitwise against the eager result, with unrelated
eager work and synchronisations between the replays.  Calls on concurrent
streams are independent: two rollouts with their adjoints run side by side
reproduce their serial results bitwise.
"""
import sys

import numpy as np
import pytest

from paper_2203_08263_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_08263_amd import binding
    binding.load_library()
    return binding


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_nf"])
def test_graph_replay_rollout_and_adjoint(B, oracle, prec):
    say("graph replay", prec)
    dev = torch.device("cuda:0")
    # FP64 at N = 1024 steps in one launch per step; the near / far mode
    # needs more than 1024 bodies to split (below it is all near)
    n, S, K = (1536 if prec == "mixed_nf" else 1024), 20, 5
    pos, vel, mass = inputs.uniform_cube(n, 1001)
    if prec == "mixed_nf":   # spatial order, so the far form is exercised too
        o = oracle.morton_order(pos)
        pos, vel, mass = pos[:, o].copy(), vel[:, o].copy(), mass[o].copy()
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    P0, V0, M = T(pos), T(vel), T(mass)
    GX0 = T(inputs.upstream_normal(n, 77))
    A0 = B.nbody_accel(P0, M, 1.0, 1e-3, prec)
    P, V, A = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(P0)
    GX, GV, GM = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(M)
    CK = torch.empty(B.nbody_checkpoint_bytes(n, S, K) // 8, dtype=torch.float64,
                     device=dev)
    nb = max(B.nbody_workspace_bytes(B.NBODY_OP_STEP, n, S, K, prec),
             B.nbody_workspace_bytes(B.NBODY_OP_STEP_ADJOINT, n, S, K, prec))
    WS = torch.empty(nb, dtype=torch.uint8, device=dev)

    def work():
        B.nbody_step(P, V, A, M, 1.0, 1e-3, 1e-3, S, prec, acc_valid=True, ckpt=CK,
                     ckpt_every=K, workspace=WS)
        B.nbody_step_adjoint(CK, M, GX, GV, 1.0, 1e-3, 1e-3, S, K, prec, gmass=GM,
                             workspace=WS)

    def reset():
        P.copy_(P0)
        V.copy_(V0)
        A.copy_(A0)
        GX.copy_(GX0)
        GV.zero_()

    reset()
    work()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (P, V, A, GX, GV, GM)]

    reset()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        work()   # warm-up on the side stream before capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    torch.cuda.synchronize()
    for rep in range(4):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (P, V, A, GX, GV, GM)
        for a, b in zip(got, eager):
            assert torch.equal(a, b), "replay %d differs" % rep
        # unrelated eager work between replays
        junk = B.nbody_accel(P0 * 1.5, M, 1.0, 1e-3, prec)
        torch.cuda.synchronize()
        assert np.isfinite(junk.cpu().numpy()).all()


def test_graph_replay_f32_rollout_and_morton_sort(B):
    say("graph replay f32 + sort")
    dev = torch.device("cuda:0")
    n, S = 2000, 15
    pos, vel, mass = inputs.uniform_cube(n, 1003)
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    P64, V64, M64 = T(pos), T(vel), T(mass)
    P0, V0, M = P64.float(), V64.float(), M64.float()
    P, V, A = torch.empty_like(P0), torch.empty_like(P0), torch.empty_like(P0)
    WS = torch.empty(B.nbody_f32_workspace_bytes(B.NBODY_OP_STEP, n), dtype=torch.uint8,
                     device=dev)
    SW = torch.empty(B.nbody_workspace_bytes(B.NBODY_OP_MORTON_SORT, n, 0, 1, 0),
                     dtype=torch.uint8, device=dev)
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    PS, VS, MS = torch.empty_like(P64), torch.empty_like(P64), torch.empty_like(M64)
    lib = B.load_library()

    def work():
        B.nbody_step_f32(P, V, A, M, 1.0, 1e-3, 1e-3, S, workspace=WS)
        rc = lib.nbody_morton_sort(n, B._ptr(P64), B._ptr(V64), B._ptr(M64),
                                   B._ptr(perm), B._ptr(PS), B._ptr(VS), B._ptr(MS),
                                   B._ptr(SW), SW.numel(), B._stream(dev))
        assert rc == 0

    def reset():
        P.copy_(P0)
        V.copy_(V0)
        for t in (A, PS, VS, MS):
            t.zero_()
        perm.zero_()

    reset()
    work()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (P, V, A, perm, PS, VS, MS)]
    reset()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        work()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    torch.cuda.synchronize()
    for rep in range(4):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((P, V, A, perm, PS, VS, MS), eager):
            assert torch.equal(a, b), "replay %d differs" % rep


def test_concurrent_streams_bitwise(B):
    # The library keeps no device state between calls: two rollouts with their
    # adjoints, each on its own (default-priority) stream with its own buffers
    # and workspace, run concurrently and reproduce the serial results bitwise.
    say("two concurrent streams")
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    jobs = []
    for seed, n, prec in ((2001, 3001, "mixed"), (2002, 2048, "fp64")):
        pos, vel, mass = inputs.uniform_cube(n, seed)
        jobs.append(dict(n=n, prec=prec, P0=T(pos), V0=T(vel), M=T(mass),
                         GX0=T(inputs.upstream_normal(n, seed + 1))))
    S, K = 8, 3

    def run(j):
        P, V = j["P0"].clone(), j["V0"].clone()
        A = torch.empty_like(P)
        CK = torch.empty(B.nbody_checkpoint_bytes(j["n"], S, K) // 8,
                         dtype=torch.float64, device=dev)
        B.nbody_step(P, V, A, j["M"], 1.0, 1e-3, 1e-3, S, j["prec"], ckpt=CK,
                     ckpt_every=K)
        GX, GV = j["GX0"].clone(), torch.zeros_like(P)
        gx, gv, gm = B.nbody_step_adjoint(CK, j["M"], GX, GV, 1.0, 1e-3, 1e-3, S,
                                          K, j["prec"])
        return P, V, A, gx, gv, gm

    serial = []
    for j in jobs:
        serial.append(run(j))
        torch.cuda.synchronize()
    for rep in range(3):
        streams = [torch.cuda.Stream() for _ in jobs]
        outs = [None] * len(jobs)
        for k, (j, s) in enumerate(zip(jobs, streams)):
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                outs[k] = run(j)
        for s in streams:
            torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for got, want in zip(outs, serial):
            for a, b in zip(got, want):
                assert torch.equal(a, b), "concurrent run %d differs" % rep
