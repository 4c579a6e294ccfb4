"""nbody_accel_noalloc -- the force evaluation for callers that cannot
allocate device memory, with its split partials and box scratch in the
library's static device array -- against nbody_accel with a workspace.

Both run the same kernels and launch plan, so the results must be bitwise
equal.  Each precision makes two calls in a row on the shared array, the
second on a smaller system, so the second call runs on what the first left
behind.  The oracle is not needed: nbody_accel is held to the oracle by the
parity tests.
"""
import sys

import numpy as np
import pytest

from paper_2203_08263_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (precision, first n, second n): every pair uses the scratch (more than one
# source split; the near / far modes also put their boxes there), the second
# system ragged and smaller than the first.
CASES = [("fp64", 40000, 9001), ("mixed", 70001, 20003), ("mixed_d64", 65536, 5001),
         ("mixed_nf", 131072, 3001), ("mixed_nf64", 90000, 12345),
         ("mixed_ds", 70001, 4099)]


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


def _system(B, n, seed, prec, dev):
    pos, _, mass = inputs.plummer(n, seed, a=0.1)
    P = torch.tensor(pos, dtype=torch.float64, device=dev)
    M = torch.tensor(mass, dtype=torch.float64, device=dev)
    if prec in ("mixed_nf", "mixed_nf64"):
        _, P, _, M = B.nbody_morton_sort(P, M)
    return P, M


@pytest.mark.parametrize("prec,n1,n2", CASES)
def test_noalloc_matches_workspace_call_twice(B, prec, n1, n2):
    dev = torch.device("cuda:0")
    assert B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n1, 0, 1, prec) > 0
    assert B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, n2, 0, 1, prec) > 0
    eps = 1e-3
    P1, M1 = _system(B, n1, 71, prec, dev)
    P2, M2 = _system(B, n2, 72, prec, dev)
    say("noalloc %s n=%d then n=%d" % (prec, n1, n2))
    a1 = B.nbody_accel_noalloc(P1, M1, 1.0, eps, prec)
    a2 = B.nbody_accel_noalloc(P2, M2, 0.7, eps, prec)
    r1 = B.nbody_accel(P1, M1, 1.0, eps, prec)
    r2 = B.nbody_accel(P2, M2, 0.7, eps, prec)
    torch.cuda.synchronize()
    assert torch.isfinite(a1).all() and torch.isfinite(a2).all()
    assert torch.equal(a1, r1), "first call differs from nbody_accel"
    assert torch.equal(a2, r2), "second (smaller) call differs from nbody_accel"
    # and once more at the first size, after the smaller call
    a3 = B.nbody_accel_noalloc(P1, M1, 1.0, eps, prec)
    torch.cuda.synchronize()
    assert torch.equal(a3, r1)


def test_noalloc_small_system_and_rejection(B):
    dev = torch.device("cuda:0")
    # a small system needs no scratch at all (one source split)
    P, M = _system(B, 300, 73, "mixed", dev)
    assert B.nbody_workspace_bytes(B.NBODY_OP_ACCEL, 300, 0, 1, "mixed") == 0
    assert torch.equal(B.nbody_accel_noalloc(P, M, 1.0, 1e-3, "mixed"),
                       B.nbody_accel(P, M, 1.0, 1e-3, "mixed"))
    # FP64 at 65536 bodies needs more than the static scratch: rejected
    # before anything is enqueued, the output left untouched
    P, M = _system(B, 65536, 74, "fp64", dev)
    out = torch.full_like(P, 7.0)
    with pytest.raises(B.NBodyError) as ei:
        B.nbody_accel_noalloc(P, M, 1.0, 1e-3, "fp64", out=out)
    assert ei.value.code == 2 and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
