"""GPU parity of the row-range entry points (nbody_accel_rows,
nbody_accel_vjp_rows): the force sum and its VJP for a contiguous range of
target bodies against all n sources, i.e. one device's share when target
rows are divided among devices.

* All n rows reproduce the whole-system calls bitwise (same launch plan).
* Any range agrees with the oracle's rows within the derived bounds, and
  the shares of a partition put together agree with the oracle everywhere.
* The real share shape: N = 262144 Plummer (a = 0.1, eps = 1e-3), rows of one
  eighth, sampled rows against the oracle.
"""
import sys

import numpy as np
import pytest

import _tol
from paper_2203_08263_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["fp64", "mixed", "mixed_d64", "mixed_nf", "mixed_nf64", "mixed_ds"]


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


@pytest.fixture(scope="module")
def dev(B):
    return torch.device("cuda:0")


def T(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _check_bound(got, ref, bound, what):
    err = np.sqrt(((got - ref) ** 2).sum(axis=0))
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    assert np.all(err <= bound), "%s: row %d err %.3e bound %.3e" % (
        what, worst, err[worst], bound[worst])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 257, 3001])
def test_all_rows_bitwise_equal_whole_system(B, dev, prec, n):
    say("rows = all", prec, n)
    pos, _, mass = inputs.uniform_cube(n, 900 + n)
    g = inputs.upstream_normal(n, 950 + n)
    P, M, Gt = T(pos, dev), T(mass, dev), T(g, dev)
    a_full = N(B.nbody_accel(P, M, 1.0, 1e-3, prec))
    a_rows = N(B.nbody_accel_rows(P, M, 0, n, 1.0, 1e-3, prec))
    assert np.array_equal(a_full, a_rows)
    gx, gm = B.nbody_accel_vjp(P, M, Gt, 1.0, 1e-3, prec)
    rx, rm = B.nbody_accel_vjp_rows(P, M, Gt, 0, n, 1.0, 1e-3, prec)
    assert np.array_equal(N(gx), N(rx))
    assert np.array_equal(N(gm), N(rm))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("r0,rc", [(0, 1), (1000, 1), (17, 700), (2300, 701),
                                   (255, 257), (3000, 1)])
def test_row_range_vs_oracle(B, dev, oracle, prec, r0, rc):
    n = 3001
    say("rows", prec, r0, rc)
    pos, _, mass = inputs.uniform_cube(n, 911)
    g = inputs.upstream_normal(n, 912)
    rows = np.arange(r0, r0 + rc)
    P, M, Gt = T(pos, dev), T(mass, dev), T(g, dev)
    a = N(B.nbody_accel_rows(P, M, r0, rc, 1.0, 1e-3, prec))
    assert a.shape == (3, rc)
    ra = oracle.accel_rows(pos, mass, 1.0, 1e-3, rows)
    _check_bound(a, ra, _tol.accel_bound(pos, mass, 1.0, 1e-3, prec, rows), "accel")
    gx, gm = B.nbody_accel_vjp_rows(P, M, Gt, r0, rc, 1.0, 1e-3, prec)
    gx, gm = N(gx), N(gm)
    assert gx.shape == (3, rc) and gm.shape == (rc,)
    rx, rm = oracle.accel_vjp_rows(pos, mass, g, 1.0, 1e-3, rows)
    bx, bm = _tol.vjp_bound(pos, mass, g, 1.0, 1e-3, prec, rows)
    _check_bound(gx, rx, bx, "dL/dx")
    assert np.all(np.abs(gm - rm) <= bm), "dL/dm"


@pytest.mark.parametrize("prec", PRECS)
def test_partition_reassembles(B, dev, oracle, prec):
    # three uneven shares (one of them empty) cover all rows once
    n = 2000
    say("partition", prec)
    pos, _, mass = inputs.uniform_cube(n, 913)
    g = inputs.upstream_normal(n, 914)
    P, M, Gt = T(pos, dev), T(mass, dev), T(g, dev)
    cuts = [0, 613, 613, 1390, n]
    acc, gxs, gms = [], [], []
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        acc.append(N(B.nbody_accel_rows(P, M, r0, r1 - r0, 1.0, 1e-3, prec)))
        gx, gm = B.nbody_accel_vjp_rows(P, M, Gt, r0, r1 - r0, 1.0, 1e-3, prec)
        gxs.append(N(gx))
        gms.append(N(gm))
    assert acc[1].shape == (3, 0) and gms[1].shape == (0,)
    a = np.concatenate(acc, axis=1)
    gx, gm = np.concatenate(gxs, axis=1), np.concatenate(gms)
    _check_bound(a, oracle.accel(pos, mass, 1.0, 1e-3),
                 _tol.accel_bound(pos, mass, 1.0, 1e-3, prec), "accel")
    rx, rm = oracle.accel_vjp(pos, mass, g, 1.0, 1e-3)
    bx, bm = _tol.vjp_bound(pos, mass, g, 1.0, 1e-3, prec)
    _check_bound(gx, rx, bx, "dL/dx")
    assert np.all(np.abs(gm - rm) <= bm), "dL/dm"


def test_rows_into_caller_output(B, dev, oracle):
    n = 1000
    pos, _, mass = inputs.uniform_cube(n, 915)
    P, M = T(pos, dev), T(mass, dev)
    out = torch.full((3, 10), 7.0, dtype=torch.float64, device=dev)
    ret = B.nbody_accel_rows(P, M, 500, 10, 1.0, 1e-3, "mixed", out=out)
    assert ret.data_ptr() == out.data_ptr()
    rows = np.arange(500, 510)
    _check_bound(N(out), oracle.accel_rows(pos, mass, 1.0, 1e-3, rows),
                 _tol.accel_bound(pos, mass, 1.0, 1e-3, "mixed", rows), "accel")


@pytest.mark.parametrize("prec", PRECS)
def test_share_of_plummer262144(B, dev, oracle, prec):
    # one of eight shares of the N = 262144 Plummer system at its real shape:
    # 32768 target rows against all 262144 sources
    w = inputs.WORKLOADS["plummer262144_vjp"]
    say("share 3/8 of", w.name, prec)
    pos, _, mass = w.initial_state()
    g = inputs.upstream_normal(w.n, w.seed + 400)
    share = w.n // 8
    r0 = 3 * share
    P, M, Gt = T(pos, dev), T(mass, dev), T(g, dev)
    a = N(B.nbody_accel_rows(P, M, r0, share, w.G, w.eps, prec))
    gx, gm = B.nbody_accel_vjp_rows(P, M, Gt, r0, share, w.G, w.eps, prec)
    gx, gm = N(gx), N(gm)
    assert np.isfinite(a).all() and np.isfinite(gx).all() and np.isfinite(gm).all()
    local = inputs.subset_rows(share, 128, w.seed + 500)
    rows = r0 + local
    ra = oracle.accel_rows(pos, mass, w.G, w.eps, rows)
    _check_bound(a[:, local], ra,
                 _tol.accel_bound(pos, mass, w.G, w.eps, prec, rows), "accel")
    rx, rm = oracle.accel_vjp_rows(pos, mass, g, w.G, w.eps, rows)
    bx, bm = _tol.vjp_bound(pos, mass, g, w.G, w.eps, prec, rows)
    _check_bound(gx[:, local], rx, bx, "dL/dx")
    assert np.all(np.abs(gm[local] - rm) <= bm), "dL/dm"
