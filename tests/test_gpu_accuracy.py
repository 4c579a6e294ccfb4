"""Accuracy-regression ceilings of every FP32-pair mode on the three
full-size force workloads.

The element-wise bounds of tests/_tol.py are worst-case and would let a
tenfold loss of accuracy through; these ceilings sit at about twice the
errors measured on MI355X (E_max = largest per-body relative error,
E_norm = Frobenius relative error, both against the FP64 oracle), so a
regression of the pair arithmetic, the chunk sums or the near / far
decision fails here.  Rows: all bodies of the N = 16384 cube; for the
Plummer spheres the seeded rows plus the 256 bodies nearest the centre of
mass (where the net acceleration nearly cancels and relative errors peak).
NBODY_MIXED, NBODY_MIXED_D64 and NBODY_MIXED_DS run on the bodies in their
generated order,
the near / far modes on the same bodies in Morton order (sorted by the
oracle).  The VJP is held the same way: normwise errors of dL/dx and dL/dm
on the same rows (upstream gradient N(0, 1)) at about twice the measured.
"""
import sys

import numpy as np
import pytest

from paper_2203_08263_amd import inputs, metrics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROWS = {"cube16384": None, "plummer65536": 4096, "plummer262144_vjp": 1024}
SORTED = ("mixed_nf", "mixed_nf64")

# (workload, precision): (E_max ceiling, E_norm ceiling)
CEILING = {
    ("cube16384", "mixed"): (7.0e-5, 1.3e-5),
    ("cube16384", "mixed_d64"): (3.5e-6, 1.3e-7),
    ("cube16384", "mixed_nf"): (9.0e-6, 1.3e-7),
    ("cube16384", "mixed_nf64"): (5.0e-7, 4.0e-8),
    ("plummer65536", "mixed"): (9.0e-6, 2.5e-7),
    ("plummer65536", "mixed_d64"): (1.0e-6, 5.5e-8),
    ("plummer65536", "mixed_nf"): (1.6e-6, 7.0e-8),
    ("plummer65536", "mixed_nf64"): (8.0e-7, 5.0e-8),
    ("plummer262144_vjp", "mixed"): (3.0e-6, 1.5e-7),
    ("plummer262144_vjp", "mixed_d64"): (7.0e-7, 5.5e-8),
    ("plummer262144_vjp", "mixed_nf"): (1.2e-6, 6.5e-8),
    ("plummer262144_vjp", "mixed_nf64"): (1.0e-6, 5.5e-8),
    ("cube16384", "mixed_ds"): (3.2e-6, 1.3e-7),
    ("plummer65536", "mixed_ds"): (1.5e-6, 6.0e-8),
    ("plummer262144_vjp", "mixed_ds"): (2.3e-6, 6.0e-8),
}


# (workload, precision): (dL/dx normwise ceiling, dL/dm normwise ceiling)
VJP_CEILING = {
    ("cube16384", "mixed"): (6.5e-5, 2.5e-5),
    ("cube16384", "mixed_d64"): (3.5e-7, 3.4e-7),
    ("cube16384", "mixed_ds"): (3.5e-7, 3.4e-7),
    ("cube16384", "mixed_nf"): (4.5e-7, 2.6e-7),
    ("cube16384", "mixed_nf64"): (2.0e-10, 8.0e-9),
    ("plummer65536", "mixed"): (5.0e-6, 2.4e-6),
    ("plummer65536", "mixed_d64"): (4.5e-7, 2.9e-7),
    ("plummer65536", "mixed_ds"): (4.5e-7, 3.0e-7),
    ("plummer65536", "mixed_nf"): (4.7e-7, 2.9e-7),
    ("plummer65536", "mixed_nf64"): (1.7e-8, 4.6e-8),
    ("plummer262144_vjp", "mixed"): (5.0e-6, 2.0e-6),
    ("plummer262144_vjp", "mixed_d64"): (4.4e-7, 3.1e-7),
    ("plummer262144_vjp", "mixed_ds"): (4.5e-7, 3.1e-7),
    ("plummer262144_vjp", "mixed_nf"): (5.1e-7, 3.0e-7),
    ("plummer262144_vjp", "mixed_nf64"): (4.5e-8, 7.0e-8),
}

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


_SYSTEMS = {}


def _system(oracle, name, ordered):
    """(pos, mass, gbar, rows, oracle accelerations and VJP on rows)."""
    key = (name, ordered)
    if key not in _SYSTEMS:
        w = inputs.WORKLOADS[name]
        pos, _, mass = w.initial_state()
        g = inputs.upstream_normal(w.n, w.seed + 400)
        if ordered:
            o = oracle.morton_order(pos)
            pos, mass, g = pos[:, o].copy(), mass[o].copy(), g[:, o].copy()
        k = ROWS[name]
        if k is None:
            rows = np.arange(w.n)
        else:
            com = (mass * pos).sum(axis=1) / mass.sum()
            central = np.argsort(np.linalg.norm(pos - com[:, None], axis=0),
                                 kind="stable")[:256]
            rows = np.union1d(w.rows(k), central)
        ra = oracle.accel_rows(pos, mass, w.G, w.eps, rows)
        rx, rm = oracle.accel_vjp_rows(pos, mass, g, w.G, w.eps, rows)
        _SYSTEMS.clear()
        _SYSTEMS[key] = (w, pos, mass, g, rows, ra, rx, rm)
    return _SYSTEMS[key]


@pytest.mark.parametrize("name,prec", sorted(CEILING))
def test_accuracy_ceiling(B, oracle, name, prec):
    w, pos, mass, g, rows, ra, rx, rm = _system(oracle, name, prec in SORTED)
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    P, M = T(pos), T(mass)
    a = B.nbody_accel(P, M, w.G, w.eps, prec).cpu().numpy()[:, rows]
    gx, gm = B.nbody_accel_vjp(P, M, T(g), w.G, w.eps, prec)
    gx, gm = gx.cpu().numpy()[:, rows], gm.cpu().numpy()[rows]
    e = metrics.rel_errors(a, ra)
    emax, enorm = CEILING[(name, prec)]
    vx, vm = VJP_CEILING[(name, prec)]
    ex, em = metrics.normwise(gx, rx), metrics.normwise(gm, rm)
    say("  %s %s (%d rows): E_max %.2e (ceiling %.1e) E_norm %.2e (ceiling %.1e) "
        "E_inf %.2e E_med %.2e; VJP normwise dL/dx %.2e (ceiling %.1e) dL/dm %.2e "
        "(ceiling %.1e)"
        % (name, prec, len(rows), e["E_max"], emax, e["E_norm"], enorm, e["E_inf"],
           e["E_med"], ex, vx, em, vm))
    assert e["E_max"] <= emax
    assert e["E_norm"] <= enorm
    assert ex <= vx
    assert em <= vm
