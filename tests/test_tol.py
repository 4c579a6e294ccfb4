"""The per-body error bounds of tests/_tol.py (used by every GPU parity test)
are computed from a few cached sums over the sources; this checks that the
factored form equals the direct per-pair evaluation of the same formula for
every precision, so the refactoring changes no bound."""
import numpy as np
import pytest

import _tol
from paper_2203_08263_amd import inputs

PRECS = ["fp64", "mixed", "mixed_d64", "mixed_nf", "mixed_nf64", "mixed_ds"]


def _direct_accel(pos, mass, G, eps, prec, rows):
    n = mass.size
    xn = np.linalg.norm(pos, axis=0)
    u, L = (_tol.U64, n + 64) if prec == "fp64" else (_tol.U32, _tol.CHUNK32)
    out = []
    for i in rows:
        d = pos - pos[:, i:i + 1]
        dn = np.sqrt((d * d).sum(axis=0))
        w = mass / (dn * dn + eps * eps) ** 1.5
        delta = _tol._delta(prec, xn, np.array([i]), dn[None, :])[0] \
            if prec != "fp64" else 0.0
        t = w * (4.0 * delta + (16 + L) * u * dn)
        t[i] = 0.0
        out.append(_tol.SAFETY * abs(G) * t.sum())
    return np.array(out)


def _direct_vjp(pos, mass, g, G, eps, prec, rows):
    n = mass.size
    xn = np.linalg.norm(pos, axis=0)
    gn = np.linalg.norm(g, axis=0)
    u, L = (_tol.U64, n + 64) if prec == "fp64" else (_tol.U32, _tol.VJP_CHUNK32)
    bx, bm = [], []
    for k in rows:
        e = pos - pos[:, k:k + 1]
        en = np.sqrt((e * e).sum(axis=0))
        s = en * en + eps * eps
        y3 = s ** -1.5
        H = mass[k] * gn + mass * gn[k]
        delta = _tol._delta(prec, xn, np.array([k]), en[None, :])[0] \
            if prec != "fp64" else 0.0
        tx = y3 * H * (12.0 * delta / np.sqrt(s) + (40 + L) * u * 4.0)
        tm = y3 * gn * (4.0 * delta + (16 + L) * u * en)
        tx[k] = tm[k] = 0.0
        self_res = u * eps ** -3 * u * mass[k] * gn[k]
        bx.append(_tol.SAFETY * abs(G) * (tx.sum() + self_res))
        bm.append(_tol.SAFETY * abs(G) * tm.sum())
    return np.array(bx), np.array(bm)


@pytest.mark.parametrize("prec", PRECS)
def test_factored_bounds_equal_direct_formula(prec):
    pos, _, mass = inputs.uniform_cube(700, 4242)
    pos = pos + np.array([[0.3], [-0.2], [0.1]])      # |x| varies by body
    g = inputs.upstream_normal(700, 4243)
    rows = np.array([0, 5, 17, 350, 699])
    G, eps = 1.3, 2e-3
    ref = _direct_accel(pos, mass, G, eps, prec, rows)
    got = _tol.accel_bound(pos, mass, G, eps, prec, rows)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    rx, rm = _direct_vjp(pos, mass, g, G, eps, prec, rows)
    bx, bm = _tol.vjp_bound(pos, mass, g, G, eps, prec, rows)
    np.testing.assert_allclose(bx, rx, rtol=1e-12)
    np.testing.assert_allclose(bm, rm, rtol=1e-12)


def test_sums_cache_keys_on_content():
    pos, _, mass = inputs.uniform_cube(300, 11)
    rows = np.arange(10)
    b1 = _tol.accel_bound(pos, mass, 1.0, 1e-3, "mixed", rows)
    pos2 = pos.copy()
    pos2[0, 3] += 0.25                                  # same shape, new content
    b2 = _tol.accel_bound(pos2, mass, 1.0, 1e-3, "mixed", rows)
    assert not np.array_equal(b1, b2)
    np.testing.assert_array_equal(_tol.accel_bound(pos, mass, 1.0, 1e-3, "mixed", rows),
                                  b1)
