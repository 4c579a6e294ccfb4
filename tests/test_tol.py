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
        # FP64 pairs with h formed per pair leave a self-pair residue (the
        # split-form pairs drop the self pair)
        self_res = (_tol.U64 * eps ** -3 * _tol.U64 * mass[k] * gn[k]
                    if prec in ("fp64", "mixed_nf64") else 0.0)
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


# ------------------------------------------------------------------------
# The per-pair coordinate perturbations that every bound above is built on,
# checked against the FP32 arithmetic itself (NumPy float32 operations round
# correctly, as the GPU's do): random pairs over many decades of separation
# and offset, componentwise exactly as the kernels form the difference.

def _pairs(seed, m=200000):
    rng = np.random.default_rng(seed)
    off = 10.0 ** rng.uniform(-3, 3, m) * rng.choice([-1, 1], m)
    xi = off[None, :] + rng.normal(size=(3, m)) * 10.0 ** rng.uniform(-3, 1, m)
    d = rng.normal(size=(3, m)) * 10.0 ** rng.uniform(-7, 0.5, m)
    xj = xi + d
    d = xj - xi                       # the FP64 difference the oracle sees
    return xi, xj, d


def _worst(err, bound):
    return float(np.max(np.linalg.norm(err, axis=0) / bound))


def test_mixed_difference_within_delta():
    xi, xj, d = _pairs(1)
    got = (xj.astype(np.float32) - xi.astype(np.float32)).astype(np.float64)
    xn = np.stack([np.linalg.norm(xi, axis=0), np.linalg.norm(xj, axis=0)])
    bound = _tol.U32 * (xn[0] + xn[1] + np.linalg.norm(d, axis=0))
    assert _worst(got - d, bound) <= 1.0


def test_d64_difference_within_delta():
    xi, xj, d = _pairs(2)
    got = (xj - xi).astype(np.float32).astype(np.float64)
    bound = _tol.U32 * np.linalg.norm(d, axis=0) * (1 + 2 * _tol.U64 / _tol.U32)
    assert _worst(got - d, bound) <= 1.0


def test_two_float_difference_within_delta():
    """NBODY_MIXED_DS: hi = fl32(x), lo = fl32(x - hi); the difference is
    (x_j^hi - x_i^hi) + (x_j^lo - x_i^lo) in FP32."""
    xi, xj, d = _pairs(3)

    def split(x):
        hi = x.astype(np.float32)
        lo = (x - hi.astype(np.float64)).astype(np.float32)
        return hi, lo
    ih, il = split(xi)
    jh, jl = split(xj)
    got = ((jh - ih) + (jl - il)).astype(np.float64)          # float32 operations
    xn = np.linalg.norm(xi, axis=0) + np.linalg.norm(xj, axis=0)
    bound = (_tol.DS_DELTA * _tol.U32 * np.linalg.norm(d, axis=0)
             + _tol.DS_DELTA_X * _tol.U32 ** 2 * xn)
    w = _worst(got - d, bound)
    assert w <= 1.0
    # and it is not loose by orders of magnitude: the worst pair uses a good
    # part of it
    assert w >= 0.1


def test_near_far_recentred_difference_within_delta():
    """Far runs of the near / far modes: x - c rounded once to FP32 for both
    bodies (c the target box's centre, |x_i - c| <= b), pairs with
    |d| > kappa b (kappa = 1/2): delta < 6 u32 |d|."""
    rng = np.random.default_rng(4)
    m = 200000
    b = 10.0 ** rng.uniform(-4, 1, m)
    c = rng.normal(size=(3, m)) * 10.0 ** rng.uniform(-2, 3, m)
    u = rng.normal(size=(3, m))
    u /= np.linalg.norm(u, axis=0)
    xi = c + u * b * rng.uniform(0, 1, m)                      # |x_i - c| <= b
    dirn = rng.normal(size=(3, m))
    dirn /= np.linalg.norm(dirn, axis=0)
    xj = xi + dirn * b * (0.5 + 10.0 ** rng.uniform(-6, 3, m))  # |d| > b / 2
    d = xj - xi
    got = ((xj - c).astype(np.float32) - (xi - c).astype(np.float32)).astype(np.float64)
    bound = _tol.NF_DELTA * _tol.U32 * np.linalg.norm(d, axis=0)
    assert _worst(got - d, bound) <= 1.0


# ------------------------------------------------------------------------
# The FP32 VJP pair arithmetic (split form) against the arithmetic part of
# vjp_bound: chunks of VJP_CHUNK32 sources around one target, every
# operation rounded to FP32 as the kernels round it (an FMA of FP32 operands
# is exact in FP64 up to its one final rounding), the hardware reciprocal
# square root taken as the correctly rounded value times (1 + r) with
# |r| <= 2^-23.3, its measured worst relative error.

def _f(x):
    return np.float32(x)


def _fma(a, b, c):
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def _split_chunk(e, mj, gj, mk, gk, eps2, r):
    """dL/dx_k contribution of one chunk, FP32 split-form arithmetic."""
    acc = np.zeros(8, dtype=np.float32)             # ax ay az b cx cy cz dm
    for u in range(e.shape[1]):
        ex, ey, ez = (_f(v) for v in e[:, u])
        s = _fma(ex, ex, eps2)
        s = _fma(ey, ey, s)
        s = _fma(ez, ez, s)
        y = _f(np.float64(_f(1.0 / np.sqrt(np.float64(s)))) * (1.0 + r[u]))
        y2 = _f(y * y)
        y3 = _f(y2 * y)
        gx, gy, gz = (_f(v) for v in gj[:, u])
        ge = _fma(gz, ez, _fma(gy, ey, _f(gx * ex)))
        ek = _fma(gk[2], ez, _fma(gk[1], ey, _f(gk[0] * ex)))
        eh = _fma(mk, ge, -_f(mj[u] * ek))
        w = _f(y3 * _f(y2 * eh))
        acc[7] = _fma(ge, y3, acc[7])
        acc[0] = _fma(y3, gx, acc[0])
        acc[1] = _fma(y3, gy, acc[1])
        acc[2] = _fma(y3, gz, acc[2])
        acc[3] = _fma(y3, mj[u], acc[3])
        acc[4] = _fma(w, ex, acc[4])
        acc[5] = _fma(w, ey, acc[5])
        acc[6] = _fma(w, ez, acc[6])
    return np.array([np.float64(_fma(_f(-3.0), acc[4 + c],
                                     _fma(mk, acc[c], -_f(gk[c] * acc[3]))))
                     for c in range(3)])


def test_vjp_split_pair_arithmetic_within_bound():
    rng = np.random.default_rng(5)
    L = _tol.VJP_CHUNK32
    worst = 0.0
    for t in range(300):
        eps = 10.0 ** rng.uniform(-4, -1)
        eps2 = _f(eps * eps)
        scale = 10.0 ** rng.uniform(-4, 1)          # source distances
        e = (rng.normal(size=(3, L)) * scale).astype(np.float32).astype(np.float64)
        if t % 3 == 0:
            e[:, : L // 4] *= 1e-3                  # a few close sources
        mj = (10.0 ** rng.uniform(-3, 0, L)).astype(np.float32)
        gj = rng.normal(size=(3, L)).astype(np.float32).astype(np.float64)
        mk = _f(10.0 ** rng.uniform(-3, 0))
        gk = rng.normal(size=3).astype(np.float32)
        r = rng.uniform(-1, 1, L) * 2.0 ** -23.3
        got = _split_chunk(e, mj, gj, mk, gk, eps2, r)
        # exact row terms in FP64 from the same FP32 inputs
        s = (e * e).sum(axis=0) + np.float64(eps2)
        y3 = s ** -1.5
        h = np.float64(mk) * gj - mj.astype(np.float64) * gk.astype(np.float64)[:, None]
        eh = (e * h).sum(axis=0)
        ref = (y3 * (h - 3.0 * eh * e / s)).sum(axis=1)
        H = np.float64(mk) * np.linalg.norm(gj, axis=0) + \
            mj * np.linalg.norm(gk.astype(np.float64))
        bound = 4.0 * (40 + L) * _tol.U32 * (y3 * H).sum()
        worst = max(worst, np.linalg.norm(got - ref) / bound)
    assert worst <= 1.0, worst
