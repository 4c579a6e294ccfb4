"""Per-body error bounds of the GPU path, derived from its arithmetic.

For the acceleration a_i = G sum_j f_ij, f_ij = m_j d_ij w_ij with
w_ij = s_ij^-3/2, s_ij = |d_ij|^2 + eps^2 (d_ij = x_j - x_i):

* rounding each position to FP32 (NBODY_MIXED) perturbs d_ij by
  delta_ij <= u32 (|x_i| + |x_j| + |d_ij|); the rounded FP64 difference
  (NBODY_MIXED_D64) by delta_ij <= u32 |d_ij|; the near / far mode
  (NBODY_MIXED_NF) by delta_ij <= u32 (|x_j - c| + |x_i - c| + |d_ij|) on
  its far runs, where the workgroup target box's half-diagonal b bounds
  |x_i - c| and every pair has |d_ij| > kappa b = b / 2, so
  delta_ij < 6 u32 |d_ij|, and by u32 |d_ij| on its near runs (the D64
  arithmetic); the two-float difference (NBODY_MIXED_DS),
  (x_j^hi - x_i^hi) + (x_j^lo - x_i^lo) with hi = fl32(x), lo = fl32(x - hi),
  by delta_ij <= 2 u32 |d_ij| + 4 u32^2 (|x_i| + |x_j|) (the hi/lo split
  carries each coordinate to u32^2 |x|, the two FP32 differences and their
  sum round at most once each at the u32 level of |d| or u32^2 of |x|);
  FP64 inputs are exact;
* a perturbation delta of d changes f_ij by at most 4 G m_j w_ij delta
  (|d(d w)/dd| <= w (1 + 3 |d|^2 / s) <= 4 w);
* the pair arithmetic (three FMAs for s, the hardware reciprocal square root
  of a few ulp, three products and the accumulating FMA) adds at most
  c_pair u |f_ij| with c_pair = 16, and summing chunk sums of length L adds at
  most L u sum_j |f_ij| (gamma_L bound), L = 32 for the FP32 chunks and n for
  the FP64 path (whole source range, worst case).

so |a_i^gpu - a_i| <= SAFETY * G sum_j m_j w_ij (4 delta_ij + (16 + L) u |d_ij|).
The self pair j == i is left out: the kernels see d_ii = 0 exactly (both
ends are the same rounded value) and add exactly zero for it.
The VJP bound is the same construction over its terms (see vjp_bound).
These are worst-case bounds; the measured errors sit far below them.
"""
from __future__ import annotations

import hashlib

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
SAFETY = 2.0
CHUNK32 = 32
VJP_CHUNK32 = 32        # mixed_nf64's VJP: 16 (its bound with 32 is looser)


# Far runs of the near / far mode: a pair distance above kappa = 1/2 times
# the target box's half-diagonal gives delta < (2 + 2 / kappa) u32 |d|.
NF_DELTA = 6.0
# Two-float differences: delta <= 2 u32 |d| + 4 u32^2 (|x_i| + |x_j|).
DS_DELTA = 2.0
DS_DELTA_X = 4.0


def _delta(precision, xn, blk, dn):
    """Bound on the perturbation of the pair difference (rows blk, all j)."""
    if precision == "mixed":
        return U32 * (xn[blk, None] + xn[None, :] + dn)
    if precision == "mixed_d64":
        return U32 * dn
    if precision in ("mixed_nf", "mixed_nf64"):   # nf64: FP64 near runs, within it
        return NF_DELTA * U32 * dn
    if precision == "mixed_ds":
        return DS_DELTA * U32 * dn + DS_DELTA_X * U32 * U32 * (xn[blk, None] + xn[None, :])
    if precision == "fp64":
        return 0.0
    raise ValueError(precision)


def _rows_iter(rows, n):
    block = max(1, (1 << 22) // max(n, 1))
    for s in range(0, len(rows), block):
        yield rows[s:s + block]


# Every bound below is a fixed linear combination of a few sums over the
# source bodies that do not depend on the precision (only u, the chunk length
# and the coordinate perturbation delta do).  Those O(rows * n) sums are
# computed once per input and kept, so bounds for several precisions of the
# same system (e.g. 1024 rows of a 262144-body system) cost one pass.
_SUMS_CACHE = {}


def _key(*parts):
    h = hashlib.blake2b(digest_size=16)
    for p in parts:
        a = np.ascontiguousarray(p)
        h.update(str(a.shape).encode())
        h.update(str(a.dtype).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _cached(kind, fn, *parts):
    key = (kind, _key(*parts))
    if key not in _SUMS_CACHE:
        if len(_SUMS_CACHE) > 64:
            _SUMS_CACHE.clear()
        _SUMS_CACHE[key] = fn()
    return _SUMS_CACHE[key]


def accel_sums(pos, mass, eps, rows):
    """Per row i (self pair left out), with w = m_j s^-3/2 and dn = |d_ij|:
    S0 = sum w, S1 = sum w dn, S2 = sum w |x_j|; and |x_i|."""
    n = mass.size

    def compute():
        xn = np.linalg.norm(pos, axis=0)
        out = np.empty((4, len(rows)))
        k = 0
        for blk in _rows_iter(rows, n):
            d = pos[:, None, :] - pos[:, blk, None]             # (3, b, n)
            dn = np.sqrt((d * d).sum(axis=0))
            s = dn * dn + eps * eps
            w = mass[None, :] / (s * np.sqrt(s))
            w[np.arange(len(blk)), blk] = 0.0                   # self pair: exactly 0
            out[0, k:k + len(blk)] = w.sum(axis=1)
            out[1, k:k + len(blk)] = (w * dn).sum(axis=1)
            out[2, k:k + len(blk)] = (w * xn[None, :]).sum(axis=1)
            out[3, k:k + len(blk)] = xn[blk]
            k += len(blk)
        return out
    return _cached("accel", compute, pos, mass, np.float64(eps), rows)


def accel_bound(pos, mass, G, eps, precision, rows=None):
    """Bound on |a_i^gpu - a_i| (Euclidean) for each row i:
    SAFETY * |G| * sum_j w_ij (4 delta_ij + (16 + L) u |d_ij|)."""
    n = mass.size
    rows = np.arange(n) if rows is None else np.asarray(rows)
    S0, S1, S2, xi = accel_sums(pos, mass, eps, rows)
    if precision == "fp64":
        arith = (16 + n + 64) * U64 * S1
        pert = 0.0
    else:
        arith = (16 + CHUNK32) * U32 * S1
        if precision == "mixed":
            pert = 4.0 * U32 * (xi * S0 + S2 + S1)
        elif precision == "mixed_d64":
            pert = 4.0 * U32 * S1
        elif precision in ("mixed_nf", "mixed_nf64"):
            pert = 4.0 * NF_DELTA * U32 * S1
        elif precision == "mixed_ds":
            pert = 4.0 * (DS_DELTA * U32 * S1 + DS_DELTA_X * U32 * U32 * (xi * S0 + S2))
        else:
            raise ValueError(precision)
    return SAFETY * abs(G) * (pert + arith)


def vjp_sums(pos, mass, gacc, eps, rows):
    """Per row k (self pair left out), with y3 = s^-3/2, r = s^-1/2 and
    e = |x_j - x_k|: the sums over j of y3 |g_j| f and y3 m_j f for
    f in {1, e r, |x_j| r, r}, of y3 |g_j| f for f in {e, |x_j|}, and the
    row's own m_k, |g_k|, |x_k|."""
    n = mass.size

    def compute():
        xn = np.linalg.norm(pos, axis=0)
        gn = np.linalg.norm(gacc, axis=0)
        out = np.empty((13, len(rows)))
        k = 0
        for blk in _rows_iter(rows, n):
            e = pos[:, None, :] - pos[:, blk, None]
            en = np.sqrt((e * e).sum(axis=0))
            s = en * en + eps * eps
            r = 1.0 / np.sqrt(s)
            y3 = r * r * r
            y3[np.arange(len(blk)), blk] = 0.0                  # self pair: e = h = 0
            yg = y3 * gn[None, :]
            ym = y3 * mass[None, :]
            fs = (1.0, en * r, xn[None, :] * r, r)
            sl = slice(k, k + len(blk))
            for c, f in enumerate(fs):
                out[c, sl] = (yg * f).sum(axis=1)
                out[4 + c, sl] = (ym * f).sum(axis=1)
            out[8, sl] = (yg * en).sum(axis=1)
            out[9, sl] = (yg * xn[None, :]).sum(axis=1)
            out[10, sl] = mass[blk]
            out[11, sl] = gn[blk]
            out[12, sl] = xn[blk]
            k += len(blk)
        return out
    return _cached("vjp", compute, pos, mass, gacc, np.float64(eps), rows)


def vjp_bound(pos, mass, gacc, G, eps, precision, rows=None):
    """Bounds (|dL/dx_k err|, |dL/dm_k err|) for each row k.

    Terms: s^-3/2 [h - 3 (e.h) e / s] with |h| <= H = m_k |g_j| + m_j |g_k|,
    and (g_j . e) s^-3/2.  A perturbation delta of e changes the first by at
    most 12 H s^-3/2 delta / sqrt(s) and the second by 4 |g_j| s^-3/2 delta;
    the pair arithmetic adds c u of each term's magnitude bound 4 H s^-3/2
    (c = 40; the FP32 pairs sum y3 g_j, y3 m_j and y5 (e.h) e over a chunk
    and combine them with m_k, g_k and -3 at its end, each part carrying
    about 20 u of y3 H), plus the chunk summation as for the acceleration.
    The self pair (e = 0) is left out of the sums.  The split-form pairs
    drop it (it adds exactly 0).  The FP64 pairs that form h per pair (the
    FP64 VJP of small systems, two targets per lane, and the near runs of
    mixed_nf64) form h = fma(m_k, g_j, -(m_j g_k)), which
    for j == k is the rounding error delta of m_k g_k
    (|delta| <= u64 m_k |g_k|), add y3_self * delta with y3_self = eps^-3,
    and subtract the same product afterwards; what remains is the rounding
    of that one addition, at most u64 * eps^-3 * u64 * m_k |g_k| per row
    (added below)."""
    n = mass.size
    rows = np.arange(n) if rows is None else np.asarray(rows)
    v = vjp_sums(pos, mass, gacc, eps, rows)
    mk, gk, xk = v[10], v[11], v[12]
    # sums of A f with A = y3 H = m_k (y3 |g_j|) + |g_k| (y3 m_j)
    A = [mk * v[c] + gk * v[4 + c] for c in range(4)]     # f = 1, e r, |x_j| r, r
    Bsum, Be, Bx = v[0], v[8], v[9]                       # y3 |g_j| times 1, e, |x_j|
    if precision == "fp64":
        u, L = U64, n + 64
    else:
        u, L = U32, VJP_CHUNK32
    ax = 4.0 * (40 + L) * u * A[0]
    am = (16 + L) * u * Be
    if precision == "fp64":
        px = pm = 0.0
    elif precision == "mixed":
        px = 12.0 * U32 * (xk * A[3] + A[2] + A[1])
        pm = 4.0 * U32 * (xk * Bsum + Bx + Be)
    elif precision == "mixed_d64":
        px = 12.0 * U32 * A[1]
        pm = 4.0 * U32 * Be
    elif precision in ("mixed_nf", "mixed_nf64"):
        px = 12.0 * NF_DELTA * U32 * A[1]
        pm = 4.0 * NF_DELTA * U32 * Be
    elif precision == "mixed_ds":
        px = 12.0 * (DS_DELTA * U32 * A[1] + DS_DELTA_X * U32 * U32 * (xk * A[3] + A[2]))
        pm = 4.0 * (DS_DELTA * U32 * Be + DS_DELTA_X * U32 * U32 * (xk * Bsum + Bx))
    else:
        raise ValueError(precision)
    self_res = (U64 * eps ** -3 * U64 * mk * gk
                if precision in ("fp64", "mixed_nf64") else 0.0)
    return (SAFETY * abs(G) * (px + ax + self_res),
            SAFETY * abs(G) * (pm + am))


def adjoint_bound(oracle, pos, vel, mass, G, eps, dt, steps, gx, gv, ga,
                  precision, rows=None, scheme="kdk"):
    """Element-wise bounds (dL/dx_0, dL/dv_0, dL/dm) of the GPU reverse sweep.

    The reverse sweep is linear in the upstream gradients; its only
    approximate operation is the VJP.  Walking the exact sweep (oracle VJPs
    along the oracle trajectory) gives each step's abar_t, and each VJP adds
    at most vjp_bound(x_{t+1}, abar_t) to xbar and mbar.  An xbar error
    reaches vbar through vbar += dt xbar, and abar through (dt/2) vbar, whose
    effect on later VJPs is second order in dt and covered by a 25% margin.
    The sweep's own FP64 updates add at most 2 u64 of each running value per
    step (the GPU fuses vbar + dt xbar into one FMA, the oracle does not).
    With `rows`, bounds are formed for those rows only (the sweep itself is
    still exact over all bodies).  scheme "half_kick_drift" walks the sweep
    of the paper's update (no closing half-kick).
    """
    kdk = scheme == "kdk"
    h = 0.5 * dt
    traj = [np.array(pos, dtype=np.float64)]
    x, v, a = pos, vel, None
    for _ in range(steps):
        x, v, a = oracle.step(x, v, mass, G, eps, dt, 1, acc=a, scheme=scheme)
        traj.append(x)
    gxc = np.array(gx, dtype=np.float64)
    gvc = np.array(gv, dtype=np.float64)
    ab = (np.zeros_like(gxc) if ga is None else np.array(ga)) + (
        h * gvc if (steps and kdk) else 0)
    m = mass.size if rows is None else len(rows)
    sel = slice(None) if rows is None else np.asarray(rows)
    Bx, Bv, Bm = np.zeros(m), np.zeros(m), np.zeros(m)
    gmc = np.zeros(mass.size)

    def nrm(v):
        return np.sqrt((v[:, sel] ** 2).sum(axis=0))

    for t in range(steps - 1, -1, -1):
        vx, vm = oracle.accel_vjp(traj[t + 1], mass, ab, G, eps)
        bx, bm = vjp_bound(traj[t + 1], mass, ab, G, eps, precision, rows)
        gxc = gxc + vx
        gmc = gmc + vm
        gvc = gvc + dt * gxc
        # the sweep's own FP64 roundings (xbar += VJP, vbar += dt xbar)
        Bx += bx + 2 * U64 * nrm(gxc)
        Bm += bm + 2 * U64 * np.abs(gmc[sel])
        Bv += dt * Bx + 2 * U64 * nrm(gvc)
        ab = h * gvc + (h * gvc if (t > 0 and kdk) else 0)
    bx, bm = vjp_bound(traj[0], mass, ab, G, eps, precision, rows)
    vx, vm = oracle.accel_vjp(traj[0], mass, ab, G, eps)
    Bx += bx + 2 * U64 * nrm(gxc + vx)
    Bm += bm + 2 * U64 * np.abs((gmc + vm)[sel])
    return 1.25 * Bx, 1.25 * Bv, 1.25 * Bm


def accel_bound_f32(pos, mass, G, eps, rows=None):
    """Bound on |a_i^gpu - a_i| for the FP32-state path, whose inputs are
    exactly the FP32 values the oracle gets: each pair term carries 16 u32 of
    its magnitude, the FP32 sum over sources (each lane's share, the lane
    butterfly and the splits, depth at most n + 64) gamma_(n+64), and the
    final scaling by G one more rounding (2 u32 with the reduction's)."""
    n = mass.size
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.empty(len(rows))
    k = 0
    for blk in _rows_iter(rows, n):
        d = pos[:, None, :] - pos[:, blk, None]
        dn = np.sqrt((d * d).sum(axis=0))
        w = mass[None, :] * (dn * dn + eps * eps) ** -1.5
        term = w * dn
        term[np.arange(len(blk)), blk] = 0.0
        out[k:k + len(blk)] = abs(G) * term.sum(axis=1) * (16 + 2 + n + 64) * U32
        k += len(blk)
    return SAFETY * out


def lipschitz_accel(pos, mass, G, eps, dx):
    """max change of each a_i when every x_j moves by at most dx_j (norms):
    |d(d w)/dd| <= 4 w, so |delta a_i| <= G sum_j m_j 4 w_ij (dx_i + dx_j)."""
    n = mass.size
    out = np.empty(n)
    k = 0
    for blk in _rows_iter(np.arange(n), n):
        d = pos[:, None, :] - pos[:, blk, None]
        dn = np.sqrt((d * d).sum(axis=0))
        w = mass[None, :] * (dn * dn + eps * eps) ** -1.5
        w[np.arange(len(blk)), blk] = 0.0
        out[k:k + len(blk)] = abs(G) * (4.0 * w * (dx[blk, None] + dx[None, :])).sum(axis=1)
        k += len(blk)
    return out
