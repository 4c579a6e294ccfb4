"""Pins of the seeded input generators (paper_2203_08263_amd/inputs.py) against
the distributions they claim to sample.

* Uniform cube: positions U(-1, 1), velocities N(0, 0.1^2), masses
  U(0.5, 1)/N -- moments within a few standard errors, exact ranges.
* Plummer sphere (Aarseth, Henon & Wielen 1974 sampling, mass fraction cut at
  0.999): the radius quantiles follow the closed-form cumulative mass
  M(<r) = r^3 / (r^2 + a^2)^(3/2) (scaled by the cut) within binomial errors,
  and the sample is in virial equilibrium, 2K / |W| = 1 within its sampling
  noise (W from the oracle with a tiny softening).
* Seeds: the same seed gives the same arrays, another seed different ones.
"""
import math

import numpy as np
import pytest

from paper_2203_08263_amd import inputs


def test_uniform_cube_moments_and_ranges():
    n = 200000
    pos, vel, mass = inputs.uniform_cube(n, 11)
    assert pos.shape == (3, n) and vel.shape == (3, n) and mass.shape == (n,)
    assert pos.min() >= -1.0 and pos.max() < 1.0
    se = math.sqrt(1.0 / 3.0 / n)              # standard error of the mean
    assert np.all(np.abs(pos.mean(axis=1)) < 5 * se)
    assert np.all(np.abs(pos.var(axis=1) - 1.0 / 3.0) < 0.01)
    assert np.all(np.abs(vel.mean(axis=1)) < 5 * 0.1 / math.sqrt(n))
    assert np.all(np.abs(vel.std(axis=1) - 0.1) < 0.002)
    assert mass.min() >= 0.5 / n and mass.max() <= 1.0 / n
    assert abs(mass.sum() - 0.75) < 0.01


def _plummer_radius(q, a, cut):
    # r at which the enclosed mass fraction (of the truncated sample) is q
    x = q * cut
    return a / math.sqrt(x ** (-2.0 / 3.0) - 1.0)


@pytest.mark.parametrize("a", [1.0, 0.1])
def test_plummer_radius_quantiles(a):
    n = 40000
    pos, _, mass = inputs.plummer(n, 21, a=a)
    assert np.allclose(mass, 1.0 / n)
    r = np.sort(np.linalg.norm(pos, axis=0))
    for q in (0.05, 0.1, 0.25, 0.5, 0.75, 0.9, 0.95):
        # binomial error of the empirical quantile, mapped through the CDF:
        # the model radius must lie between the sample quantiles q -+ 4 sigma
        s = 4.0 * math.sqrt(q * (1 - q) / n)
        lo = r[int((q - s) * n)]
        hi = r[int((q + s) * n)]
        want = _plummer_radius(q, a, 0.999)
        assert lo <= want <= hi, (q, lo, want, hi)
    # the mass cut bounds every radius (plus the centre-of-mass shift)
    assert r[-1] <= _plummer_radius(1.0, a, 0.999) * 1.01 + 0.1 * a


def test_plummer_centre_of_mass_removed():
    pos, vel, mass = inputs.plummer(5000, 22)
    assert np.all(np.abs((mass * pos).sum(axis=1)) < 1e-12)
    assert np.all(np.abs((mass * vel).sum(axis=1)) < 1e-12)


def test_plummer_virial_equilibrium(oracle):
    n = 4096
    pos, vel, mass = inputs.plummer(n, 23)
    kin, pot = oracle.energy(pos, vel, mass, 1.0, 1e-4)
    ratio = 2.0 * kin / abs(pot)
    # K and W of N bodies fluctuate by ~ 1 / sqrt(N) relative (1.6 %);
    # allow 4 of those
    assert abs(ratio - 1.0) < 0.065, ratio


def test_seeds_reproducible():
    a = inputs.uniform_cube(1000, 5)
    b = inputs.uniform_cube(1000, 5)
    c = inputs.uniform_cube(1000, 6)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert not np.array_equal(a[0], c[0])
    p1 = inputs.plummer(1000, 5)
    p2 = inputs.plummer(1000, 5)
    for x, y in zip(p1, p2):
        assert np.array_equal(x, y)


def test_subset_rows_and_upstream():
    rows = inputs.subset_rows(1000, 64, 9)
    assert rows.dtype == np.int64 and len(rows) == 64
    assert np.all(np.diff(rows) > 0) and rows.min() >= 0 and rows.max() < 1000
    assert np.array_equal(rows, inputs.subset_rows(1000, 64, 9))
    g = inputs.upstream_normal(100000, 3)
    assert g.shape == (3, 100000)
    assert np.all(np.abs(g.mean(axis=1)) < 0.02)
    assert np.all(np.abs(g.std(axis=1) - 1.0) < 0.01)
