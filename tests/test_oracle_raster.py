"""Pins for the oracle's mean raster (Sec. 2.1.1: rasterisation + scatter adding)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import raster as R
from paper_2104_08265_amd import synth

ERF3 = 0.9973002039367398  # erf(3/sqrt2): mass of a unit Gaussian inside +-3 sigma


def test_interior_axis_sum_closed_form():
    for mu, s in [(10.37, 1.3), (50.0, 2.0), (20.5, 0.71), (33.999, 0.05)]:
        _, w = R.axis_weights(mu, s, 3.0, 1000)
        assert abs(w.sum() - ERF3) < 1e-14
    assert abs(math.erf(3 / math.sqrt(2)) - ERF3) < 1e-16


@pytest.mark.parametrize("mu,s", [(10.37, 1.3), (5.2, 0.4), (7.0, 2.6)])
def test_bins_match_quadrature(mu, s):
    """Each clipped bin weight equals the numerically integrated Gaussian pdf over the clipped cell."""
    bins, w = R.axis_weights(mu, s, 3.0, 1000)
    lo, hi = mu - 3 * s, mu + 3 * s
    for k, wk in zip(bins, w):
        a, b = max(k, lo), min(k + 1, hi)
        ref, _ = integrate.quad(lambda x: stats.norm.pdf(x, mu, s), a, b, epsabs=1e-15, epsrel=1e-14)
        assert abs(ref - wk) < 1e-14


def test_symmetric_about_bin_centre():
    bins, w = R.axis_weights(12.5, 1.7, 3.0, 100)
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-15)
    assert bins[0] + bins[-1] == 24


def test_grid_edge_drops_charge_exactly():
    """A window straddling the grid's low edge keeps exactly Phi(hi) - Phi(edge) of the mass."""
    mu, s = 1.2, 1.0
    bins, w = R.axis_weights(mu, s, 3.0, 100)
    assert bins[0] == 0
    expect = stats.norm.cdf(3.0) - stats.norm.cdf((0.0 - mu) / s)
    assert abs(w.sum() - expect) < 1e-14


def test_patch_sum_interior_and_clipped():
    q = 5123.0
    rows, ticks, w = R.patch(q, 100.3, 20.41, 2.1, 0.7, 10, 500, 400)
    assert abs(w.sum() - R.interior_patch_sum(q)) < 1e-12 * q
    assert abs(R.interior_patch_sum(1.0) - 0.9946076967722628) < 1e-15
    # at the top-right corner of the grid: product of the kept fractions
    rows, ticks, w = R.patch(q, 398.9, 49.95, 1.5, 0.5, 10, 500, 400)
    fa = stats.norm.cdf((500 - 499.5) / 5.0) - stats.norm.cdf(-3.0)
    fb = stats.norm.cdf((400 - 398.9) / 1.5) - stats.norm.cdf(-3.0)
    assert abs(w.sum() - q * fa * fb) < 1e-10 * q


def test_small_sigma_limit():
    bins, w = R.axis_weights(7.3, 1e-4, 3.0, 100)
    assert list(bins) == [7]
    assert abs(w[0] - ERF3) < 1e-12


def test_continuity_when_a_bin_enters_the_window():
    """Moving mu across the point where lo = integer changes the weights continuously."""
    s = 1.0
    mu0 = 10.0 + 3.0  # lo = 10 exactly
    for eps in (1e-9, 1e-7):
        b1, w1 = R.axis_weights(mu0 - eps, s, 3.0, 100)
        b2, w2 = R.axis_weights(mu0 + eps, s, 3.0, 100)
        d1 = dict(zip(b1.tolist(), w1.tolist()))
        d2 = dict(zip(b2.tolist(), w2.tolist()))
        for k in set(d1) | set(d2):
            assert abs(d1.get(k, 0.0) - d2.get(k, 0.0)) < 10 * eps


def test_linearity():
    wl = synth.tiny(n_depos=10, seed=3)
    pl = wl.planes
    d = wl.depos
    g_all = R.raster(d, pl)[0][0]
    g1 = R.raster(d.select(np.arange(len(d)) < 4), pl)[0][0]
    g2 = R.raster(d.select(np.arange(len(d)) >= 4), pl)[0][0]
    assert np.allclose(g_all, g1 + g2, rtol=0, atol=1e-12)
    d3 = d.astype(np.float64)
    d3.q = d3.q * 2.5
    g3 = R.raster(d3, pl)[0][0]
    assert np.allclose(g3, 2.5 * g_all, rtol=1e-14, atol=1e-12)


def test_raster_at_matches_full_grid():
    wl = synth.tiny(n_wires=8, n_ticks=50, n_depos=15, seed=5)
    g = R.raster(wl.depos, wl.planes)[0][0]
    rng = np.random.default_rng(0)
    rows = rng.integers(0, g.shape[0], 200)
    ticks = rng.integers(0, g.shape[1], 200)
    v = R.raster_at(wl.depos, 0, wl.planes[0], rows, ticks)
    assert np.allclose(v, g[rows, ticks], rtol=1e-14, atol=1e-12)


def test_invalid_rows_contribute_nothing():
    """Rows that are not depositions (Q < 0, sigma_t or sigma_p <= 0, a non-finite value) add
    nothing: the grid with them equals the grid of the valid rows alone, exactly, and the
    sampled evaluation skips them too."""
    pl = synth.Plane(12, 200, 10, 2, 12)
    rng = np.random.default_rng(5)
    good = [(float(rng.lognormal(7, 1)), float(rng.uniform(10, 190)), float(rng.uniform(1, 11)),
             float(rng.uniform(0.5, 3)), float(rng.uniform(0.1, 1))) for _ in range(10)]
    bad = [(-500.0, 50.0, 5.0, 1.0, 0.3), (900.0, 50.0, 5.0, 0.0, 0.3), (900.0, 50.0, 5.0, 1.0, 0.0),
           (900.0, 50.0, 5.0, -1.0, 0.3), (900.0, float("nan"), 5.0, 1.0, 0.3),
           (900.0, 50.0, float("inf"), 1.0, 0.3), (float("nan"), 50.0, 5.0, 1.0, 0.3)]
    a = np.array(good + bad)
    n = len(a)
    d = synth.Depos(a[:, 0], a[:, 1], a[:, 2], a[:, 3], a[:, 4], np.zeros(n, np.int32), np.zeros(n, np.int32),
                    np.arange(n, dtype=np.int32))
    for row in bad:
        rows, ticks, w = R.patch(*row, 10, pl.n_rows, pl.n_ticks)
        assert rows.size == 0 and ticks.size == 0 and w.size == 0
    ref = R.raster(d.select(np.arange(n) < len(good)), [pl])[0][0]
    got = R.raster(d, [pl])[0][0]
    assert np.isfinite(got).all() and np.array_equal(got, ref)
    b, k = np.nonzero(ref)
    assert np.allclose(R.raster_at(d, 0, pl, b[:40], k[:40]), ref[b[:40], k[:40]], rtol=1e-14, atol=0)
