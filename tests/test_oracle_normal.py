"""Pins of the normal-approximation fluctuation oracle (oracle/normal.py; Sec. 4.3.1's
Box-Muller transform).

The deterministic sqrt, cos and sin are checked against libm; the cell normals against a
Box-Muller transform written with numpy's own log, sqrt, cos and sin on the binomial
mode's cell uniforms (which pins the word pairing and the complement u1 = 1 - u), and
against the normal and chi-square laws; the count against its closed form and its edge
cases; the patch against the moments of the approximated binomial over many seeds.
"""
import dataclasses

import numpy as np
from scipy import stats

from oracle import fluct as OF
from oracle import normal as ON
from oracle import raster as OR
from paper_2104_08265_amd import synth


def test_det_sqrt_within_two_ulp():
    rng = np.random.default_rng(1)
    x = np.concatenate([np.logspace(-300, 300, 20001), rng.random(100000) * 1e6, [0.25, 1.0, 2.0, 4.0, 1e-320]])
    r = ON.det_sqrt(x)
    ref = np.sqrt(x)
    assert np.all(np.abs(r - ref) <= 2 * np.spacing(ref))
    assert ON.det_sqrt(0.0) == 0.0
    k = np.arange(1, 5000, dtype=np.float64)
    assert np.all(np.abs(ON.det_sqrt(k * k) - k) <= 2 * np.spacing(k))


def test_det_sincos2pi_against_libm():
    rng = np.random.default_rng(2)
    u = np.concatenate([rng.random(200000), np.arange(256) / 256.0, 1.0 - 2.0 ** -53 * np.arange(1, 9)])
    c, s = ON.det_sincos2pi(u)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 1e-15
    assert np.max(np.abs(s - np.sin(2 * np.pi * u))) < 1e-15
    # quadrant edges are exact
    c, s = ON.det_sincos2pi(np.array([0.0, 0.25, 0.5, 0.75]))
    assert np.array_equal(c, [1.0, 0.0, -1.0, 0.0]) and np.array_equal(s, [0.0, 1.0, 0.0, -1.0])


def test_cell_normal_is_box_muller_of_the_cell_uniforms():
    """z(b, 2m) = sqrt(-2 ln(1 - u_even)) cos(2 pi u_odd), z(b, 2m+1) = ... sin(2 pi u_odd),
    where u_even and u_odd are the binomial mode's uniforms of the two cells."""
    seed, plane, event, depo, nt = 77, 2, 3, 12345, 101
    b = np.arange(40)[:, None]
    m = np.arange(51)[None, :]
    ue = OF.cell_uniform(seed, plane, event, depo, b, 2 * m, nt)
    uo = OF.cell_uniform(seed, plane, event, depo, b, 2 * m + 1, nt)
    r = np.sqrt(-2.0 * np.log(1.0 - ue))
    ze = ON.cell_normal(seed, plane, event, depo, b, 2 * m, nt)
    zo = ON.cell_normal(seed, plane, event, depo, b, 2 * m + 1, nt)
    assert np.allclose(ze, r * np.cos(2 * np.pi * uo), rtol=1e-13, atol=1e-14)
    assert np.allclose(zo, r * np.sin(2 * np.pi * uo), rtol=1e-13, atol=1e-14)


def test_cell_normals_follow_the_normal_law():
    b = np.arange(300)[:, None]
    k = np.arange(400)[None, :]
    z = ON.cell_normal(5, 1, 0, 42, b, k, 400)
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-4
    # the two normals of a pair: uncorrelated, and their squared sum is chi-square(2)
    ze, zo = z[:, 0::2].ravel(), z[:, 1::2].ravel()
    assert abs(np.corrcoef(ze, zo)[0, 1]) < 5.0 / np.sqrt(ze.size)
    assert stats.kstest(ze ** 2 + zo ** 2, "chi2", args=(2,)).pvalue > 1e-4
    # neighbouring pairs along ticks and rows are uncorrelated
    assert abs(np.corrcoef(ze[:-1], ze[1:])[0, 1]) < 5.0 / np.sqrt(ze.size)


def test_normal_count_closed_form_and_edges():
    rng = np.random.default_rng(3)
    N = rng.integers(1, 10 ** 6, 50000)
    p = rng.random(50000)
    z = rng.standard_normal(50000) * 2.0
    got = ON.normal_count(N, p, z)
    x = N * p + np.sqrt(N * p * (1.0 - p)) * z + 0.5
    ref = np.clip(np.floor(x), 0, N)
    near_half = np.abs(x - np.round(x)) < 1e-6  # a rounding-order difference may move these
    assert np.array_equal(got[~near_half], ref[~near_half])
    assert np.all(np.abs(got - ref) <= 1)
    # p = 0 gives 0, p = 1 gives N, N = 0 gives 0, z = 0 gives the rounded mean
    assert np.all(ON.normal_count(1000, np.zeros(5), np.linspace(-3, 3, 5)) == 0)
    assert np.all(ON.normal_count(1000, np.ones(5), np.linspace(-3, 3, 5)) == 1000)
    assert np.all(ON.normal_count(0, np.full(5, 0.3), np.linspace(-3, 3, 5)) == 0)
    assert ON.normal_count(1000, 0.2504, 0.0) == 250 and ON.normal_count(1000, 0.2506, 0.0) == 251
    # clamped to [0, N]
    assert ON.normal_count(10, 0.1, -50.0) == 0 and ON.normal_count(10, 0.9, 50.0) == 10


def test_patch_moments_match_the_binomial():
    """Over many seeds each cell's count has mean N p and variance N p (1 - p) (those of
    the binomial it approximates), p from the clipped axis integrals."""
    q, t, p, st, sp = 20000.0, 30.3, 0.52, 2.0, 0.05
    I, nr, nt = 10, 200, 64
    rows, ticks, a = None, None, []
    for seed in range(1500):
        rows, ticks, n = ON.normal_patch(q, t, p, st, sp, 0, 0, 7, I, nr, nt, seed)
        a.append(n)
    a = np.array(a, np.float64)
    rr, wa = OF.det_axis_probs(I * p, I * sp, 3.0, nr)
    tt, wb = OF.det_axis_probs(t, st, 3.0, nt)
    assert np.array_equal(rr, rows) and np.array_equal(tt, ticks)
    prob = wa[:, None] * wb[None, :]
    N = OF.electrons(q)
    mean, var = N * prob, N * prob * (1.0 - prob)
    big = mean > 50  # the normal approximation's regime (no clamping at 0 within 7 sigma)
    se = np.sqrt(var / a.shape[0])
    assert np.all(np.abs(a.mean(0) - mean)[big] < 5.0 * se[big] + 0.02)
    rel = a.var(0, ddof=1)[big] / var[big]
    assert np.all(np.abs(rel - 1.0) < 5.0 * np.sqrt(2.0 / (a.shape[0] - 1)))


def test_invalid_rows_and_zero_charge_draw_nothing():
    for row in ((-5.0, 10.0, 0.5, 1.0, 0.1), (1e4, np.nan, 0.5, 1.0, 0.1), (1e4, 10.0, 0.5, 0.0, 0.1),
                (1e4, 10.0, 0.5, 1.0, -0.1), (0.3, 10.0, 0.5, 1.0, 0.1)):
        rows, ticks, n = ON.normal_patch(*row, 0, 0, 1, 10, 100, 64, 9)
        assert n.sum() == 0


def test_sampled_cells_equal_the_full_grid():
    wl = synth.config1()
    grids = ON.raster_normal(wl.depos, wl.planes, 123)
    rng = np.random.default_rng(4)
    for pi, pl in enumerate(wl.planes):
        g = grids[0][pi]
        nz = np.argwhere(g != 0)
        pick = nz[rng.choice(len(nz), 60, replace=False)]
        rows = np.concatenate([pick[:, 0], rng.integers(0, g.shape[0], 20)])
        ticks = np.concatenate([pick[:, 1], rng.integers(0, g.shape[1], 20)])
        got = ON.raster_normal_at(wl.depos, pi, pl, rows, ticks, 123)
        assert np.array_equal(got, g[rows, ticks])


def test_mean_grid_is_the_expectation():
    """Summed over 400 seeds the normal-mode grid approaches the mean raster Q A_b B_k (for
    integer Q), cells of mean above 30 within 5 standard errors."""
    wl = synth.config1()
    mask = np.zeros(len(wl.depos), bool)
    mask[np.nonzero(wl.depos.plane == 0)[0][:6]] = True
    d = wl.depos.select(mask)
    d = dataclasses.replace(d, q=np.floor(d.q + 0.5))
    mean = OR.raster(d, wl.planes)[0][0]
    acc = np.zeros_like(mean)
    for seed in range(400):
        acc += ON.raster_normal(d, wl.planes, seed)[0][0]
    acc /= 400
    big = mean > 30
    assert big.sum() > 10
    assert np.all(np.abs(acc - mean)[big] < 5.0 * np.sqrt(mean[big] / 400) + 0.02)
