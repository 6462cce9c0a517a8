"""Oracle: the normal-approximation fluctuation mode (Sec. 4.3.1, the Kokkos port).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Kokkos port had no binomial or normal generator and drew normal deviates
from uniform ones with the Box-Muller transform (Box and Muller, 1958).  This module
takes the reading of a fluctuation mode that replaces each cell's binomial count by its
normal approximation:

* a cell (b, k) with N = floor(Q + 1/2) electrons and probability p = A_b * B_k (the
  same clipped axis integrals as the binomial mode) receives
  n = min(max(floor(N p + sqrt(N p (1 - p)) z + 1/2), 0), N), z a standard normal;
* the cells (b, 2m) and (b, 2m+1) take the two normals of one Box-Muller pair, from the
  Philox4x32-10 block the binomial mode gives them (counter (b ceil(N_t/2) + m,
  depo_id, event, plane << 24), key = the seed): u1 = 1 - uniform53(words 0, 1) in
  (0, 1], u2 = uniform53(words 2, 3) in [0, 1), r = sqrt(-2 ln u1), theta = 2 pi u2,
  z = r cos theta for the even tick and r sin theta for the odd one;
* so that an independent implementation reproduces every count bit for bit, ln is the
  sampler's det_log, and sqrt, cos and sin are evaluated here with IEEE-754 double
  +, -, *, / only, in a fixed order:
  - sqrt(x): x = m 2^e with e even and m in [1/2, 2); y = 1/sqrt(m) by seven Newton
    steps y <- y (3/2 - (m y) y / 2) from y = 3/2 - m/2; sqrt(x) = (m y) 2^(e/2);
  - cos 2 pi u, sin 2 pi u: t = 4u (exact), quadrant j = floor(t), f = t - j; for
    f > 1/2 the complement g = 1 - f (exact) is used, else g = f; x = g * (pi/2) rounded;
    sin x and cos x by their Maclaurin series to x^15 and x^16 in Horner form
    (coefficients 1/j! correctly rounded); then the complement swaps sin and cos and
    the quadrant rotates the pair.
"""
from __future__ import annotations

import numpy as np

from .fluct import _INV_FACT as INV_FACT_TABLE
from .fluct import MASK32, det_axis_probs, det_log, electrons, philox4x32_10, uniform53
from .raster import rows_touching, valid_row

HALF_PI = 1.5707963267948966
RSQRT_STEPS = 7


def det_sqrt(x):
    """sqrt(x) for x >= 0 by Newton steps on 1/sqrt(m) (IEEE +, -, *, / only)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)  # x = m 2^e, m in [1/2, 1)
    odd = (e & 1) == 1
    m = np.where(odd, m * 2.0, m)
    e = np.where(odd, e - 1, e)
    y = 1.5 - m * 0.5
    for _ in range(RSQRT_STEPS):
        y = y * (1.5 - ((m * y) * y) * 0.5)
    out = np.ldexp(m * y, e // 2)
    return np.where(x > 0.0, out, 0.0)


def det_sincos2pi(u):
    """(cos 2 pi u, sin 2 pi u) for u in [0, 1) (IEEE +, -, *, / only)."""
    u = np.asarray(u, np.float64)
    t = u * 4.0
    j = np.floor(t)
    f = t - j
    swap = f > 0.5
    g = np.where(swap, 1.0 - f, f)
    x = g * HALF_PI
    x2 = x * x
    s = INV_FACT_TABLE[15]
    for n in (13, 11, 9, 7, 5, 3, 1):  # sin x = x (1 - x^2/3! + x^4/5! - ...)
        s = INV_FACT_TABLE[n] - x2 * s
    s = x * s
    c = INV_FACT_TABLE[16]
    for n in (14, 12, 10, 8, 6, 4, 2, 0):  # cos x = 1 - x^2/2! + x^4/4! - ...
        c = INV_FACT_TABLE[n] - x2 * c
    sp = np.where(swap, c, s)  # sin and cos of (pi/2) f
    cp = np.where(swap, s, c)
    j = j.astype(np.int64)
    cos_t = np.select([j == 0, j == 1, j == 2], [cp, -sp, -cp], sp)
    sin_t = np.select([j == 0, j == 1, j == 2], [sp, cp, -sp], -cp)
    return cos_t, sin_t


def cell_normal(seed, plane, event, depo_id, b, k, n_ticks):
    """Standard normal of cell (b, k): the Box-Muller pair of the tick pair's Philox block."""
    b = np.asarray(b, np.int64)
    k = np.asarray(k, np.int64)
    b, k = np.broadcast_arrays(b, k)
    c0 = (b * ((int(n_ticks) + 1) // 2) + (k >> 1)).astype(np.uint64)
    c1 = np.asarray(depo_id, np.uint64) + np.zeros_like(c0)
    c2 = np.asarray(event, np.uint64) + np.zeros_like(c0)
    c3 = (np.asarray(plane, np.uint64) << np.uint64(24)) + np.zeros_like(c0)
    w0, w1, w2, w3 = philox4x32_10(c0, c1, c2, c3, int(seed) & MASK32, (int(seed) >> 32) & MASK32)
    z_even, z_odd = box_muller_words(w0, w1, w2, w3)
    return np.where((k & 1) == 1, z_odd, z_even)


def box_muller_words(w0, w1, w2, w3):
    """The Box-Muller pair of one Philox block's words: (r cos theta, r sin theta)."""
    u1 = 1.0 - uniform53(w0, w1)
    u2 = uniform53(w2, w3)
    r = det_sqrt(-2.0 * det_log(u1))
    cos_t, sin_t = det_sincos2pi(u2)
    return r * cos_t, r * sin_t


def normal_count(N, p, z):
    """min(max(floor(N p + sqrt(N p (1 - p)) z + 1/2), 0), N), elementwise (N >= 0, p in [0, 1])."""
    p = np.asarray(p, np.float64)
    z = np.asarray(z, np.float64)
    N = np.broadcast_to(np.asarray(N, np.int64), p.shape)
    Nf = N.astype(np.float64)
    mu = Nf * p
    var = mu * (1.0 - p)
    sd = det_sqrt(np.maximum(var, 0.0))
    x = np.floor((mu + sd * z) + 0.5)
    return np.minimum(np.maximum(x, 0.0), Nf).astype(np.int64)


def normal_patch(q, t, p, sigma_t, sigma_p, plane, event, depo_id, n_impacts, n_rows, n_ticks, seed,
                 nsigma=3.0, box=None):
    """Counts of one depo-plane row in the normal mode: (rows, ticks, n[b, k]) as int64."""
    q, t, p, st, sp = (float(v) for v in (q, t, p, sigma_t, sigma_p))
    if not valid_row(q, t, p, st, sp):
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 0), np.int64)
    N = electrons(q)
    b_lo, b_hi, k_lo, k_hi = box if box is not None else (0, None, 0, None)
    rows, a = det_axis_probs(n_impacts * p, n_impacts * sp, nsigma, n_rows, b_lo, b_hi)
    ticks, b = det_axis_probs(t, st, nsigma, n_ticks, k_lo, k_hi)
    if rows.size == 0 or ticks.size == 0 or N == 0:
        return rows, ticks, np.zeros((rows.size, ticks.size), np.int64)
    prob = a[:, None] * b[None, :]
    z = cell_normal(seed, plane, event, depo_id, rows[:, None], ticks[None, :], n_ticks)
    return rows, ticks, normal_count(N, prob, z)


def raster_normal(depos, planes, seed, nsigma=3.0, n_events=1):
    """Normal-mode grids (electron counts as float64), list over events of lists over planes."""
    grids = [[np.zeros((pl.n_impacts * pl.n_wires, pl.n_ticks)) for pl in planes] for _ in range(n_events)]
    for j in range(len(depos.q)):
        pi = int(depos.plane[j])
        ev = int(depos.event[j])
        pl = planes[pi]
        g = grids[ev][pi]
        rows, ticks, n = normal_patch(depos.q[j], depos.t[j], depos.p[j], depos.sigma_t[j], depos.sigma_p[j],
                                      pi, ev, int(depos.depo_id[j]), pl.n_impacts, g.shape[0], g.shape[1],
                                      seed, nsigma)
        if rows.size and ticks.size:
            g[np.ix_(rows, ticks)] += n
    return grids


def raster_normal_at(depos, plane_idx, plane, rows, ticks, seed, nsigma=3.0, event=0):
    """Normal-mode counts at selected cells of one plane (sampled checks of full-size grids):
    the sum over the rows touching the cells' bounding box of each row's restricted patch."""
    rows = np.asarray(rows, np.int64)
    ticks = np.asarray(ticks, np.int64)
    out = np.zeros(rows.size, np.int64)
    if rows.size == 0:
        return out
    b_lo, b_hi, k_lo, k_hi = int(rows.min()), int(rows.max()) + 1, int(ticks.min()), int(ticks.max()) + 1
    box = np.zeros((b_hi - b_lo, k_hi - k_lo), np.int64)
    for j in rows_touching(depos, plane_idx, plane, b_lo, b_hi, k_lo, k_hi, nsigma, event):
        rr, tt, n = normal_patch(depos.q[j], depos.t[j], depos.p[j], depos.sigma_t[j], depos.sigma_p[j],
                                 plane_idx, event, int(depos.depo_id[j]) & MASK32, plane.n_impacts, plane.n_rows,
                                 plane.n_ticks, seed, nsigma, box=(b_lo, b_hi, k_lo, k_hi))
        if rr.size and tt.size:
            box[np.ix_(rr - b_lo, tt - k_lo)] += n
    return box[rows - b_lo, ticks - k_lo]
