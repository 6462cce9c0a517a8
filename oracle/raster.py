"""Oracle: rasterisation of depositions into impact x tick charge grids (mean, no fluctuation).

Follows Sec. 2.1.1 of the paper: S(t, x) is computed by rasterising each energy
deposition into a small patch (about 20x20 cells) and scatter-adding all patches into
a large grid.  The paper fixes neither the patch shape nor the bin-integral formula;
this oracle takes the reading:

* the deposition is a 2D Gaussian in (tick, impact) with widths (sigma_t, I*sigma_p),
  truncated to the rectangle mu +- nsigma*sigma on each axis;
* each cell receives the Gaussian's integral over the part of the cell inside the
  rectangle: an erf difference per axis, the patch is the outer product;
* cells outside the grid are dropped (their charge is lost), no normalisation;
* a row whose values are not a deposition (Q < 0, sigma_t <= 0, sigma_p <= 0, or any of
  Q, t, p, sigma_t, sigma_p not finite) contributes nothing: the paper states the method
  for physical depositions only and is silent on such input (``valid_row``).

Everything is FP64.  Window bounds are formed as ``u = I*p``, ``su = I*sigma_p``,
``half = nsigma*su``, ``lo = u - half``, ``hi = u + half`` (same for time without the
factor I); bins run from floor(lo) to ceil(hi) - 1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def valid_row(q, t, p, sigma_t, sigma_p) -> bool:
    """Whether a depo-plane row describes a deposition: Q >= 0, both widths > 0, all finite.

    Rows failing this contribute nothing to the grid (and get zero gradients); the paper
    is silent on such input, this is the reading taken.
    """
    v = [float(x) for x in (q, t, p, sigma_t, sigma_p)]
    return all(math.isfinite(x) for x in v) and v[0] >= 0.0 and v[3] > 0.0 and v[4] > 0.0


def valid_rows(depos) -> np.ndarray:
    """``valid_row`` element-wise over a Depos structure of arrays."""
    q, t, p = (np.asarray(a, np.float64) for a in (depos.q, depos.t, depos.p))
    st, sp = (np.asarray(a, np.float64) for a in (depos.sigma_t, depos.sigma_p))
    fin = np.isfinite(q) & np.isfinite(t) & np.isfinite(p) & np.isfinite(st) & np.isfinite(sp)
    with np.errstate(invalid="ignore"):
        return fin & (q >= 0.0) & (st > 0.0) & (sp > 0.0)


def window(mu: float, sigma: float, nsigma: float):
    """Truncation window [lo, hi] and the bin range [k0, k1) it touches."""
    half = nsigma * sigma
    lo = mu - half
    hi = mu + half
    return lo, hi, math.floor(lo), math.ceil(hi)


def axis_weights(mu: float, sigma: float, nsigma: float, n_bins: int):
    """Clipped Gaussian bin integrals along one axis.

    Returns (bins, weights) for the bins that intersect the truncation window and lie in
    [0, n_bins).  weight_k = Phi((hi_k - mu)/sigma) - Phi((lo_k - mu)/sigma) with
    lo_k = max(k, lo), hi_k = min(k+1, hi).
    """
    lo, hi, k0, k1 = window(mu, sigma, nsigma)
    ks = np.arange(k0, k1, dtype=np.int64)
    if ks.size == 0:
        return ks, np.zeros(0)
    elo = np.maximum(ks.astype(np.float64), lo)
    ehi = np.minimum(ks.astype(np.float64) + 1.0, hi)
    w = 0.5 * (erf((ehi - mu) / (sigma * SQRT2)) - erf((elo - mu) / (sigma * SQRT2)))
    keep = (ks >= 0) & (ks < n_bins)
    return ks[keep], w[keep]


def patch(q, t, p, sigma_t, sigma_p, n_impacts, n_rows, n_ticks, nsigma=3.0):
    """Mean patch of one depo-plane row: (rows, ticks, Q * A_b * B_k); empty for an invalid row."""
    q, t, p, st, sp = (float(v) for v in (q, t, p, sigma_t, sigma_p))
    if not valid_row(q, t, p, st, sp):
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 0))
    u = n_impacts * p
    su = n_impacts * sp
    rows, a = axis_weights(u, su, nsigma, n_rows)
    ticks, b = axis_weights(t, st, nsigma, n_ticks)
    return rows, ticks, q * np.outer(a, b)


def raster(depos, planes, nsigma=3.0, n_events=1):
    """Scatter-add every row's patch into per-(event, plane) grids.

    Returns a list over events of lists over planes of float64 arrays [N_b][N_t].
    """
    grids = [[np.zeros((pl.n_impacts * pl.n_wires, pl.n_ticks)) for pl in planes] for _ in range(n_events)]
    for j in range(len(depos.q)):
        pl = planes[int(depos.plane[j])]
        g = grids[int(depos.event[j])][int(depos.plane[j])]
        rows, ticks, w = patch(depos.q[j], depos.t[j], depos.p[j], depos.sigma_t[j], depos.sigma_p[j],
                               pl.n_impacts, g.shape[0], g.shape[1], nsigma)
        if rows.size and ticks.size:
            g[np.ix_(rows, ticks)] += w
    return grids


def rows_touching(depos, plane_idx, plane, b_lo, b_hi, k_lo, k_hi, nsigma=3.0, event=0):
    """Indices of the depo rows of one plane whose window meets rows [b_lo, b_hi) x ticks [k_lo, k_hi).

    Window bounds are formed element-wise exactly as ``window`` forms them; invalid rows
    (``valid_row``) touch nothing.
    """
    I = plane.n_impacts
    m = (depos.plane == plane_idx) & (depos.event == event) & valid_rows(depos)
    p = depos.p.astype(np.float64)
    sp = depos.sigma_p.astype(np.float64)
    t = depos.t.astype(np.float64)
    st = depos.sigma_t.astype(np.float64)
    u = float(I) * p
    hu = nsigma * (float(I) * sp)
    ht = nsigma * st
    with np.errstate(invalid="ignore"):
        b0 = np.floor(u - hu)
        b1 = np.ceil(u + hu)
        k0 = np.floor(t - ht)
        k1 = np.ceil(t + ht)
        m &= (b0 < b_hi) & (b1 > b_lo) & (k0 < k_hi) & (k1 > k_lo)
    return np.nonzero(m)[0]


def raster_at(depos, plane_idx, plane, rows, ticks, nsigma=3.0, event=0):
    """Mean raster value at selected cells (rows[j], ticks[j]) of one plane.

    Only the depo rows whose window covers a cell contribute; used for sampled checks of
    full-size grids.
    """
    rows = np.asarray(rows, np.int64)
    ticks = np.asarray(ticks, np.int64)
    out = np.zeros(rows.size)
    if rows.size == 0:
        return out
    sel = rows_touching(depos, plane_idx, plane, rows.min(), rows.max() + 1, ticks.min(), ticks.max() + 1,
                        nsigma, event)
    I = plane.n_impacts
    for j in sel:
        q, t, p, st, sp = (float(v) for v in (depos.q[j], depos.t[j], depos.p[j], depos.sigma_t[j],
                                                depos.sigma_p[j]))
        ulo, uhi, b0, b1 = window(I * p, I * sp, nsigma)
        tlo, thi, k0, k1 = window(t, st, nsigma)
        hit = np.nonzero((rows >= b0) & (rows < b1) & (ticks >= k0) & (ticks < k1))[0]
        if hit.size == 0:
            continue
        r, a = axis_weights(I * p, I * sp, nsigma, plane.n_rows)
        k, b = axis_weights(t, st, nsigma, plane.n_ticks)
        amap = dict(zip(r.tolist(), a.tolist()))
        bmap = dict(zip(k.tolist(), b.tolist()))
        for h in hit:
            out[h] += q * amap.get(int(rows[h]), 0.0) * bmap.get(int(ticks[h]), 0.0)
    return out


def interior_patch_sum(q, nsigma=3.0):
    """Closed form: a patch whose window lies inside the grid sums to Q * erf(nsigma/sqrt2)^2."""
    return q * math.erf(nsigma / SQRT2) ** 2
