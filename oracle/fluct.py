"""Oracle: binomial fluctuation of the rasterised charge (Sec. 4.3.1, Table 2).

The paper states that the fluctuation is binomial (the CPU reference draws with
std::binomial_distribution) and that generating the random numbers dominated the CPU
rasterisation time, which is why the GPU ports factor the RNG out of the main loop.
It fixes neither the generator nor the sampler.  This module takes the reading:

* every impact x tick cell (b, k) of a deposition's truncated window receives an
  independent count n_bk ~ Binomial(N, p_bk) with N = floor(Q + 1/2) electrons and
  p_bk = A_b * B_k, the product of the two clipped axis integrals (no renormalisation,
  so E[n_bk] equals the mean raster for integer Q);
* the uniform variate of cell (b, k) comes from the counter-based generator
  Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) keyed by the run seed; the two
  cells (b, 2m) and (b, 2m+1) share the block with counter
  (b*ceil(N_t/2) + m, depo_id, event, plane << 24), the even tick using output words
  0-1 and the odd tick words 2-3 (draw-stream version 2);
* the variate is mapped to a count by a fixed two-regime sampler, where
  p' = min(p, 1-p), q = 1 - p' and a draw with p > 1/2 is N minus the draw with p':
  - N = 0 or p <= 0 gives 0, p >= 1 gives N;
  - inversion from 0 when N*p' < 10: f = q^N by left-to-right square-and-multiply,
    F = f, k = 0; while u >= F and k < min(N, 128): f = f * (r * (N - k)) * (1/(k+1))
    with r = p'/q and 1/(k+1) a correctly rounded table entry, k = k + 1, F = F + f.
    The step cap INVERSION_CAP = 128 is part of the stream: with N*p' < 10 the exact
    probability of a count >= 128 is below 1e-70, so the cap only decides the rare u
    that exceed the rounded sum F (which can saturate just below 1), and those return
    min(N, 128);
  - otherwise a chop-down search from the mode m = min(floor((N+1) p'), N) with
    P(m) = exp(ln N! - ln m! - ln (N-m)! + m ln p' + (N-m) ln q), v = u - P(m), then
    alternately one step below (while the lower side is above 0 and its probability
    has not underflowed) and one step above, subtracting each new probability from v,
    returning the first index where v < 0 (m if both sides are exhausted).

Because the sampler is part of the specification, every step uses only IEEE-754
double +, -, *, / (no fused multiply-add, no library transcendental), in a fixed order,
so an independent implementation reproduces every count bit for bit.  The erf, log,
exp and log-factorial used by the sampler are written here as plain series:

* erf(x)   = 2/sqrt(pi) * sum_{j<60} x * (-x^2)^j / j! / (2j+1), by term recurrence;
* log(x)   = e*ln2 + 2*atanh(s), x = m*2^e with m in [sqrt(1/2), sqrt(2)),
             s = (m-1)/(m+1), 12 odd terms in Horner form;
* exp(x)   = 2^n * sum_{j<=16} r^j/j!, n = rint(x*log2 e), r = x - n*ln2;
* ln n!    = log(n!) for n <= 18, else Stirling with terms to 1/(1680 n^7).

Vectorised numpy code is used where the operation order per element is unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from .raster import rows_touching, valid_row, window

# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11): 10 rounds, two 32x32->64 multiplies per round,
# key bumped by the Weyl constants between rounds.
# ---------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 counters; returns four uint32 words."""
    c0 = np.asarray(c0, np.uint64) & MASK32
    c1 = np.asarray(c1, np.uint64) & MASK32
    c2 = np.asarray(c2, np.uint64) & MASK32
    c3 = np.asarray(c3, np.uint64) & MASK32
    k0 = np.uint64(k0 & MASK32) + np.zeros_like(c0)
    k1 = np.uint64(k1 & MASK32) + np.zeros_like(c0)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(MASK32)
            k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(MASK32)
        p0 = c0 * m0  # < 2^64: exact in uint64
        p1 = c2 * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32), c3.astype(np.uint32))


def uniform53(w0, w1):
    """Exact 53-bit uniform in [0, 1): ((w0 >> 6) * 2^27 + (w1 >> 5)) * 2^-53."""
    a = (np.asarray(w0, np.uint64) >> np.uint64(6)).astype(np.float64)
    b = (np.asarray(w1, np.uint64) >> np.uint64(5)).astype(np.float64)
    return (a * 134217728.0 + b) * (2.0 ** -53)


def cell_uniform(seed, plane, event, depo_id, b, k, n_ticks):
    """Uniform variate of cell (b, k): the block of counter
    (b*ceil(N_t/2) + floor(k/2), depo_id, event, plane << 24) under key = seed, words 0-1
    for even k and words 2-3 for odd k."""
    b = np.asarray(b, np.int64)
    k = np.asarray(k, np.int64)
    b, k = np.broadcast_arrays(b, k)
    c0 = (b * ((int(n_ticks) + 1) // 2) + (k >> 1)).astype(np.uint64)
    c1 = np.asarray(depo_id, np.uint64) + np.zeros_like(c0)
    c2 = np.asarray(event, np.uint64) + np.zeros_like(c0)
    c3 = (np.asarray(plane, np.uint64) << np.uint64(24)) + np.zeros_like(c0)
    w0, w1, w2, w3 = philox4x32_10(c0, c1, c2, c3, int(seed) & MASK32, (int(seed) >> 32) & MASK32)
    return np.where((k & 1) == 1, uniform53(w2, w3), uniform53(w0, w1))


# ---------------------------------------------------------------------------
# deterministic double-precision functions (IEEE +,-,*,/ only)
# ---------------------------------------------------------------------------
ERF_TERMS = 60
TWO_OVER_SQRTPI = 1.1283791670955126
SQRT2 = 1.4142135623730951
SQRT_HALF = 0.7071067811865476
LN2 = 0.6931471805599453
LOG2E = 1.4426950408889634
HALF_LN_2PI = 0.91893853320467274
INV_INT = [0.0] + [1.0 / j for j in range(1, 256)]  # correctly rounded 1/j


def det_erf(x):
    """erf by its Maclaurin series, term recurrence t_j = t_{j-1} * (-x^2) / j, sum t_j/(2j+1)."""
    x = np.asarray(x, np.float64)
    mx2 = -(x * x)
    term = x.copy()
    acc = x.copy()
    for j in range(1, ERF_TERMS):
        term = (term * mx2) * INV_INT[j]
        acc = acc + term * INV_INT[2 * j + 1]
    return TWO_OVER_SQRTPI * acc


def det_log(x):
    """Natural log of x > 0: frexp range reduction and the atanh series."""
    m, e = np.frexp(np.asarray(x, np.float64))
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    poly = np.full_like(s, INV_INT[23])
    for j in range(10, -1, -1):
        poly = poly * s2 + INV_INT[2 * j + 1]
    return (s * poly) * 2.0 + e * LN2


_INV_FACT = [1.0 / math.factorial(j) for j in range(17)]


def det_exp(x):
    """exp(x): n = rint(x log2 e), r = x - n ln2, degree-16 Taylor polynomial, times 2^n."""
    x = np.asarray(x, np.float64)
    n = np.rint(x * LOG2E)
    r = x - n * LN2
    poly = np.full_like(r, _INV_FACT[16])
    for j in range(15, -1, -1):
        poly = poly * r + _INV_FACT[j]
    return np.ldexp(poly, n.astype(np.int64))


_FACT_SMALL = [float(math.factorial(n)) for n in range(19)]  # exact in FP64


def det_lfact(n):
    """ln(n!) for integer n >= 0."""
    n = np.asarray(n, np.int64)
    out = np.empty(n.shape, np.float64)
    small = n <= 18
    if np.any(small):
        out[small] = det_log(np.array([_FACT_SMALL[v] for v in n[small].ravel()]).reshape(n[small].shape))
    big = ~small
    if np.any(big):
        x = n[big].astype(np.float64)
        r = 1.0 / x
        r2 = r * r
        series = r * ((1.0 / 12.0) - r2 * ((1.0 / 360.0) - r2 * ((1.0 / 1260.0) - r2 * (1.0 / 1680.0))))
        out[big] = (x + 0.5) * det_log(x) - x + HALF_LN_2PI + series
    return out


# ---------------------------------------------------------------------------
# binomial sampler
# ---------------------------------------------------------------------------
MU_SWITCH = 10.0
INVERSION_CAP = 128


def _pow_int(q, n):
    """q^n by left-to-right square-and-multiply over the bits of n (n >= 1, scalar or per element).

    Leading zero bits square 1.0, which is exact, so every element sees exactly the
    squarings and multiplications of its own bits.
    """
    n = np.broadcast_to(np.asarray(n, np.int64), q.shape)
    f = np.ones_like(q)
    for bit in range(int(n.max()).bit_length() - 1, -1, -1):
        f = f * f
        on = ((n >> bit) & 1) == 1
        f = np.where(on, f * q, f)
    return f


def _inversion(N, pp, q, u):
    f = _pow_int(q, N)
    r = pp / q
    F = f.copy()
    k = np.zeros(u.shape, np.int64)
    cap = np.minimum(N, INVERSION_CAP)
    inv = np.array(INV_INT)
    active = u >= F
    while np.any(active):
        act = active & (k < cap)
        if not np.any(act):
            break
        kk = k[act]
        fa = (f[act] * (r[act] * (N[act] - kk).astype(np.float64))) * inv[kk + 1]
        f[act] = fa
        k[act] = kk + 1
        F[act] = F[act] + fa
        active = u >= F
    return k


def _chopdown(N, pp, q, u):
    Nf = N.astype(np.float64)
    m = np.floor((Nf + 1.0) * pp).astype(np.int64)
    m = np.minimum(m, N)
    x = det_lfact(N) - det_lfact(m) - det_lfact(N - m) \
        + m.astype(np.float64) * det_log(pp) + (N - m).astype(np.float64) * det_log(q)
    Pm = det_exp(x)
    v = u - Pm
    out = m.copy()
    done = v < 0.0
    lo = m.copy()
    hi = m.copy()
    plo = Pm.copy()
    phi = Pm.copy()
    while not np.all(done):
        act = ~done
        moved = np.zeros(u.shape, bool)
        # step down while the lower side is neither at 0 nor underflowed
        s = act & (lo > 0) & (plo > 0.0)
        if np.any(s):
            lf = lo[s].astype(np.float64)
            plo[s] = plo[s] * (lf * q[s]) / ((N[s] - lo[s] + 1).astype(np.float64) * pp[s])
            lo[s] -= 1
            v[s] = v[s] - plo[s]
            moved |= s
            hit = s & (v < 0.0)
            out[hit] = lo[hit]
            done |= hit
        # then step up, same rule for the upper side
        s = act & ~done & (hi < N) & (phi > 0.0)
        if np.any(s):
            hf = hi[s].astype(np.float64)
            phi[s] = phi[s] * ((N[s] - hi[s]).astype(np.float64) * pp[s]) / ((hf + 1.0) * q[s])
            hi[s] += 1
            v[s] = v[s] - phi[s]
            moved |= s
            hit = s & (v < 0.0)
            out[hit] = hi[hit]
            done |= hit
        # both sides exhausted without reaching u: return the mode
        stuck = act & ~done & ~moved
        out[stuck] = m[stuck]
        done |= stuck
    return out


def binomial(N, p, u):
    """Counts k ~ Binomial(N, p) for arrays p, u in [0, 1) and N >= 0 (scalar or per element)."""
    p = np.asarray(p, np.float64)
    u = np.asarray(u, np.float64)
    N = np.broadcast_to(np.asarray(N, np.int64), p.shape).copy()
    k = np.zeros(p.shape, np.int64)
    pos = N > 0
    full = pos & (p >= 1.0)
    k[full] = N[full]
    live = pos & (p > 0.0) & ~full
    if not np.any(live):
        return k
    pl = p[live]
    Nl = N[live]
    flip = pl > 0.5
    pp = np.where(flip, 1.0 - pl, pl)
    q = 1.0 - pp
    mu = Nl.astype(np.float64) * pp
    ul = u[live]
    kl = np.zeros(pl.shape, np.int64)
    small = mu < MU_SWITCH
    if np.any(small):
        kl[small] = _inversion(Nl[small], pp[small], q[small], ul[small])
    if np.any(~small):
        kl[~small] = _chopdown(Nl[~small], pp[~small], q[~small], ul[~small])
    k[live] = np.where(flip, Nl - kl, kl)
    return k


def electrons(q) -> int:
    """N = floor(Q + 1/2) for Q >= 0."""
    return int(math.floor(float(q) + 0.5))


# ---------------------------------------------------------------------------
# fluctuated raster
# ---------------------------------------------------------------------------

def det_axis_probs(mu: float, sigma: float, nsigma: float, n_bins: int, keep_lo: int = 0, keep_hi: int | None = None):
    """Clipped axis integrals with det_erf: bins in [0, n_bins) and their probabilities.

    Edge values: d = edge - mu, x = d / (sigma * sqrt2), weight = 0.5*(erf(x_hi) - erf(x_lo)).
    keep_lo/keep_hi optionally restrict the bins returned (each bin's value depends only on
    its own edges, so a restricted evaluation returns the same values).
    """
    lo, hi, k0, k1 = window(mu, sigma, nsigma)
    keep_hi = n_bins if keep_hi is None else min(keep_hi, n_bins)
    ks = np.arange(max(k0, 0, keep_lo), min(k1, keep_hi), dtype=np.int64)
    if ks.size == 0:
        return ks, np.zeros(0)
    elo = np.maximum(ks.astype(np.float64), lo)
    ehi = np.minimum(ks.astype(np.float64) + 1.0, hi)
    s2 = sigma * SQRT2
    return ks, 0.5 * (det_erf((ehi - mu) / s2) - det_erf((elo - mu) / s2))


def fluct_patch(q, t, p, sigma_t, sigma_p, plane, event, depo_id, n_impacts, n_rows, n_ticks, seed,
                nsigma=3.0, box=None):
    """Counts of one depo-plane row: (rows, ticks, n[b, k]) as int64.

    box = (b_lo, b_hi, k_lo, k_hi) restricts the evaluation to those cells (same values).
    An invalid row (``raster.valid_row``) draws nothing.
    """
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
    u = cell_uniform(seed, plane, event, depo_id, rows[:, None], ticks[None, :], n_ticks)
    return rows, ticks, binomial(N, prob, u)


def raster_fluct(depos, planes, seed, nsigma=3.0, n_events=1):
    """Fluctuated grids (electron counts as float64), list over events of lists over planes."""
    grids = [[np.zeros((pl.n_impacts * pl.n_wires, pl.n_ticks)) for pl in planes] for _ in range(n_events)]
    for j in range(len(depos.q)):
        pi = int(depos.plane[j])
        ev = int(depos.event[j])
        pl = planes[pi]
        g = grids[ev][pi]
        rows, ticks, n = fluct_patch(depos.q[j], depos.t[j], depos.p[j], depos.sigma_t[j], depos.sigma_p[j],
                                     pi, ev, int(depos.depo_id[j]), pl.n_impacts, g.shape[0], g.shape[1],
                                     seed, nsigma)
        if rows.size and ticks.size:
            g[np.ix_(rows, ticks)] += n
    return grids


def raster_fluct_at(depos, plane_idx, plane, rows, ticks, seed, nsigma=3.0, event=0):
    """Fluctuated counts at selected cells of one plane (sampled checks of full-size grids).

    Evaluated for all (row, cell) pairs of the cells' bounding box at once; per element the
    operations are those of ``fluct_patch`` (pinned against the full raster in the tests).
    """
    rows = np.asarray(rows, np.int64)
    ticks = np.asarray(ticks, np.int64)
    out = np.zeros(rows.size, np.int64)
    if rows.size == 0:
        return out
    b_lo, b_hi, k_lo, k_hi = int(rows.min()), int(rows.max()) + 1, int(ticks.min()), int(ticks.max()) + 1
    sel = rows_touching(depos, plane_idx, plane, b_lo, b_hi, k_lo, k_hi, nsigma, event)
    if sel.size == 0:
        return out
    I = plane.n_impacts
    nb, nk = b_hi - b_lo, k_hi - k_lo
    # every (row, cell of the box) pair; cells outside a row's window get probability 0
    jj = np.repeat(sel, nb * nk)
    bb = np.tile(np.repeat(np.arange(b_lo, b_hi), nk), sel.size)
    kk = np.tile(np.tile(np.arange(k_lo, k_hi), nb), sel.size)
    q = depos.q[jj].astype(np.float64)
    t = depos.t[jj].astype(np.float64)
    p = depos.p[jj].astype(np.float64)
    st = depos.sigma_t[jj].astype(np.float64)
    sp = depos.sigma_p[jj].astype(np.float64)
    u = float(I) * p
    su = float(I) * sp

    def probs(mu, sigma, cell):
        half = nsigma * sigma
        lo = mu - half
        hi = mu + half
        inside = (cell >= np.floor(lo)) & (cell < np.ceil(hi)) & (cell >= 0)
        elo = np.maximum(cell.astype(np.float64), lo)
        ehi = np.minimum(cell.astype(np.float64) + 1.0, hi)
        s2 = sigma * SQRT2
        w = 0.5 * (det_erf((ehi - mu) / s2) - det_erf((elo - mu) / s2))
        return np.where(inside, w, 0.0), inside

    a, ina = probs(u, su, bb)
    b, inb = probs(t, st, kk)
    ok = ina & inb & (bb < plane.n_rows) & (kk < plane.n_ticks)
    N = np.floor(q + 0.5).astype(np.int64)
    prob = a * b
    uu = cell_uniform(seed, plane_idx, event, depos.depo_id[jj].astype(np.int64) & MASK32, bb, kk,
                      plane.n_ticks)
    cnt = np.where(ok, binomial(N, np.where(ok, prob, 0.0), uu), 0)
    box = cnt.reshape(sel.size, nb, nk).sum(axis=0)
    return box[rows - b_lo, ticks - k_lo]
