"""Oracle: per-deposition gradients of the simulated waveform (differentiable mode).

The paper computes the forward signal only (Eq. 1, Eq. 2).  Differentiation is a
reading added on top of it: for a loss L(M), with G = dL/dM,

* the convolution's adjoint H = dL/dS = R^T G (``convolve.adjoint_fft``);
* the raster is S = sum_j Q_j A_j (x) B_j (``raster.patch``), so for row j
      dL/dQ       = sum_{b,k} H[b,k] A_b B_k
      dL/dt       = Q sum H A_b dB_k/dt,        dL/dsigma_t = Q sum H A_b dB_k/dsigma_t
      dL/dp       = Q sum H dA_b/dp B_k,        dL/dsigma_p = Q sum H dA_b/dsigma_p B_k
  with, per axis (time shown; pitch uses u = I p, sigma_u = I sigma_p and the chain rule
  d/dp = I d/du, d/dsigma_p = I d/dsigma_u):
      dB_k/dt     = -(1/sigma) [phi(z_hi)(1-c_hi) - phi(z_lo)(1-c_lo)]
      dB_k/dsigma = -(1/sigma) [z_hi phi(z_hi)(1-c_hi) - z_lo phi(z_lo)(1-c_lo)]
  where z = (edge - t)/sigma, phi is the standard normal pdf and c flags an edge clipped
  to the truncation window (such an edge sits at z = +-nsigma and does not move).

Fluctuation is off in this mode.  Everything is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .raster import valid_row, window

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def axis_weights_and_derivs(mu, sigma, nsigma, n_bins):
    """(bins, w, dw/dmu, dw/dsigma) for the clipped bins inside [0, n_bins)."""
    lo, hi, k0, k1 = window(mu, sigma, nsigma)
    ks = np.arange(k0, k1, dtype=np.int64)
    kf = ks.astype(np.float64)
    c_lo = kf < lo  # lower edge clipped to the window
    c_hi = kf + 1.0 > hi
    elo = np.where(c_lo, lo, kf)
    ehi = np.where(c_hi, hi, kf + 1.0)
    zlo = (elo - mu) / sigma
    zhi = (ehi - mu) / sigma
    w = 0.5 * (erf(zhi / SQRT2) - erf(zlo / SQRT2))
    plo = INV_SQRT_2PI * np.exp(-0.5 * zlo * zlo) * (~c_lo)
    phi = INV_SQRT_2PI * np.exp(-0.5 * zhi * zhi) * (~c_hi)
    dmu = -(phi - plo) / sigma
    dsig = -(zhi * phi - zlo * plo) / sigma
    keep = (ks >= 0) & (ks < n_bins)
    return ks[keep], w[keep], dmu[keep], dsig[keep]


def row_gradients(H, q, t, p, sigma_t, sigma_p, n_impacts, nsigma=3.0):
    """(g_q, g_t, g_p, g_sigma_t, g_sigma_p) of one depo-plane row given H = dL/dS of its plane.

    An invalid row (``raster.valid_row``) contributes nothing to S, so all five are 0.
    """
    q, t, p, st, sp = (float(v) for v in (q, t, p, sigma_t, sigma_p))
    if not valid_row(q, t, p, st, sp):
        return 0.0, 0.0, 0.0, 0.0, 0.0
    I = n_impacts
    rows, a, da_du, da_dsu = axis_weights_and_derivs(I * p, I * sp, nsigma, H.shape[0])
    ticks, b, db_dt, db_dst = axis_weights_and_derivs(t, st, nsigma, H.shape[1])
    if rows.size == 0 or ticks.size == 0:
        return 0.0, 0.0, 0.0, 0.0, 0.0
    h = H[np.ix_(rows, ticks)]
    r0 = h @ b
    r1 = h @ db_dt
    r2 = h @ db_dst
    g_q = float(a @ r0)
    g_t = q * float(a @ r1)
    g_st = q * float(a @ r2)
    g_p = q * I * float(da_du @ r0)
    g_sp = q * I * float(da_dsu @ r0)
    return g_q, g_t, g_p, g_st, g_sp


def gradients(Hs, depos, planes, nsigma=3.0):
    """Per-row gradients; Hs[event][plane] = dL/dS.  Returns an array [n_rows, 5]
    with columns (q, t, p, sigma_t, sigma_p)."""
    out = np.zeros((len(depos.q), 5))
    for j in range(len(depos.q)):
        pi = int(depos.plane[j])
        out[j] = row_gradients(Hs[int(depos.event[j])][pi], depos.q[j], depos.t[j], depos.p[j],
                               depos.sigma_t[j], depos.sigma_p[j], planes[pi].n_impacts, nsigma)
    return out


def edge_distance(mu, sigma, nsigma):
    """Distance of the nearer truncation edge to an integer bin boundary (kink detector)."""
    lo, hi, _, _ = window(mu, sigma, nsigma)
    return min(abs(lo - round(lo)), abs(hi - round(hi)))
