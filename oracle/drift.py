"""Oracle: drift, diffusion, attenuation and projection of ionisation clouds onto the wire
planes (Fig. 2: clouds drift to the readout, spread along and across the drift, and
overlap there; Sec. 2.1.1: the rasteriser takes each cloud's Gaussian at the plane).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper shows the step but gives no formulas.  This module takes the standard reading
of a uniform drift field along -x towards readout planes at x = 0:

* drift time t_d = x / v (v the drift speed); a deposition with x < 0, or with a value
  that is not finite, is not drifted: its rows carry charge 0;
* diffusion adds variance 2 D t_d along (D_L) and across (D_T) the drift:
  sigma_L^2 = sigma_L0^2 + 2 D_L t_d, sigma_T^2 = sigma_T0^2 + 2 D_T t_d;
* attachment with electron lifetime tau leaves Q = q exp(-t_d / tau) (tau <= 0: none);
* plane k with wire-normal angle theta_k, pitch P_k, offset o_k (the pitch coordinate of
  y = z = 0) and time offset d_k receives the row
      p = (z cos theta_k + y sin theta_k) / P_k + o_k      (pitches),
      sigma_p = sigma_T / P_k,
      t = (t0 + t_d + d_k) / T_tick                          (ticks),
      sigma_t = sigma_L / (v T_tick),
  with the plane index k, the deposition's event and id; rows are plane-major (row
  k n + j for deposition j of n).

Everything is FP64 (numpy's exp, sqrt, cos and sin).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class DriftParams:
    drift_speed: float      # cm / us
    diffusion_l: float      # cm^2 / us
    diffusion_t: float      # cm^2 / us
    lifetime: float         # us; <= 0: no attenuation
    tick: float             # us per tick
    angles: tuple           # per plane: wire-normal angle theta (radians)
    pitches: tuple          # per plane: wire pitch (cm)
    wire_offsets: tuple     # per plane: pitch coordinate of y = z = 0 (pitches)
    time_offsets: tuple     # per plane: time added at the plane (us)


def drift_rows(x, y, z, t0, q, sigma_l0, sigma_t0, event, depo_id, prm: DriftParams):
    """Rows (q, t, p, sigma_t, sigma_p, plane, event, depo_id) of every (plane, deposition)."""
    x, y, z, t0, q, sl0, st0 = (np.asarray(a, np.float64) for a in (x, y, z, t0, q, sigma_l0, sigma_t0))
    n = x.size
    ok = (x >= 0) & np.isfinite(x) & np.isfinite(y) & np.isfinite(z) & np.isfinite(t0) & np.isfinite(q) \
        & np.isfinite(sl0) & np.isfinite(st0)
    td = np.where(ok, x, 0.0) / prm.drift_speed
    sl = np.sqrt(sl0 * sl0 + 2.0 * prm.diffusion_l * td)
    st = np.sqrt(st0 * st0 + 2.0 * prm.diffusion_t * td)
    Q = q * np.exp(-td / prm.lifetime) if prm.lifetime > 0 else q.copy()
    Q = np.where(ok, Q, 0.0)
    out = {k: [] for k in ("q", "t", "p", "sigma_t", "sigma_p", "plane", "event", "depo_id")}
    for k, (th, P, off, dk) in enumerate(zip(prm.angles, prm.pitches, prm.wire_offsets, prm.time_offsets)):
        out["q"].append(Q)
        out["t"].append((t0 + td + dk) / prm.tick)
        with np.errstate(invalid="ignore"):  # infinite coordinates (rows without charge)
            out["p"].append((z * np.cos(th) + y * np.sin(th)) / P + off)
        out["sigma_t"].append(sl / (prm.drift_speed * prm.tick))
        out["sigma_p"].append(st / P)
        out["plane"].append(np.full(n, k, np.int32))
        out["event"].append(np.asarray(event, np.int32))
        out["depo_id"].append(np.asarray(depo_id, np.int32))
    return {k: np.concatenate(v) for k, v in out.items()}
