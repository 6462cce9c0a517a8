"""Oracle: the noise term N(t, x) of Eq. 1 (M = R (*) S + N).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper writes the measured waveform as the signal convolution plus an additive noise
term and notes that simulating the noise is cheaper than the signal part (Sec. 2); it
does not specify the noise model.  This module takes the reading of a stationary noise
per wire given by an amplitude spectrum, synthesised in the frequency domain:

* the noise of wire w of plane p in event e is n[t] = irfft(A * Z, L)[t] for t < N_t,
  where L is the plan's tick transform length, irfft the inverse real transform
  (n[t] = (1/L) sum over the full Hermitian spectrum, numpy's convention), A[k] >= 0
  the plane's amplitude spectrum on the F = L/2 + 1 frequencies and Z[k] a complex
  normal variate with E|Z|^2 = 1;
* Z[k] comes from one Philox4x32-10 block (Salmon et al., SC'11) keyed by the run seed
  with counter (k, w, e, (p << 24) | 2^23) -- the bit 2^23 keeps these counters apart
  from the fluctuation's, whose last word is p << 24 -- turned into two 53-bit uniforms
  u1 = 1 - ((w0 >> 6) 2^27 + (w1 >> 5)) 2^-53 (in (0, 1]) and
  u2 = ((w2 >> 6) 2^27 + (w3 >> 5)) 2^-53, and the Box-Muller transform (Box and
  Muller, 1958): r = sqrt(-2 ln u1), theta = 2 pi u2;
* for 0 < k < L/2, Z[k] = (r cos theta + i r sin theta) / sqrt(2) (a circular complex
  normal); at k = 0 and k = L/2, where the spectrum of a real signal is real,
  Z[k] = r cos theta (a real standard normal).

Then E[n] = 0 and E|X[k]|^2 = A[k]^2 with X = A * Z, and by Parseval
E sum_{t<L} n[t]^2 = (A[0]^2 + 2 sum_{0<k<L/2} A[k]^2 + A[L/2]^2) / L.  Everything is
FP64 (numpy's log, sqrt, cos, sin and FFT).
"""
from __future__ import annotations

import numpy as np

from .fluct import MASK32, philox4x32_10, uniform53

NOISE_STREAM_BIT = 1 << 23


def noise_normals(seed, event, plane, wires, ks):
    """(z_cos, z_sin): the two Box-Muller normals of (wire, frequency) pairs (broadcast)."""
    w = np.asarray(wires, np.int64)
    k = np.asarray(ks, np.int64)
    w, k = np.broadcast_arrays(w, k)
    c0 = k.astype(np.uint64)
    c1 = w.astype(np.uint64)
    c2 = np.full(c0.shape, int(event), np.uint64)
    c3 = np.full(c0.shape, (int(plane) << 24) | NOISE_STREAM_BIT, np.uint64)
    w0, w1, w2, w3 = philox4x32_10(c0, c1, c2, c3, int(seed) & MASK32, (int(seed) >> 32) & MASK32)
    u1 = 1.0 - uniform53(w0, w1)
    u2 = uniform53(w2, w3)
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    return r * np.cos(theta), r * np.sin(theta)


def noise_spectrum(amp, seed, event, plane, n_wires, L, wires=None):
    """X[w][k] = A[k] Z[k] for w < n_wires (or the listed wires), k <= L/2 (complex,
    [wires][L/2 + 1])."""
    F = L // 2 + 1
    amp = np.asarray(amp, np.float64)
    assert amp.shape == (F,), "one amplitude per frequency of the L-point transform"
    w = np.arange(n_wires) if wires is None else np.asarray(wires, np.int64)
    zc, zs = noise_normals(seed, event, plane, w[:, None], np.arange(F)[None, :])
    Z = (zc + 1j * zs) / np.sqrt(2.0)
    Z[:, 0] = zc[:, 0]
    Z[:, F - 1] = zc[:, F - 1]  # L even: frequency L/2 is real
    return amp[None, :] * Z


def noise_waveforms(amp, seed, event, plane, n_wires, n_ticks, L, wires=None):
    """Noise of every wire (or the listed wires) of one plane and event: [wires][n_ticks] (FP64)."""
    X = noise_spectrum(amp, seed, event, plane, n_wires, L, wires)
    return np.fft.irfft(X, n=L, axis=1)[:, :n_ticks]


def expected_power(amp, L):
    """E sum_{t<L} n[t]^2 of one wire's full-length noise (Parseval)."""
    a2 = np.asarray(amp, np.float64) ** 2
    return (a2[0] + 2.0 * a2[1:-1].sum() + a2[-1]) / L
