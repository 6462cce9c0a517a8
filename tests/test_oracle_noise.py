"""Pins of the noise oracle (oracle/noise.py; Eq. 1's additive term N, Sec. 2).

Nothing here compares the oracle with itself: the normals are checked against the
normal and exponential laws (Kolmogorov-Smirnov), the spectrum against its variance
law E|X[k]|^2 = A[k]^2 (chi-square bounds), the waveform against closed forms for
single-frequency spectra (which pin the transform's direction, normalisation, indexing
and the 1/sqrt(2) of the circular normal) and against Parseval's power.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import fluct as OF
from oracle import noise as ON


def test_normals_follow_the_normal_law():
    zc, zs = ON.noise_normals(7, 3, 1, np.arange(400)[:, None], np.arange(500)[None, :])
    zc, zs = zc.ravel(), zs.ravel()
    assert np.all(np.isfinite(zc)) and np.all(np.isfinite(zs))
    assert stats.kstest(zc, "norm").pvalue > 1e-4
    assert stats.kstest(zs, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(zc, zs)[0, 1]) < 5.0 / np.sqrt(zc.size)
    # |Z|^2 = (zc^2 + zs^2) / 2 is exponential with mean 1 (Box-Muller: -ln u1)
    assert stats.kstest((zc ** 2 + zs ** 2) / 2, "expon").pvalue > 1e-4


def test_normals_depend_on_every_key_word():
    base = ON.noise_normals(5, 2, 1, 10, np.arange(64))
    for other in (ON.noise_normals(6, 2, 1, 10, np.arange(64)), ON.noise_normals(5, 3, 1, 10, np.arange(64)),
                  ON.noise_normals(5, 2, 2, 10, np.arange(64)), ON.noise_normals(5, 2, 1, 11, np.arange(64))):
        assert not np.any(np.isclose(other[0], base[0], rtol=0, atol=0))
    # neighbouring frequencies and wires are uncorrelated
    zc, _ = ON.noise_normals(9, 0, 0, np.arange(300)[:, None], np.arange(300)[None, :])
    assert abs(np.corrcoef(zc[:, 1:].ravel(), zc[:, :-1].ravel())[0, 1]) < 5.0 / 300
    assert abs(np.corrcoef(zc[1:].ravel(), zc[:-1].ravel())[0, 1]) < 5.0 / 300


def test_noise_counters_are_apart_from_the_fluctuation_stream():
    """The noise block of (k, w, e, p) is not the fluctuation block of any cell: its last
    counter word carries bit 23, which the fluctuation's (p << 24) never sets."""
    k, w, e, p = 4, 7, 1, 2
    c3 = (p << 24) | ON.NOISE_STREAM_BIT
    assert c3 & ((1 << 24) - 1) != 0
    noise_words = OF.philox4x32_10(k, w, e, c3, 11, 0)
    fluct_words = OF.philox4x32_10(k, w, e, p << 24, 11, 0)
    assert noise_words != fluct_words


def test_dc_and_nyquist_are_real_and_variance_law():
    L = 64
    amp = np.linspace(1.0, 2.0, L // 2 + 1)
    X = ON.noise_spectrum(amp, 3, 0, 0, 20000, L)
    assert np.all(X[:, 0].imag == 0) and np.all(X[:, -1].imag == 0)
    # E|X[k]|^2 = A[k]^2: the mean over W wires of |X|^2 / A^2 is a chi-square(2W)/(2W)
    # variable (chi-square(W)/W at the two real frequencies); 5-sigma bounds
    W = X.shape[0]
    ratio = np.mean(np.abs(X) ** 2, axis=0) / amp ** 2
    assert np.all(np.abs(ratio[1:-1] - 1.0) < 5.0 / np.sqrt(W))
    assert np.all(np.abs(ratio[[0, -1]] - 1.0) < 5.0 * np.sqrt(2.0 / W))
    # the real and imaginary parts of the circular normal each carry half the power
    assert np.all(np.abs(np.mean(X[:, 1:-1].real ** 2, axis=0) / amp[1:-1] ** 2 - 0.5) < 5.0 / np.sqrt(W))


@pytest.mark.parametrize("k0", [0, 5, 32])
def test_single_frequency_closed_form(k0):
    """A = a at one frequency k0: n[t] = (2a/L) Re(Z e^{2 pi i k0 t / L}) for 0 < k0 < L/2,
    a Z / L at k0 = 0 and a Z (-1)^t / L at k0 = L/2, with Z from the normals."""
    L, a, W, nt = 64, 3.5, 6, 50
    amp = np.zeros(L // 2 + 1)
    amp[k0] = a
    n = ON.noise_waveforms(amp, 13, 2, 1, W, nt, L)
    zc, zs = ON.noise_normals(13, 2, 1, np.arange(W), k0)
    t = np.arange(nt)
    if k0 == 0:
        ref = (a * zc / L)[:, None] * np.ones(nt)[None, :]
    elif k0 == L // 2:
        ref = (a * zc / L)[:, None] * ((-1.0) ** t)[None, :]
    else:
        zr, zi = zc / np.sqrt(2.0), zs / np.sqrt(2.0)
        ph = 2.0 * np.pi * k0 * t / L
        ref = (2.0 * a / L) * (zr[:, None] * np.cos(ph)[None, :] - zi[:, None] * np.sin(ph)[None, :])
    assert np.allclose(n, ref, rtol=0, atol=1e-13 * a)


def test_power_and_zero_mean():
    L = 128
    k = np.arange(L // 2 + 1)
    amp = 10.0 * (1.0 + k) * np.exp(-k / 20.0)  # shaped, no zero
    W = 4000
    n = ON.noise_waveforms(amp, 21, 0, 2, W, L, L)
    p = np.sum(n ** 2, axis=1)
    expect = ON.expected_power(amp, L)
    # the per-wire power is a weighted sum of exponential variables: mean within 5 standard errors
    assert abs(p.mean() / expect - 1.0) < 5.0 * p.std() / expect / np.sqrt(W)
    # over a whole period a wire's time mean is its DC term X[0] / L = A[0] Z[0] / L, so the
    # mean over W wires is normal with standard deviation A[0] / (L sqrt(W))
    assert abs(n.mean()) < 5.0 * amp[0] / (L * np.sqrt(W))
