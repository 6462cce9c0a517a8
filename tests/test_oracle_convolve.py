"""Pins for the oracle's convolution (Eq. 1 signal term; Eq. 2 frequency-domain evaluation)."""
import numpy as np
import pytest

from oracle import convolve as C
from oracle import raster as RS
from paper_2104_08265_amd import synth

I = 10


def rand_grid(rng, nw, nt, density=0.3):
    S = rng.standard_normal((I * nw, nt))
    S[rng.uniform(size=S.shape) > density] = 0.0
    return S


def rand_resp(rng, K, T):
    return rng.standard_normal((2 * K + 1, I, T))


def test_point_charge_places_response_by_its_definition():
    """Unit charge at impact row I*c0+i0, tick t0 gives M[w, t] = R[k=c0-w, i0, t-t0].

    This pins the index convention of R (response of wire w to charge in impact row
    I*(w+k)+i, tau ticks later) independently of how the sum is organised.
    """
    rng = np.random.default_rng(1)
    nw, nt, K, T = 9, 30, 3, 7
    R = rand_resp(rng, K, T)
    c0, i0, t0 = 4, 7, 11
    S = np.zeros((I * nw, nt))
    S[I * c0 + i0, t0] = 1.0
    expect = np.zeros((nw, nt))
    for w in range(nw):
        k = c0 - w
        if -K <= k <= K:
            expect[w, t0:t0 + T] = R[k + K, i0, :]
    for M in (C.convolve_direct(S, R, I), C.convolve_fft(S, R, I)):
        assert np.allclose(M, expect, rtol=0, atol=1e-13)


def test_direct_equals_fft_tiny():
    rng = np.random.default_rng(2)
    for nw, nt, K, T in [(6, 40, 2, 12), (5, 17, 3, 9), (1, 8, 0, 3)]:
        S = rand_grid(rng, nw, nt)
        R = rand_resp(rng, K, T)
        Md = C.convolve_direct(S, R, I)
        Mf = C.convolve_fft(S, R, I)
        assert np.linalg.norm(Md - Mf) <= 1e-12 * np.linalg.norm(Md)


def test_padding_invariance():
    rng = np.random.default_rng(3)
    S = rand_grid(rng, 12, 60)
    R = rand_resp(rng, 3, 15)
    a = C.convolve_fft(S, R, I)
    b = C.convolve_fft(S, R, I, lw=15, lt=74)  # minimal lengths N_w+K, N_t+T-1
    c = C.convolve_fft(S, R, I, lw=45, lt=100)  # non-power-of-two
    assert np.allclose(a, b, rtol=0, atol=1e-11)
    assert np.allclose(a, c, rtol=0, atol=1e-11)


def test_delta_responses():
    rng = np.random.default_rng(4)
    nw, nt, K, T = 7, 25, 2, 5
    S = rand_grid(rng, nw, nt)
    R = np.zeros((2 * K + 1, I, T))
    R[K, :, 0] = 1.0  # k=0, tau=0, every phase
    M = C.convolve_fft(S, R, I)
    assert np.allclose(M, S.reshape(nw, I, nt).sum(axis=1), rtol=0, atol=1e-13)
    R = np.zeros((2 * K + 1, I, T))
    R[K, 3, 0] = 1.0
    M = C.convolve_fft(S, R, I)
    assert np.allclose(M, S[3::I], rtol=0, atol=1e-13)


@pytest.mark.parametrize("k0,tau0", [(1, 0), (-2, 3), (2, 4)])
def test_shift_response(k0, tau0):
    rng = np.random.default_rng(5)
    nw, nt, K, T = 7, 25, 2, 5
    S = rand_grid(rng, nw, nt)
    R = np.zeros((2 * K + 1, I, T))
    R[k0 + K, :, tau0] = 1.0
    M = C.convolve_fft(S, R, I)
    wire_sum = S.reshape(nw, I, nt).sum(axis=1)
    expect = np.zeros((nw, nt))
    for w in range(nw):
        c = w + k0
        if 0 <= c < nw:
            expect[w, tau0:] = wire_sum[c, : nt - tau0]
    assert np.allclose(M, expect, rtol=0, atol=1e-13)


def test_linearity_in_charge():
    wl = synth.tiny(n_wires=6, n_ticks=40, n_depos=8, seed=11)
    d = wl.depos
    S = RS.raster(d, wl.planes)[0][0]
    d2 = d.astype(np.float64)
    d2.q = 3.0 * d2.q
    S2 = RS.raster(d2, wl.planes)[0][0]
    R = wl.responses[0]
    assert np.allclose(C.convolve_fft(S2, R, I), 3.0 * C.convolve_fft(S, R, I), rtol=1e-12, atol=1e-10)


def test_translation():
    """Moving every depo by +1 pitch and +1 tick shifts M by one wire and one tick (away from edges)."""
    wl = synth.tiny(n_wires=12, n_ticks=60, half_wires=2, resp_ticks=8, n_depos=6, seed=12)
    d = wl.depos
    keep = (d.p > 3) & (d.p < 7) & (d.t > 15) & (d.t < 35)
    d = d.select(keep)
    assert len(d) > 0
    S = RS.raster(d, wl.planes)[0][0]
    d2 = d.astype(np.float64)
    d2.p = d2.p + 1.0
    d2.t = d2.t + 1.0
    S2 = RS.raster(d2, wl.planes)[0][0]
    R = wl.responses[0]
    M = C.convolve_fft(S, R, I)
    M2 = C.convolve_fft(S2, R, I)
    assert np.allclose(M2[1:, 1:], M[:-1, :-1], rtol=0, atol=1e-10 * np.abs(M).max())


def test_induction_sum_rule():
    """Zero-sum bipolar responses give zero time-integrated signal when the signal fits the window."""
    wl = synth.tiny(n_wires=10, n_ticks=80, half_wires=2, resp_ticks=20, n_depos=5, seed=13, kind="induction")
    R = wl.responses[0]
    assert np.allclose(R.sum(axis=2), 0.0, atol=1e-12)
    d = wl.depos.select((wl.depos.t > 10) & (wl.depos.t < 40))
    S = RS.raster(d, wl.planes)[0][0]
    M = C.convolve_fft(S, R, I)
    assert np.abs(M.sum(axis=1)).max() < 1e-10 * np.abs(M).max() * M.shape[1]


def test_adjoint_identity_and_forms():
    rng = np.random.default_rng(6)
    nw, nt, K, T = 6, 30, 2, 9
    S = rand_grid(rng, nw, nt)
    G = rng.standard_normal((nw, nt))
    R = rand_resp(rng, K, T)
    Hd = C.adjoint_direct(G, R, I)
    Hf = C.adjoint_fft(G, R, I)
    assert np.linalg.norm(Hd - Hf) <= 1e-12 * np.linalg.norm(Hd)
    lhs = float(np.sum(C.convolve_direct(S, R, I) * G))
    rhs = float(np.sum(S * Hd))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_convolve_at_samples():
    rng = np.random.default_rng(7)
    nw, nt, K, T = 8, 40, 2, 9
    S = rand_grid(rng, nw, nt)
    R = rand_resp(rng, K, T)
    M = C.convolve_direct(S, R, I)
    rows = lambda b: S[b] if 0 <= b < S.shape[0] else None
    for w, t in [(0, 0), (3, 17), (7, 39), (5, 8)]:
        assert abs(C.convolve_at(rows, R, I, w, t) - M[w, t]) < 1e-12
