"""Oracle: the signal term of Eq. 1, M = R (*) S, by definition and by FFT (Eq. 2).

Discretisation (the paper states Eq. 1 only in continuous (t, x)): the grid S has
N_b = I*N_w impact rows by N_t ticks; R[k][i][tau] (k = -K..K stored at k+K, i in
[0, I), tau in [0, T_R)) is the response of wire w to unit charge in impact row
I*(w+k)+i arriving tau ticks earlier.  Then, for w in [0, N_w), t in [0, N_t):

    M[w, t] = sum_{k, i, tau} R[k, i, tau] * S[I*(w+k)+i, t-tau]

with S = 0 outside the grid: the convolution is linear (not circular), causal in
time, a correlation in the wire index, and the output window is the grid's own.
The sum over i (the impact phase) is the impact-to-wire reduction.

``convolve_direct`` writes this sum out (brute force, tiny grids only).
``convolve_fft`` evaluates it as Eq. 2 does: transform S, multiply by the
pre-computed response spectrum, transform back.  It zero-pads to powers of two
(>= N_w + 2K, >= N_t + T_R), deliberately not the lengths the GPU path uses, so that
agreement also shows padding invariance.  Transforms are numpy's FP64 FFTs.
"""
from __future__ import annotations

import numpy as np


def _next_pow2(n: int) -> int:
    return 1 << (int(n) - 1).bit_length()


def convolve_direct(S: np.ndarray, R: np.ndarray, n_impacts: int) -> np.ndarray:
    """Brute-force discrete Eq. 1 (signal part)."""
    I = n_impacts
    nb, nt = S.shape
    nw = nb // I
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    M = np.zeros((nw, nt))
    for w in range(nw):
        for k in range(-K, K + 1):
            for i in range(I):
                b = I * (w + k) + i
                if b < 0 or b >= nb:
                    continue
                row = S[b]
                for tau in range(T):
                    if tau >= nt:
                        break
                    M[w, tau:] += R[k + K, i, tau] * row[: nt - tau]
    return M


def response_kernel(R: np.ndarray, n_impacts: int, lw: int, lt: int) -> np.ndarray:
    """Per-phase 2D kernels on an (lw x lt) torus: Kr_i[(-k) mod lw, tau] = R[k, i, tau].

    With this placement the circular convolution (Kr_i (*) S_i)[w, t] equals
    sum_{k,tau} R[k,i,tau] S_i[w+k, t-tau], i.e. the correlation in the wire index.
    """
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    ker = np.zeros((n_impacts, lw, lt))
    for k in range(-K, K + 1):
        ker[:, (-k) % lw, :T] = R[k + K]
    return ker


def convolve_fft(S: np.ndarray, R: np.ndarray, n_impacts: int, lw: int | None = None,
                 lt: int | None = None) -> np.ndarray:
    """Eq. 2: FT(S) x pre-calculated R(omega) -> inverse FT, per impact phase, summed."""
    I = n_impacts
    nb, nt = S.shape
    nw = nb // I
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    lw = lw or _next_pow2(nw + 2 * K)
    lt = lt or _next_pow2(nt + T)
    assert lw >= nw + K and lt >= nt + T - 1, "padding too short for a linear convolution"
    ker = response_kernel(R, I, lw, lt)
    acc = np.zeros((lw, lt // 2 + 1), dtype=np.complex128)
    for i in range(I):
        Si = np.zeros((lw, lt))
        Si[:nw, :nt] = S[i::I][:nw]
        acc += np.fft.rfft2(Si) * np.fft.rfft2(ker[i])
    return np.fft.irfft2(acc, s=(lw, lt))[:nw, :nt]


def adjoint_direct(G: np.ndarray, R: np.ndarray, n_impacts: int) -> np.ndarray:
    """Adjoint of convolve_direct: H[I*c+i, t'] = sum_{k,tau} R[k,i,tau] G[c-k, t'+tau].

    G is zero outside [0, N_w) x [0, N_t).  <convolve(S), G> = <S, adjoint(G)>.
    """
    I = n_impacts
    nw, nt = G.shape
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    H = np.zeros((I * nw, nt))
    for c in range(nw):
        for k in range(-K, K + 1):
            w = c - k
            if w < 0 or w >= nw:
                continue
            for i in range(I):
                for tau in range(T):
                    if tau >= nt:
                        break
                    H[I * c + i, : nt - tau] += R[k + K, i, tau] * G[w, tau:]
    return H


def adjoint_fft(G: np.ndarray, R: np.ndarray, n_impacts: int, lw: int | None = None,
                lt: int | None = None) -> np.ndarray:
    """Adjoint by FFT: per phase, correlate G with the phase kernel (conjugate spectrum)."""
    I = n_impacts
    nw, nt = G.shape
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    lw = lw or _next_pow2(nw + 2 * K)
    lt = lt or _next_pow2(nt + T)
    ker = response_kernel(R, I, lw, lt)
    Gp = np.zeros((lw, lt))
    Gp[:nw, :nt] = G
    Gf = np.fft.rfft2(Gp)
    H = np.zeros((I * nw, nt))
    for i in range(I):
        Hi = np.fft.irfft2(Gf * np.conj(np.fft.rfft2(ker[i])), s=(lw, lt))
        H[i::I] = Hi[:nw, :nt]
    return H


def convolve_at(S_rows, R: np.ndarray, n_impacts: int, w: int, t: int) -> float:
    """One output sample M[w, t] by the definition; S_rows(b) returns row b (or None)."""
    I = n_impacts
    K = (R.shape[0] - 1) // 2
    T = R.shape[2]
    acc = 0.0
    for k in range(-K, K + 1):
        for i in range(I):
            row = S_rows(I * (w + k) + i)
            if row is None:
                continue
            lo = max(0, t - (T - 1))
            seg = row[lo: t + 1][::-1]  # S[b, t - tau] for tau = 0 .. len-1
            acc += float(np.dot(R[k + K, i, : seg.size], seg))
    return acc
