"""Pins of the ADC oracle (oracle/adc.py; Eq. 1's M as an ADC value, Sec. 2).

The codes are checked against their real-arithmetic definition away from the code edges
(exact rationals from Python's fractions), against the closed-form edges of a ramp, and
on the cases the definition fixes: the pedestal at M = 0, round-half-up at exact ties,
saturation at both ends, and non-numbers.
"""
from fractions import Fraction

import numpy as np

from oracle import adc as OA


def test_codes_equal_exact_rational_rounding():
    rng = np.random.default_rng(1)
    M = rng.normal(0.0, 300.0, 4000)
    gain, base, cmax = 0.7, 400.0, 4095
    got = OA.digitize(M, gain, base, cmax)
    for m, c in zip(M[:1500], got[:1500]):
        x = Fraction(float(m)) * Fraction(gain) + Fraction(base) + Fraction(1, 2)
        fl = x.numerator // x.denominator
        exact = min(max(fl, 0), cmax)
        # FP64 rounding can move a code only where x lies within a few ulp of an integer
        if abs(float(x - round(x))) > 1e-9:
            assert c == exact, (m, c, exact)


def test_ramp_steps_at_the_closed_form_edges():
    gain, base, cmax = 2.5, 10.0, 255
    edges = OA.code_edges(gain, base, cmax)
    # just inside each side of every edge
    lo = OA.digitize(edges - 1e-9, gain, base, cmax)
    hi = OA.digitize(edges + 1e-9, gain, base, cmax)
    k = np.arange(1, cmax + 1)
    assert np.array_equal(hi, k) and np.array_equal(lo, k - 1)
    # a fine ramp visits every code, each over an interval of width 1 / gain
    M = np.linspace(edges[0] - 1.0, edges[-1] + 1.0, 2_000_001)
    codes = OA.digitize(M, gain, base, cmax)
    assert np.all(np.diff(codes) >= 0)
    counts = np.bincount(codes, minlength=cmax + 1)[1:cmax]
    width = (M[1] - M[0]) * counts
    assert np.allclose(width, 1.0 / gain, atol=2 * (M[1] - M[0]))


def test_pedestal_ties_saturation_and_nan():
    assert OA.digitize(0.0, 1.3, 400.0, 4095) == 400
    assert OA.digitize(0.0, 1.3, 400.4, 4095) == 400 and OA.digitize(0.0, 1.3, 400.5, 4095) == 401
    # M g + b = k + 1/2 exactly rounds up (floor of x + 1/2)
    assert OA.digitize(2.5, 1.0, 0.0, 4095) == 3 and OA.digitize(-0.5, 1.0, 0.0, 4095) == 0
    assert OA.digitize(1e9, 1.0, 0.0, 4095) == 4095 and OA.digitize(-1e9, 1.0, 0.0, 4095) == 0
    assert OA.digitize(np.nan, 1.0, 100.0, 4095) == 0
    assert OA.digitize(np.inf, 1.0, 100.0, 4095) == 4095 and OA.digitize(-np.inf, 1.0, 100.0, 4095) == 0


def test_float32_decision_is_the_float32_arithmetic():
    """In FP32 each step rounds to single precision: the code of the rounded sum."""
    rng = np.random.default_rng(2)
    M = rng.normal(0.0, 1000.0, 10000).astype(np.float32)
    g, b = np.float32(0.37), np.float32(512.25)
    t = (M * g).astype(np.float32)
    t = (t + b).astype(np.float32)
    t = (t + np.float32(0.5)).astype(np.float32)
    ref = np.clip(np.floor(t.astype(np.float64)), 0, 4095)
    assert np.array_equal(OA.digitize(M, float(g), float(b), 4095, np.float32), ref)
