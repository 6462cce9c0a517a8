"""Oracle: ADC digitisation of the measured waveform M (Eq. 1; Sec. 2 calls M a
measurement such as an analog-to-digital converter value).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the ADC value as what M represents but gives no converter model.  This
module takes the reading of a linear converter per plane with a gain g (counts per unit
of M), a pedestal b (counts) and a largest code c_max (2^bits - 1):

    code = min(max(floor(M g + b + 1/2), 0), c_max),

a value that is not a number giving code 0.  The arithmetic is carried out in a stated
floating-point type, one rounding per operation in the order written (M g, then + b,
then + 1/2), so that a code decided in that type is defined bit for bit.
"""
from __future__ import annotations

import numpy as np


def digitize(M, gain, baseline, max_code, dtype=np.float64):
    """ADC codes (int64) of the waveform M, computed in `dtype` (np.float32 or np.float64)."""
    dt = np.dtype(dtype).type
    m = np.asarray(M).astype(dt)
    t = m * dt(gain)
    t = t + dt(baseline)
    t = t + dt(0.5)
    x = np.floor(t)
    with np.errstate(invalid="ignore"):
        code = np.where(x >= 0, np.where(x <= max_code, x, max_code), 0)
    return code.astype(np.int64)


def code_edges(gain, baseline, max_code):
    """The M at which the exact (real-arithmetic) code steps from k - 1 to k, k = 1..c_max."""
    k = np.arange(1, int(max_code) + 1, dtype=np.float64)
    return (k - 0.5 - baseline) / gain
