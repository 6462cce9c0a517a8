"""ADC digitisation on the GPU (wct_digitize; Eq. 1's M as an ADC value, Sec. 2).

* The codes are the plan dtype's arithmetic: for every sample, floor(M g + b + 1/2) with
  one rounding per operation, clamped to [0, max_code], 0 for a non-number; checked bit
  for bit on seeded waveforms written on the host (FP32 and FP64, two events, distinct
  converters per plane, a plane whose sample count is odd so the element path runs, values
  on code edges and half-code ties) and on planted special values (saturation,
  infinities, NaN).
* Against the oracle (its FP64 M, digitised in FP32 as the FP32 plan does): every code
  equal except where the oracle's unrounded code lies within the FP32 waveform's error
  of a code edge, and there within one count.
"""
import numpy as np
import pytest
import torch

from gpu_util import device_depos, make_plan, say, to_np
from oracle import adc as OA
from oracle import convolve as OC
from oracle import raster as OR
from paper_2104_08265_amd import synth
from test_gpu_parity import slice_workload

pytestmark = pytest.mark.gpu

CONVERTERS = [(0.9, 400.0, 4095), (2.3, 2048.0, 4095), (0.35, 900.0, 16383)]


def expected_codes(M, gain, base, cmax, dtype):
    """The plan dtype's arithmetic written out with numpy scalars of that type."""
    dt = np.dtype(dtype).type
    t = M.astype(dt) * dt(gain)
    t = t + dt(base)
    t = t + dt(0.5)
    x = np.floor(t)
    with np.errstate(invalid="ignore"):
        return np.where(x >= 0, np.minimum(x, cmax), 0).astype(np.int64)


def codes_np(plan, adc, n_events):
    a = adc.cpu().numpy().view(np.uint16).astype(np.int64)
    out = []
    for e in range(n_events):
        base = e * plan.wave_elems
        out.append([a[base + i["wave_off"]: base + i["wave_off"] + i["n_wires"] * i["n_ticks"]]
                    .reshape(i["n_wires"], i["n_ticks"]) for i in plan.info])
    return out


@pytest.mark.parametrize("dtype,n_ticks", [("f32", 960), ("f32", 961), ("f64", 961)])
def test_codes_are_the_dtype_arithmetic(wct, dtype, n_ticks):
    """Seeded waveforms written on the host (two events, three planes with distinct
    converters; 960 ticks: the 4-sample vector path, 961: odd plane sizes, the element
    path), with values placed on code edges, on half-code ties and past both ends."""
    wl = synth.config2(n_depos=10, n_tracks=1, n_ticks=n_ticks, wires=(240, 240, 347), dtype=dtype)
    plan = make_plan(wct, wl, max_events=2)
    for p, (g, b, c) in enumerate(CONVERTERS):
        plan.set_adc(p, g, b, c)
    npdt = np.float32 if dtype == "f32" else np.float64
    rng = np.random.default_rng(12)
    host = np.empty(2 * plan.wave_elems, npdt)
    for e in range(2):
        for p, i in enumerate(plan.info):
            g, b, c = CONVERTERS[p]
            n = i["n_wires"] * i["n_ticks"]
            v = rng.normal(0.0, 0.25 * c / g, n)                      # most of the code range
            pick = rng.random(n)
            k = rng.integers(-50, c + 50, n).astype(np.float64)
            v = np.where(pick < 0.1, (k - b) / g, v)                  # on code edges
            v = np.where((pick >= 0.1) & (pick < 0.2), (k - b + 0.5) / g, v)  # half-code ties
            v = np.where(pick > 0.995, rng.choice([1e30, -1e30], n), v)        # far past the ends
            off = e * plan.wave_elems + i["wave_off"]
            host[off: off + n] = v.astype(npdt)
    wave = torch.as_tensor(host).to("cuda:0")
    say("digitize", dtype, n_ticks)
    adc = plan.digitize(wave, 2)
    torch.cuda.synchronize()
    got = codes_np(plan, adc, 2)
    for e in range(2):
        for p, i in enumerate(plan.info):
            off = e * plan.wave_elems + i["wave_off"]
            M = host[off: off + i["n_wires"] * i["n_ticks"]].reshape(i["n_wires"], i["n_ticks"])
            ref = expected_codes(M, *CONVERTERS[p], npdt)
            assert np.array_equal(got[e][p], ref), (e, p, int(np.sum(got[e][p] != ref)))
            assert 0 < np.count_nonzero(ref == CONVERTERS[p][2]) and 0 < np.count_nonzero(ref == 0)
    plan.close()


def test_special_values(wct):
    wl = synth.config1(n_depos=10, n_wires=8, n_ticks=64)
    plan = make_plan(wct, wl)
    plan.set_adc(0, 1.0, 0.0, 4095)
    vals = np.array([0.0, 2.5, -0.5, 3.4999, 1e9, -1e9, np.inf, -np.inf, np.nan, 4094.5, 4095.6, -0.4999],
                    np.float64)
    w = np.zeros(plan.wave_elems)
    w[:vals.size] = vals
    wave = torch.as_tensor(w).to("cuda:0")
    got = plan.digitize(wave, 1).cpu().numpy().view(np.uint16)[:vals.size].astype(np.int64)
    assert got.tolist() == [0, 3, 0, 3, 4095, 0, 4095, 0, 0, 4095, 4095, 0]
    plan.close()


def test_codes_against_the_oracle(wct):
    wl = slice_workload()
    S = OR.raster(wl.depos, wl.planes)[0]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    Ms = [OC.convolve_fft(S[p], R[p], pl.n_impacts) for p, pl in enumerate(wl.planes)]
    plan = make_plan(wct, wl)
    # converters spanning about +-1500 counts around the pedestal over each plane's range
    conv = [(1500.0 / np.max(np.abs(M)), 2048.0, 4095) for M in Ms]
    for p, (g, b, c) in enumerate(conv):
        plan.set_adc(p, g, b, c)
    say("digitize vs oracle")
    wave = plan.simulate(device_depos(wct, wl), wct.opts(3.0, False, 1, wl.seed))
    got = codes_np(plan, plan.digitize(wave, 1), 1)[0]
    near_total = 0
    for p, (M, w) in enumerate(zip(Ms, plan.wave_view(wave))):
        g, b, c = conv[p]
        peak = np.max(np.abs(M))
        # the FP32 waveform's per-sample error, bounded at 1e-5 of the plane's peak
        assert np.max(np.abs(to_np(w) - M)) < 1e-5 * peak, p
        ref = OA.digitize(M, g, b, c, np.float32)
        t = M * g + b + 0.5
        near = np.abs(t - np.round(t)) < g * 1e-5 * peak + 1e-3  # + FP32 rounding of t near 2048
        diff = got[p] != ref
        assert not np.any(diff & ~near), (p, int(np.sum(diff & ~near)))
        assert np.all(np.abs(got[p] - ref) <= 1)
        near_total += int(near.sum())
        assert np.count_nonzero(ref != 2048) > 1000
    assert near_total < 0.05 * sum(pl.n_wires * pl.n_ticks for pl in wl.planes)
    plan.close()


def test_adc_arguments_refused(wct):
    wl = synth.config1(n_depos=10, n_wires=8, n_ticks=64)
    plan = make_plan(wct, wl)
    for args in ((1, 1.0, 0.0, 4095), (0, np.nan, 0.0, 4095), (0, 1.0, np.inf, 4095), (0, 1.0, 0.0, 0),
                 (0, 1.0, 0.0, 65536)):
        with pytest.raises(wct.WctError):
            plan.set_adc(*args)
    plan.close()
