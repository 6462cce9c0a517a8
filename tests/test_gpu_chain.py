"""The whole chain on the GPU against the oracle's chain: 3D depositions -> wct_drift (Fig. 2)
-> wct_simulate with each plane's noise (Eq. 1, signal and noise terms) -> wct_digitize
(M as an ADC value, Sec. 2).

FP64 plan, mean charge (the oracle's rows and the GPU's agree to ~1e-15, so a count decided
by a rounding boundary could differ; the fluctuated and normal-mode grids are checked bit
for bit elsewhere from identical rows).  The waveform equals the oracle's drift, raster,
FFT convolution and noise to a relative L2 of 1e-12; the ADC codes equal the oracle's FP64
decision except within 1e-9 counts of a code edge.
"""
import numpy as np
import pytest
import torch

from gpu_util import rel_l2, say, to_np
from oracle import adc as OA
from oracle import convolve as OC
from oracle import drift as OD
from oracle import noise as ONZ
from oracle import raster as OR
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu


def test_drift_simulate_noise_digitize(wct):
    pts, det, prm, resp = synth.config2_points(n_depos=2000, n_tracks=4, n_ticks=1024, wires=(240, 240, 346),
                                               dtype="f64")
    plan = wct.Plan(det.planes, resp, dtype="f64")
    amps, conv = [], []
    for p in range(plan.n_planes):
        a = synth.noise_amplitude(plan.plane_info(p)["lt"], 200.0 + 50.0 * p)
        plan.set_noise(p, a)
        amps.append(a)
    seed = 41
    say("chain: drift, simulate with noise, digitize (FP64)")
    rows = plan.drift(wct.DevicePoints.from_numpy(pts, "cuda:0", torch.float64), wct.drift_params(**prm))
    wave = plan.simulate(rows, wct.opts(3.0, False, 1, seed, noise=True))
    # the oracle's chain
    r = OD.drift_rows(pts.x, pts.y, pts.z, pts.t0, pts.q, pts.sigma_l, pts.sigma_t, pts.event, pts.depo_id,
                      OD.DriftParams(**prm))
    d = synth.Depos(r["q"], r["t"], r["p"], r["sigma_t"], r["sigma_p"], r["plane"], r["event"], r["depo_id"])
    S = OR.raster(d, det.planes)[0]
    refs = []
    for k, pl in enumerate(det.planes):
        lt = plan.plane_info(k)["lt"]
        M = OC.convolve_fft(S[k], np.asarray(resp[k], np.float64), pl.n_impacts)
        M = M + ONZ.noise_waveforms(amps[k], seed, 0, k, pl.n_wires, pl.n_ticks, lt)
        refs.append(M)
        assert rel_l2(to_np(plan.wave_view(wave)[k]), M) < 1e-12, k
        g, b = 1500.0 / np.max(np.abs(M)), 2048.0
        conv.append((g, b, 4095))
        plan.set_adc(k, g, b, 4095)
    adc = plan.digitize(wave, 1).cpu().numpy().view(np.uint16).astype(np.int64)
    for k, (M, info) in enumerate(zip(refs, plan.info)):
        got = adc[info["wave_off"]: info["wave_off"] + info["n_wires"] * info["n_ticks"]].reshape(M.shape)
        g, b, c = conv[k]
        ref = OA.digitize(M, g, b, c, np.float64)
        t = M * g + b + 0.5
        near = np.abs(t - np.round(t)) < 1e-9
        assert not np.any((got != ref) & ~near), k
        assert np.count_nonzero(ref != 2048) > 1000
    plan.close()
