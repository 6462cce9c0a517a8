"""The noise term of Eq. 1 (M = R (*) S + N) on the GPU against the oracle (oracle/noise.py).

wct_simulate with opts.noise adds each plane's noise in the frequency domain just before
the inverse row transform.  Checked against the oracle's FP64 noise (relative L2 1e-5 in
FP32, 1e-12 in FP64):
* noise alone (no depositions), three planes, with the compiled and the runtime inverse
  row transform;
* signal plus noise (fluctuated raster);
* a batch of events in sub-batches: each event's waveform equals its one-event call bit
  for bit and the oracle's noise of that event id;
* full three-plane geometry (9600 ticks): sampled wires;
* noise off leaves the waveform unchanged; bad spectra are refused.
"""
import numpy as np
import pytest

from gpu_util import device_depos, make_plan, rel_l2, say, to_np
from oracle import convolve as OC
from oracle import fluct as OF
from oracle import noise as ON
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu
TOL32, TOL64 = 1e-5, 1e-12
RMS = (250.0, 300.0, 180.0)


def set_noise(plan, wl):
    amps = []
    for p in range(plan.n_planes):
        lt = plan.plane_info(p)["lt"]
        a = synth.noise_amplitude(lt, RMS[p % 3], shaping_ticks=1.5 + p)
        plan.set_noise(p, a)
        amps.append(a)
    return amps


def oracle_noise(plan, wl, amps, seed, event):
    out = []
    for p, pl in enumerate(wl.planes):
        lt = plan.plane_info(p)["lt"]
        out.append(ON.noise_waveforms(amps[p], seed, event, p, pl.n_wires, pl.n_ticks, lt))
    return out


def empty_depos(wct, wl):
    return device_depos(wct, wl, wl.depos.select(np.zeros(len(wl.depos), bool)))


def test_noise_alone_fp32_compiled_and_runtime(wct):
    wl = synth.config2(n_depos=10, n_ticks=1024, wires=(240, 240, 346))  # L_t = 1250: compiled tick plans exist
    plan = make_plan(wct, wl)
    amps = set_noise(plan, wl)
    ref = oracle_noise(plan, wl, amps, 77, 0)
    for choice in plan.fft_candidates(0, 0):
        for p in range(plan.n_planes):
            plan.set_fft(p, 0, choice)
        say("noise alone, tick plan", choice)
        w = plan.simulate(empty_depos(wct, wl), wct.opts(3.0, True, 1, 77, noise=True))
        for k, wv in enumerate(plan.wave_view(w)):
            assert rel_l2(to_np(wv), ref[k]) < TOL32, (choice, k)
    plan.close()


def test_noise_alone_fp64(wct):
    wl = synth.config1(n_depos=10)
    plan = make_plan(wct, wl)
    amps = set_noise(plan, wl)
    ref = oracle_noise(plan, wl, amps, 5, 0)
    for choice in plan.fft_candidates(0, 0):
        plan.set_fft(0, 0, choice)
        say("noise alone fp64, tick plan", choice)
        w = plan.simulate(empty_depos(wct, wl), wct.opts(3.0, False, 1, 5, noise=True))
        assert rel_l2(to_np(plan.wave_view(w)[0]), ref[0]) < TOL64, choice
    plan.close()


def test_signal_plus_noise(wct):
    wl = synth.config2(n_depos=2000, n_tracks=5, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    plan = make_plan(wct, wl)
    amps = set_noise(plan, wl)
    say("signal + noise, fluctuated raster of 2000 depositions")
    w = plan.simulate(device_depos(wct, wl), wct.opts(3.0, True, 1, wl.seed, noise=True))
    grids = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    noise = oracle_noise(plan, wl, amps, wl.seed, 0)
    for k, wv in enumerate(plan.wave_view(w)):
        ref = OC.convolve_fft(grids[k], R[k], wl.planes[k].n_impacts) + noise[k]
        assert rel_l2(to_np(wv), ref) < TOL32, k
    # noise off: the plain simulation, bit for bit, even with spectra set
    w0 = plan.simulate(device_depos(wct, wl), wct.opts(3.0, True, 1, wl.seed))
    plain = make_plan(wct, wl)
    w1 = plain.simulate(device_depos(wct, wl), wct.opts(3.0, True, 1, wl.seed))
    assert np.array_equal(to_np(w0), to_np(w1))
    plan.close()
    plain.close()


def test_noise_in_batches_keyed_by_event(wct):
    import torch
    wl = synth.config2(n_depos=900, n_tracks=3, n_ticks=1024, wires=(240, 240, 346), fluctuate=True)
    d = wl.depos
    d.event = (np.arange(len(d)) % 3).astype(np.int32)
    plan = make_plan(wct, wl, max_events=2)
    amps = set_noise(plan, wl)
    dd = device_depos(wct, wl, d)
    say("noise, 3 events in sub-batches of 2 vs single calls")
    batched = plan.simulate(dd, wct.opts(3.0, True, 3, 9, noise=True)).clone()
    singles = [plan.simulate(dd, wct.opts(3.0, True, 1, 9, event_base=e, noise=True)).clone() for e in range(3)]
    torch.cuda.synchronize()
    assert torch.equal(batched, torch.cat(singles))
    # event 2 is its signal plus the oracle's noise of event id 2
    grids = OF.raster_fluct(d, wl.planes, seed=9, n_events=3)[2]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    noise = oracle_noise(plan, wl, amps, 9, 2)
    for k, a in enumerate(plan.wave_view(singles[2])):
        ref = OC.convolve_fft(grids[k], R[k], wl.planes[k].n_impacts) + noise[k]
        assert rel_l2(to_np(a), ref) < TOL32, k
    plan.close()


def test_noise_full_geometry_sampled_wires(wct):
    wl = synth.config2(n_depos=10)
    plan = make_plan(wct, wl)
    amps = set_noise(plan, wl)
    say("noise alone, three-plane geometry, 9600 ticks")
    w = plan.simulate(empty_depos(wct, wl), wct.opts(3.0, True, 1, 31, noise=True))
    rng = np.random.default_rng(2)
    for p, pl in enumerate(wl.planes):
        wires = np.concatenate([[0, pl.n_wires - 1], rng.integers(0, pl.n_wires, 4)])
        ref = ON.noise_waveforms(amps[p], 31, 0, p, pl.n_wires, pl.n_ticks, plan.plane_info(p)["lt"], wires=wires)
        got = to_np(plan.wave_view(w)[p])[wires]
        assert rel_l2(got, ref) < TOL32, p
        # the waveform's RMS is the spectrum's (Parseval; a sample of wires: loose bound)
        assert abs(np.sqrt(np.mean(got ** 2)) / RMS[p] - 1.0) < 0.2
    plan.close()


def test_bad_noise_spectra_refused(wct):
    wl = synth.config1(n_depos=10)
    plan = make_plan(wct, wl)
    F = plan.plane_info(0)["lt"] // 2 + 1
    with pytest.raises(wct.WctError) as e:
        plan.set_noise(0, np.ones(F - 1))
    assert e.value.code == wct.WCT_E_INVALID
    bad = np.ones(F)
    bad[3] = -1.0
    with pytest.raises(wct.WctError):
        plan.set_noise(0, bad)
    with pytest.raises(wct.WctError):
        plan.set_noise(5, np.ones(F))
    plan.set_noise(0, np.ones(F))
    plan.set_noise(0, None)  # removed: noise = 1 then adds nothing
    w = plan.simulate(empty_depos(wct, wl), wct.opts(3.0, False, 1, 1, noise=True))
    assert float(np.abs(to_np(w)).max()) == 0.0
    plan.close()
