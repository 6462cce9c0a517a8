"""wct_simulate_graph: wct_simulate replayed from a HIP graph the plan captures and keeps.

* Every launch of the graph equals the eager wct_simulate bit for bit (fluctuated grid,
  noise on every plane, five events in sub-batches of two), on the current stream and on
  another one, with eager calls of other arguments and synchronisations between launches.
* The graph reads its buffers when it runs: depositions changed in place give the eager
  result of the new values.  New options (a seed) capture a new graph; the old one still
  launches.  Set-up calls (noise amplitudes, tile shape, the wire pass's variant) drop the
  graphs, and the next call captures with the new settings.
* The first graph's waveform equals the oracle's fluctuated raster, FFT convolution and
  noise (FP32, relative L2 1e-5 per plane).
* No depositions: the noise alone, equal to the eager call.
* Refused while kernel timing is on.
"""
import numpy as np
import pytest
import torch

from gpu_util import device_depos, make_plan, rel_l2, say, to_np
from oracle import convolve as OC
from oracle import fluct as OF
from oracle import noise as ONZ
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu


def five_events():
    wl = synth.config2(n_depos=1500, n_tracks=5, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    rng = np.random.default_rng(6)
    ev = rng.choice(5, size=len(wl.depos), p=[0.1, 0.35, 0.1, 0.3, 0.15]).astype(np.int32)
    order = np.argsort(ev, kind="stable")
    d = wl.depos.select(order)
    d.event = ev[order]
    return wl, d


def noise_on(plan, scale=1.0):
    amps = []
    for p in range(plan.n_planes):
        a = synth.noise_amplitude(plan.plane_info(p)["lt"], scale * (150.0 + 40.0 * p))
        plan.set_noise(p, a)
        amps.append(a)
    return amps


def eager(plan, dd, o):
    w = plan.simulate(dd, o)
    torch.cuda.synchronize()
    return w.clone()


def test_graph_replays_equal_eager(wct):
    wl, d = five_events()
    plan = make_plan(wct, wl, max_events=2)
    amps = noise_on(plan)
    dd = device_depos(wct, wl, d)
    o = wct.opts(3.0, True, 5, 33, noise=True)
    ref = eager(plan, dd, o)
    wave = plan.new_wave(5)
    say("simulate_graph: capture, 5 events in sub-batches of 2, noise on")
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    # the oracle's waveform of event 1
    S = OF.raster_fluct(d, wl.planes, seed=33, n_events=5)[1]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    for k, (w, pl) in enumerate(zip(plan.wave_view(wave, 1), wl.planes)):
        M = OC.convolve_fft(S[k], R[k], pl.n_impacts)
        M = M + ONZ.noise_waveforms(amps[k], 33, 1, k, pl.n_wires, pl.n_ticks, plan.plane_info(k)["lt"])
        assert rel_l2(to_np(w), M) < 1e-5, k
    for rep in range(3):
        wave.fill_(-1.0)
        other = plan.simulate(dd, wct.opts(3.0, True, 1, 90 + rep, event_base=rep))  # eager work between
        torch.cuda.synchronize()
        say("simulate_graph: launch", rep)
        plan.simulate_graph(dd, o, wave)
        torch.cuda.synchronize()
        assert torch.equal(wave, ref), rep
        del other
    # launched on another stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    wave.fill_(-1.0)
    with torch.cuda.stream(s):
        plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    plan.close()


def test_graph_reads_buffers_and_keys_options(wct):
    wl, d = five_events()
    plan = make_plan(wct, wl, max_events=2)
    noise_on(plan)
    dd = device_depos(wct, wl, d)
    o = wct.opts(3.0, True, 5, 7, noise=True)
    wave = plan.new_wave(5)
    say("simulate_graph: depositions changed in place")
    plan.simulate_graph(dd, o, wave)
    dd.q.mul_(0.5)
    dd.t.add_(3.0)
    ref = eager(plan, dd, o)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    say("simulate_graph: a new seed, then the first graph again")
    o2 = wct.opts(3.0, True, 5, 8, noise=True)
    ref2 = eager(plan, dd, o2)
    assert not torch.equal(ref, ref2)
    plan.simulate_graph(dd, o2, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref2)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    plan.close()


def test_setup_calls_drop_graphs(wct):
    wl, d = five_events()
    plan = make_plan(wct, wl, max_events=2)
    noise_on(plan)
    dd = device_depos(wct, wl, d)
    o = wct.opts(3.0, True, 3, 12, noise=True)
    wave = plan.new_wave(3)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    say("simulate_graph: after set_noise")
    noise_on(plan, scale=3.0)
    ref = eager(plan, dd, o)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    say("simulate_graph: after set_tile")
    tiles = plan.tile_candidates()
    plan.set_tile(tiles[-1])
    ref = eager(plan, dd, o)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    say("simulate_graph: after set_fft")
    cands = plan.fft_candidates(0, 1)  # the wire pass: direct sum, compiled and runtime transforms
    cur = plan.get_fft(0, 1)
    plan.set_fft(0, 1, next(v for v in cands if v != cur))
    ref = eager(plan, dd, o)
    plan.simulate_graph(dd, o, wave)
    torch.cuda.synchronize()
    assert torch.equal(wave, ref)
    plan.close()


def test_refused_while_timing(wct):
    wl, d = five_events()
    plan = make_plan(wct, wl, max_events=2)
    dd = device_depos(wct, wl, d)
    plan.profile(True)
    with pytest.raises(wct.WctError):
        plan.simulate_graph(dd, wct.opts(3.0, True, 1, 1))
    plan.profile(False)
    w = plan.simulate_graph(dd, wct.opts(3.0, True, 1, 1))
    torch.cuda.synchronize()
    assert torch.equal(w, eager(plan, dd, wct.opts(3.0, True, 1, 1)))
    plan.close()


def test_empty_depositions(wct):
    """No depositions: the graph holds the transform passes alone (the waveform is the
    noise), equal to the eager call."""
    wl, d = five_events()
    plan = make_plan(wct, wl, max_events=2)
    noise_on(plan)
    dd = device_depos(wct, wl, d).slice(0, 0)
    o = wct.opts(3.0, True, 3, 5, noise=True)
    ref = eager(plan, dd, o)
    say("simulate_graph: no depositions, 3 events")
    w = plan.simulate_graph(dd, o)
    torch.cuda.synchronize()
    assert torch.equal(w, ref) and bool(torch.any(ref != 0))
    plan.close()
