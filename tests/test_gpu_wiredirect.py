"""The direct wire pass (WCT_WIRE_DIRECT): pass B as sums over the response's 21 wires.

* FP32 three-plane geometry (reduced to 240/240/346 wires x 960 ticks so the oracle is
  quick): every plane's waveform equals the oracle's FFT convolution (Eq. 2) of the
  same grid to the FP32 tolerance, with wire counts that leave a partial last tile.
* FP64 single plane (256 wires, one partial tile): to 1e-12.
* Several events in one call equal one call per event bit for bit (the sum order does
  not depend on the batch).
* Adjoint: the gradients of wct_simulate_backward with the direct adjoint equal those of
  the transform adjoints (runtime plan and every compiled wire variant) to FP32 rounding,
  so both adjoint paths stay covered (the gradient tests run the default, direct).
* A response of another width is refused (WCT_E_UNSUPPORTED).
"""
import numpy as np
import pytest

from gpu_util import device_depos, make_plan, rel_l2, say, to_np
from oracle import convolve as OC
from oracle import fluct as OF
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def sparse_grid(plan, seed, density=0.05):
    """A seeded sparse grid written on the host, then uploaded."""
    import torch
    rng = np.random.default_rng(seed)
    g = rng.random(plan.grid_elems)
    g[rng.random(plan.grid_elems) > density] = 0
    return torch.as_tensor(g).to("cuda:0", plan.torch_dtype)


def test_direct_matches_oracle_fp32(wct):
    wl = synth.config2(n_depos=2000, n_tracks=6, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    plan = make_plan(wct, wl)
    for p in range(plan.n_planes):
        plan.set_fft(p, 1, wct.WCT_WIRE_DIRECT)
        assert plan.get_fft(p, 1) == wct.WCT_WIRE_DIRECT
    say("direct wire pass, fluctuated raster of 2000 depositions, 3 reduced planes")
    grid = plan.raster(device_depos(wct, wl), wct.opts(3.0, True, 1, wl.seed))
    wave = plan.convolve(grid, 1)
    ref = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    for k, w in enumerate(plan.wave_view(wave)):
        assert rel_l2(to_np(w), OC.convolve_fft(ref[k], R[k], wl.planes[k].n_impacts)) < TOL32, k
    plan.close()


def test_direct_matches_oracle_fp64(wct):
    wl = synth.config1(n_depos=300)
    plan = make_plan(wct, wl)
    plan.set_fft(0, 1, wct.WCT_WIRE_DIRECT)
    g = sparse_grid(plan, 5, 0.2)
    say("direct wire pass, FP64, 256 wires")
    w = plan.convolve(g, 1)
    S = to_np(g).reshape(wl.planes[0].n_impacts * wl.planes[0].n_wires, wl.planes[0].n_ticks)
    R = synth.round_responses(wl)[0].astype(np.float64)
    assert rel_l2(to_np(plan.wave_view(w)[0]), OC.convolve_fft(S, R, wl.planes[0].n_impacts)) < 1e-12
    plan.close()


def test_direct_event_batch(wct):
    import torch
    wl = synth.config2(n_depos=10, n_ticks=960, wires=(240, 240, 346))
    plan = make_plan(wct, wl, max_events=3)
    ref_plan = make_plan(wct, wl, max_events=3)
    for p in range(plan.n_planes):
        plan.set_fft(p, 1, wct.WCT_WIRE_DIRECT)
        ref_plan.set_fft(p, 1, -1)  # the runtime wire transform, not the direct sums
        assert ref_plan.get_fft(p, 1) == -1
    gs = [sparse_grid(plan, 11 + e) for e in range(3)]
    say("direct wire pass, 3 events in one call vs 3 calls")
    batched = plan.convolve(torch.cat(gs), 3).clone()
    singles = torch.cat([plan.convolve(g, 1).clone() for g in gs])
    torch.cuda.synchronize()
    assert torch.equal(batched, singles)
    # the transform path of the other plan agrees to FP32 rounding
    other = ref_plan.convolve(torch.cat(gs), 3)
    assert rel_l2(to_np(batched), to_np(other)) < 1e-6
    plan.close()
    ref_plan.close()


def test_direct_adjoint_matches_transform_adjoints(wct):
    import torch
    wl = synth.config2(n_depos=300, n_tracks=3, n_ticks=1024, wires=(240, 240, 346), fluctuate=False)
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    o = wct.opts(3.0, False, 1, 1)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(23)
    gw = torch.randn(plan.wave_elems, device="cuda:0", dtype=plan.torch_dtype, generator=gen)
    for p in range(plan.n_planes):
        plan.set_fft(p, 1, wct.WCT_WIRE_DIRECT)
    say("direct adjoint vs transform adjoints")
    ref = [g.clone() for g in plan.simulate_backward(dd, o, gw)]
    cands = [v for v in plan.fft_candidates(0, 1) if v != wct.WCT_WIRE_DIRECT]
    for v in cands:
        for p in range(plan.n_planes):
            if v in plan.fft_candidates(p, 1):
                plan.set_fft(p, 1, v)
        got = plan.simulate_backward(dd, o, gw)
        for a, b in zip(got, ref):
            assert rel_l2(to_np(a), to_np(b)) < 1e-5, v
    plan.close()


def test_direct_needs_21_wire_response(wct):
    pl = synth.Plane(64, 256, 10, 5, 50)
    resp = [synth.make_response(pl, np.random.default_rng(2)).astype(np.float32)]
    plan = wct.Plan([pl], resp, dtype="f32")
    with pytest.raises(wct.WctError) as e:
        plan.set_fft(0, 1, wct.WCT_WIRE_DIRECT)
    assert e.value.code == wct.WCT_E_UNSUPPORTED
    assert wct.WCT_WIRE_DIRECT not in plan.fft_candidates(0, 1)
    plan.close()


def test_simulate_skips_empty_rows_exactly(wct):
    """wct_simulate passes the raster's row flags to the row transform, which then writes
    the zero spectrum of a pair of empty rows without loading or transforming it, and its
    wire flags to the inverse row transform, which writes the zero waveform of a wire no
    window reaches within the response's 21 wires: a sparse event (most impact rows and
    many wires empty) gives the same waveforms as wct_raster followed by wct_convolve
    (every row and wire transformed), for every tick transform (compiled plans with and
    without a partial last wave, the runtime plan), and the flags of an earlier, denser
    call leave nothing behind."""
    import torch
    for n_ticks in (1024, 9600):
        wl = synth.config2(n_depos=60, n_tracks=2, n_ticks=n_ticks, wires=(240, 240, 346), fluctuate=True)
        plan = make_plan(wct, wl, max_events=2)
        cands = plan.fft_candidates(0, 0)
        assert len(cands) > 1  # compiled tick plans (wire-pair kernel)
        dd = device_depos(wct, wl)
        o = wct.opts(3.0, True, 1, wl.seed)
        dense_dd = device_depos(wct, synth.config2(n_depos=3000, n_tracks=8, n_ticks=n_ticks, wires=(240, 240, 346)))
        for v in cands:
            for p in range(plan.n_planes):
                plan.set_fft(p, 0, v)
            say(f"simulate with row flags vs raster + convolve, sparse event, {n_ticks} ticks, tick plan {v}")
            dense = plan.simulate(dense_dd, o).clone()
            w1 = plan.simulate(dd, o).clone()  # after a dense call: rows it reached must not leak in
            w2 = plan.convolve(plan.raster(dd, o), 1)
            torch.cuda.synchronize()
            assert torch.equal(w1, w2), (n_ticks, v)
            assert not torch.equal(w1, dense)
            quiet = [int((wv.abs().amax(dim=1) == 0).sum()) for wv in plan.wave_view(w1)]
            assert all(0 < q < info["n_wires"] for q, info in zip(quiet, plan.info)), quiet
        if n_ticks == 1024:
            ref = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
            R = [r.astype(np.float64) for r in synth.round_responses(wl)]
            for k, w in enumerate(plan.wave_view(w1)):
                assert rel_l2(to_np(w), OC.convolve_fft(ref[k], R[k], wl.planes[k].n_impacts)) < TOL32, k
        plan.close()
