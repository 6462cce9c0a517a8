"""The wire pass by transforms along impact bins (Eq. 2): every wire-transform choice
against the FP64 oracle.

A plan starts on the direct 21-wire sums wherever the response is 21 wires wide, so the
other forward wire passes (a length-L_w transform of each impact phase, the product with
the two-dimensional response spectrum, the phase sum, the inverse transform) only run
when selected.  Here each of them is selected on every plane it applies to and the
waveforms are compared with the oracle's FFT convolution of the same grid (responses
jittered per wire and phase: neither separable nor mirror-symmetric, so an index,
sign or conjugation error in the product shows):

* three reduced planes (240/240/346 wires x 960 ticks, FP32): the runtime plan;
* full wire counts of the three-plane (2400/2400/3456) and two-face (800/800/960)
  geometries with 256 ticks (FP32): every compiled whole-chunk and half-chunk variant
  of their lengths 2430, 3600, 810, 972, and the runtime plan;
* the single-plane FP64 geometry (256 wires, L_w = 270): the compiled FP64 variant and
  the runtime plan, to 1e-12;
* full-size planes (9600 and 6000 ticks): one compiled variant per plane, at sampled
  outputs computed one by one by the oracle's direct sum.

Grids are the oracle's fluctuated rasters or seeded sparse grids made on the host, so
the comparison covers the convolution alone.  Bars: relative L2 1e-5 (FP32), 1e-12 (FP64).
"""
import numpy as np
import pytest

from gpu_util import make_plan, rel_l2, say, to_np
from oracle import convolve as OC
from oracle import fluct as OF
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu
TOL32 = 1e-5
TOL64 = 1e-12


def transform_choices(wct, plan, plane):
    return [v for v in plan.fft_candidates(plane, 1) if v != wct.WCT_WIRE_DIRECT]


def sparse_host_grid(rng, nb, nt, n_nonzero, dtype):
    g = np.zeros((nb, nt), dtype)
    idx = rng.integers(0, nb * nt, n_nonzero)
    g.ravel()[idx] = rng.integers(1, 300, n_nonzero).astype(dtype)
    return g


def upload(grids):
    import torch
    return torch.as_tensor(np.concatenate([g.ravel() for g in grids])).to("cuda:0")


def check_all_choices(wct, wl, grids, tol):
    """Every transform choice of every plane against the oracle; returns the choices run
    and the planes' wire transform lengths."""
    plan = make_plan(wct, wl)
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    refs = [OC.convolve_fft(g.astype(np.float64), R[k], pl.n_impacts) for k, (g, pl) in
            enumerate(zip(grids, wl.planes))]
    dev = upload(grids)
    lengths = {plan.plane_info(p)["lw"] for p in range(plan.n_planes)}
    ran = set()
    for p in range(plan.n_planes):
        for v in transform_choices(wct, plan, p):
            plan.set_fft(p, 1, v)
            assert plan.get_fft(p, 1) == v
            say("wire transform plane", p, "variant", v)
            w = to_np(plan.wave_view(plan.convolve(dev, 1))[p])
            err = rel_l2(w, refs[p])
            assert err < tol, (p, v, err)
            ran.add(v)
    plan.close()
    return ran, lengths


def test_runtime_wire_transform_slice_fp32(wct):
    wl = synth.config2(n_depos=2000, n_tracks=5, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    grids = [g.astype(np.float32) for g in OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]]
    say("reduced three-plane geometry, fluctuated oracle grid")
    ran, _ = check_all_choices(wct, wl, grids, TOL32)
    assert -1 in ran


@pytest.mark.parametrize("geom", ["tracks", "showers"])
def test_compiled_wire_transforms_fp32(wct, geom):
    if geom == "tracks":
        wl = synth.config2(n_depos=10, n_ticks=256)
    else:
        wl = synth.config3(n_depos=10, n_ticks=256)
    rng = np.random.default_rng(31 if geom == "tracks" else 37)
    grids = [sparse_host_grid(rng, pl.n_rows, pl.n_ticks, pl.n_rows * 6, np.float32) for pl in wl.planes]
    ran, lengths = check_all_choices(wct, wl, grids, TOL32)
    # every compiled FP32 wire variant of these lengths ran
    want = {v["index"] for v in wct.fft_variants()
            if v["kind"] in (1, 2) and v["dtype"] == "f32" and v["n"] in lengths}
    assert want and want <= ran, (sorted(want), sorted(ran))
    assert -1 in ran


def test_wire_transforms_fp64(wct):
    wl = synth.config1(n_depos=10)
    rng = np.random.default_rng(41)
    pl = wl.planes[0]
    grids = [rng.standard_normal((pl.n_rows, pl.n_ticks)) * (rng.random((pl.n_rows, pl.n_ticks)) < 0.2)]
    ran, _ = check_all_choices(wct, wl, grids, TOL64)
    f64 = {v["index"] for v in wct.fft_variants() if v["kind"] in (1, 2) and v["dtype"] == "f64" and v["n"] == 270}
    assert f64 and f64 <= ran
    assert -1 in ran


@pytest.mark.parametrize("name", ["config2", "config3"])
def test_full_plane_wire_transform_samples(wct, name):
    wl = synth.config2(n_depos=10) if name == "config2" else synth.config3(n_depos=10)
    plan = make_plan(wct, wl)
    for p in range(plan.n_planes):
        comp = [v for v in transform_choices(wct, plan, p) if v >= 0]
        assert comp, p
        plan.set_fft(p, 1, comp[0])
    rng = np.random.default_rng(13)
    grids = [sparse_host_grid(rng, pl.n_rows, pl.n_ticks, 400_000, np.float32) for pl in wl.planes]
    say(name, "full-plane convolution, compiled wire transforms")
    views = plan.wave_view(plan.convolve(upload(grids), 1))
    R = synth.round_responses(wl)
    for k, pl in enumerate(wl.planes):
        got = to_np(views[k])
        g64 = grids[k].astype(np.float64)
        rows = lambda b, g=g64: g[b] if 0 <= b < g.shape[0] else None
        ws = rng.integers(0, pl.n_wires, 60)
        ts = rng.integers(0, pl.n_ticks, 60)
        ws[:4] = [0, pl.n_wires - 1, 0, pl.n_wires - 1]
        ts[:4] = [0, 0, pl.n_ticks - 1, pl.n_ticks - 1]
        ref = np.array([OC.convolve_at(rows, R[k].astype(np.float64), pl.n_impacts, int(w), int(t))
                        for w, t in zip(ws, ts)])
        assert rel_l2(got[ws, ts], ref) < TOL32, k
    plan.close()
