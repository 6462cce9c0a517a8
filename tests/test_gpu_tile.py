"""Raster tile variants and their tuner (Sec. 2.1.1 scatter adding through LDS tiles).

* Every compiled tile shape gives the same grid: fluctuated counts bit for bit equal to
  the oracle's (the reduced three-plane track geometry, crowded tiles split across work
  items, rows at and beyond the grid edges, rows wider than four tiles), mean grids to the
  FP32 / FP64 bars; wct_simulate after a change of tile equals the oracle's waveform.
* wct_plan_tune_raster keeps one of the candidates, appends its cache line, and a second
  plan reading the cache makes the same choice without timing.
"""
import numpy as np
import pytest

from gpu_util import device_depos, make_plan, rel_l2, say, to_np
from oracle import convolve as OC
from oracle import fluct as OF
from oracle import raster as OR
from paper_2104_08265_amd import synth
from test_gpu_parity import edge_workload

pytestmark = pytest.mark.gpu


def crowded_workload():
    pl = synth.Plane(40, 300, 10, 2, 12)
    rng = np.random.default_rng(8)
    n = 1500
    d = synth.Depos(rng.lognormal(7, 0.5, n), rng.uniform(40, 80, n), rng.uniform(10, 13, n),
                    rng.uniform(0.5, 1.5, n), rng.uniform(0.05, 0.2, n), np.zeros(n, np.int32),
                    np.zeros(n, np.int32), np.arange(n, dtype=np.int32))
    return synth.Workload("crowd", [pl], [synth.make_response(pl, rng)], synth._finish(d, "f32"), dtype="f32", seed=3)


@pytest.mark.parametrize("name", ["slice", "crowded", "edges32", "edges64"])
def test_every_tile_variant_gives_the_same_grid(wct, name):
    if name == "slice":
        wl = synth.config2(n_depos=1500, n_tracks=5, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    elif name == "crowded":
        wl = crowded_workload()
    else:
        wl = edge_workload("f32" if name == "edges32" else "f64")
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    reff = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
    refm = OR.raster(wl.depos, wl.planes)[0]
    tol = 1e-12 if wl.dtype == "f64" else 1e-5
    cands = plan.tile_candidates()
    assert len(cands) >= 2
    for v in cands:
        plan.set_tile(v)
        assert plan.get_tile() == v
        say(name, "tile variant", v)
        g = plan.raster(dd, wct.opts(3.0, True, 1, wl.seed))
        for k, gv in enumerate(plan.grid_view(g)):
            assert np.array_equal(to_np(gv), reff[k]), (v, k)
        g = plan.raster(dd, wct.opts(3.0, False, 1, wl.seed))
        for k, gv in enumerate(plan.grid_view(g)):
            assert rel_l2(to_np(gv), refm[k]) < tol, (v, k)
    plan.close()


def test_simulate_after_tile_change(wct):
    wl = synth.config2(n_depos=800, n_tracks=3, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    grids = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
    R = [r.astype(np.float64) for r in synth.round_responses(wl)]
    for v in plan.tile_candidates()[::-1]:
        plan.set_tile(v)
        say("simulate with tile variant", v)
        w = plan.simulate(dd, wct.opts(3.0, True, 1, wl.seed))
        for k, wv in enumerate(plan.wave_view(w)):
            assert rel_l2(to_np(wv), OC.convolve_fft(grids[k], R[k], wl.planes[k].n_impacts)) < 1e-5, (v, k)
    plan.close()


def test_tune_raster_and_cache(wct, tmp_path):
    wl = synth.config2(n_depos=3000, n_tracks=8, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    cache = tmp_path / "tune.txt"
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    o = wct.opts(3.0, True, 1, wl.seed)
    say("tune raster tile")
    v = plan.tune_raster(dd, o, cache)
    assert v in plan.tile_candidates()
    lines = [ln for ln in cache.read_text().splitlines() if ln.startswith("wct-tile")]
    assert len(lines) == 1 and " fluct 1 -> " in lines[0]
    plan2 = make_plan(wct, wl)
    assert plan2.tune_raster(dd, o, cache) == v
    assert len([ln for ln in cache.read_text().splitlines() if ln.startswith("wct-tile")]) == 1
    # the tuned plan still rasterises exactly
    g = plan2.raster(dd, o)
    ref = OF.raster_fluct(wl.depos, wl.planes, seed=wl.seed)[0]
    for k, gv in enumerate(plan2.grid_view(g)):
        assert np.array_equal(to_np(gv), ref[k]), k
    plan.close()
    plan2.close()


def test_bad_tile_variant_refused(wct):
    wl = synth.config1(n_depos=10)
    plan = make_plan(wct, wl)  # FP64: the FP32 variants do not apply
    f32 = [v["index"] for v in wct.tile_variants() if v["dtype"] == "f32"]
    with pytest.raises(wct.WctError):
        plan.set_tile(f32[0])
    with pytest.raises(wct.WctError):
        plan.set_tile(999)
    plan.close()
