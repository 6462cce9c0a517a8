"""GPU parity of the normal-approximation fluctuation mode (fluctuate = 2; Sec. 4.3.1's
Box-Muller normals) against the oracle (oracle/normal.py).

Counts are integers drawn through IEEE +, -, *, / only on both sides, so every grid must
equal the oracle's bit for bit: the reduced three-plane track geometry, rows at and
beyond the grid edges with invalid rows (FP32 and FP64), crowded tiles split across work
items, rows wider than four tiles, every tile variant, several events in one call, and
sampled 8 x 8 boxes of the full three-plane track event.
"""
import numpy as np
import pytest

from gpu_util import device_depos, make_plan, say, to_np
from oracle import normal as ON
from paper_2104_08265_amd import synth
from test_gpu_fullsize import boxes
from test_gpu_parity import edge_workload, slice_workload
from test_gpu_tile import crowded_workload

pytestmark = pytest.mark.gpu

NORMAL = 2


def check_grid(wct, wl, plan=None, n_events=1):
    plan = plan or make_plan(wct, wl)
    grid = plan.raster(device_depos(wct, wl), wct.opts(3.0, NORMAL, n_events, wl.seed))
    ref = ON.raster_normal(wl.depos, wl.planes, wl.seed, n_events=n_events)
    for e in range(n_events):
        for k, g in enumerate(plan.grid_view(grid, e)):
            got = to_np(g)
            assert ref[e][k].max() < 2 ** 24
            assert np.array_equal(got, ref[e][k]), (e, k, int(np.sum(got != ref[e][k])))
    return plan, ref


def test_slice_fp32_normal_bitexact(wct):
    wl = slice_workload(fluctuate=True)
    say("slice fp32 normal mode", len(wl.depos))
    plan, ref = check_grid(wct, wl)
    assert sum(float(r.sum()) for r in ref[0]) > 0
    # the simulation runs the same raster: simulate == convolve(raster)
    dd = device_depos(wct, wl)
    o = wct.opts(3.0, NORMAL, 1, wl.seed)
    w1 = plan.simulate(dd, o)
    w2 = plan.convolve(plan.raster(dd, o), 1)
    assert np.array_equal(to_np(w1), to_np(w2))
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_edge_rows_normal(wct, dtype):
    wl = edge_workload(dtype)
    say("edge rows normal mode", dtype)
    check_grid(wct, wl)[0].close()


@pytest.mark.parametrize("name", ["slice", "crowded", "edges64"])
def test_every_tile_variant_normal(wct, name):
    if name == "slice":
        wl = synth.config2(n_depos=1500, n_tracks=5, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    elif name == "crowded":
        wl = crowded_workload()
    else:
        wl = edge_workload("f64")
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    ref = ON.raster_normal(wl.depos, wl.planes, wl.seed)[0]
    for v in plan.tile_candidates():
        plan.set_tile(v)
        say(name, "normal mode, tile variant", v)
        g = plan.raster(dd, wct.opts(3.0, NORMAL, 1, wl.seed))
        for k, gv in enumerate(plan.grid_view(g)):
            assert np.array_equal(to_np(gv), ref[k]), (v, k)
    plan.close()


def test_multi_event_normal(wct):
    """Three events in one call: each event's counts are the oracle's for that event."""
    wl = slice_workload(fluctuate=True, n_depos=600)
    parts = []
    for e in range(3):
        d = wl.depos.select(np.arange(len(wl.depos)) % 3 == e)
        d.event = np.full(len(d), e, np.int32)
        parts.append(d)
    allrows = synth.Depos.concat(parts)
    say("normal mode, three events in one call", len(allrows))
    plan = make_plan(wct, wl, max_events=3)
    grid = plan.raster(device_depos(wct, wl, allrows), wct.opts(3.0, NORMAL, 3, 11))
    ref = ON.raster_normal(allrows, wl.planes, 11, n_events=3)
    for e in range(3):
        for k, g in enumerate(plan.grid_view(grid, e)):
            assert np.array_equal(to_np(g), ref[e][k]), (e, k)
    plan.close()


def test_config2_normal_boxes(wct):
    wl = synth.config2()
    say("config2 full normal-mode raster", len(wl.depos))
    plan = make_plan(wct, wl)
    grid = plan.raster(device_depos(wct, wl), wct.opts(3.0, NORMAL, 1, wl.seed))
    views = plan.grid_view(grid)
    rng = np.random.default_rng(6)
    checked = 0
    for k, pl in enumerate(wl.planes):
        g = to_np(views[k])
        for (b0, k0) in boxes(g, 5, 3, rng):
            rr, kk = np.meshgrid(np.arange(b0, b0 + 8), np.arange(k0, k0 + 8), indexing="ij")
            ref = ON.raster_normal_at(wl.depos, k, pl, rr.ravel(), kk.ravel(), wl.seed)
            assert np.array_equal(g[b0:b0 + 8, k0:k0 + 8].ravel(), ref.astype(np.float64)), (k, b0, k0)
            checked += int(np.count_nonzero(ref))
    assert checked > 100
    plan.close()


def test_backward_rejects_normal_mode(wct):
    wl = slice_workload(fluctuate=True, n_depos=50)
    plan = make_plan(wct, wl)
    dd = device_depos(wct, wl)
    gw = plan.new_wave()
    gw.zero_()
    with pytest.raises(wct.WctError):
        plan.simulate_backward(dd, wct.opts(3.0, NORMAL, 1, wl.seed), gw)
    with pytest.raises(wct.WctError):
        plan.raster(dd, wct.opts(3.0, 3, 1, wl.seed))
    plan.close()
