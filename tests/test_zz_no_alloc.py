"""wct_raster_noalloc: the raster with the library's static device scratch, for callers
that cannot allocate.

Two calls in a row through the C ABI, the second with fewer rows (and a different event
window) than the first, so the second runs on scratch that still holds the first call's
contents: each grid equals wct_raster's grid of the same input (fluctuated: bit for bit;
mean: to the FP32 relative-L2 bar, the atomics' order aside) and the oracle's fluctuated
counts.  A call whose scratch need exceeds WCT_NOALLOC_SCRATCH_BYTES is refused with
WCT_E_WORKSPACE before anything is enqueued.
"""
import numpy as np
import pytest

from gpu_util import device_depos, make_plan, rel_l2, say, to_np
from oracle import fluct as OF
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu


def test_noalloc_raster_two_calls(wct):
    import torch
    wl = synth.config2(n_depos=3000, n_tracks=6, n_ticks=960, wires=(240, 240, 346), fluctuate=True)
    plan = make_plan(wct, wl, max_events=2)
    d_all = wl.depos
    ev = (np.arange(len(d_all)) % 2).astype(np.int32)
    d_all.event = ev
    big = device_depos(wct, wl, d_all)
    small_rows = d_all.select(np.arange(len(d_all)) < len(d_all) // 3)
    small = device_depos(wct, wl, small_rows)
    cases = [(big, d_all, wct.opts(3.0, True, 2, 17)), (small, small_rows, wct.opts(3.0, True, 1, 17, event_base=1))]
    for n, (dd, host, o) in enumerate(cases):
        say("noalloc raster call", n, "rows", dd.n, "events", o.n_events)
        grid = plan.new_grid(o.n_events)
        grid.fill_(-7.0)  # every cell must be written
        plan.raster_noalloc(dd, o, grid)
        ref = plan.raster(dd, o)
        torch.cuda.synchronize()
        assert torch.equal(grid, ref), n
        oracle = OF.raster_fluct(host, wl.planes, seed=17, n_events=2)
        for slot in range(o.n_events):
            for k, g in enumerate(plan.grid_view(grid, slot)):
                assert np.array_equal(to_np(g), oracle[o.event_base + slot][k]), (n, slot, k)
    # the mean raster (float atomics: equal up to the order of additions)
    for n, (dd, host, o) in enumerate(cases):
        om = wct.opts(3.0, False, o.n_events, 17, event_base=o.event_base)
        grid = plan.new_grid(o.n_events)
        plan.raster_noalloc(dd, om, grid)
        ref = plan.raster(dd, om)
        assert rel_l2(to_np(grid), to_np(ref)) < 1e-6, n
    plan.close()


def test_noalloc_raster_refuses_oversized_input(wct):
    import torch
    wl = synth.config2(n_depos=10, n_ticks=960, wires=(240, 240, 346))
    plan = make_plan(wct, wl)
    n = 4_000_000  # rows: their lists alone need more than the static scratch
    assert wct.wct_workspace_bytes(plan.h, wct.OP_RASTER, 1, n) > wct.NOALLOC_SCRATCH_BYTES
    z = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    dd = wct.DeviceDepos(z, z, z, z + 1, z + 1)
    grid = plan.new_grid(1)
    with pytest.raises(wct.WctError) as e:
        plan.raster_noalloc(dd, wct.opts(3.0, True, 1, 1), grid)
    assert e.value.code == wct.WCT_E_WORKSPACE
    assert "scratch" in wct.last_error()
    plan.close()
