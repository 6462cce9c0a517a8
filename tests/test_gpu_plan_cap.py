"""Plan creation under a device memory cap (WCT_PLAN_MEM_CAP): a plan whose tables need
more than the cap fails with WCT_E_NOMEM and a message naming the cap, leaves no plan
behind, and the same description builds and simulates once the cap allows it (or is
unset).  The cap binds plan creation only: set-up calls after it allocate freely.
"""
import pytest
import torch

from gpu_util import device_depos, make_plan, say
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu


def small():
    return synth.config2(n_depos=300, n_tracks=2, n_ticks=960, wires=(240, 240, 346), fluctuate=True)


def test_cap_refuses_then_allows(wct, monkeypatch):
    wl = small()
    for cap in ("4096", "1000000"):
        monkeypatch.setenv("WCT_PLAN_MEM_CAP", cap)
        say("plan creation under a cap of", cap, "bytes")
        with pytest.raises(wct.WctError) as ei:
            make_plan(wct, wl)
        assert ei.value.code == wct.WCT_E_NOMEM
        assert "WCT_PLAN_MEM_CAP" in str(ei.value)
    monkeypatch.setenv("WCT_PLAN_MEM_CAP", str(1 << 40))
    plan = make_plan(wct, wl)
    # later set-up calls are not capped
    plan.set_fft(0, 1, -1)
    dd = device_depos(wct, wl)
    o = wct.opts(3.0, True, 1, 4)
    w1 = plan.simulate(dd, o).clone()
    plan.close()
    monkeypatch.delenv("WCT_PLAN_MEM_CAP")
    plan = make_plan(wct, wl)
    plan.set_fft(0, 1, -1)
    w2 = plan.simulate(dd, o)
    torch.cuda.synchronize()
    assert torch.equal(w1, w2)
    plan.close()
