"""The throughput probes (include/wct_probe.h): float atomic adds into LDS and device
memory, and the issue rates of the instruction kinds the kernels use.  Each returns a
positive rate below the chip's nominal bound (256 CUs x 64 lanes x 2.4 GHz lane operations
per second, twice that for FP32 FMAs, which can issue two per lane and cycle), and bad
arguments are refused before anything is launched."""
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu
LANE_RATE = 256 * 64 * 2.4e9


def test_issue_rates(wct):
    rates = {}
    for kind in wct.ISSUE_KINDS:
        say("issue rate", kind)
        rates[kind] = wct.probe_issue_rate(kind, iters=512)
        bound = (2.2 if kind == "fma_f32_vgpr" else 1.1) * LANE_RATE
        assert 0.05 * LANE_RATE < rates[kind] < bound, (kind, rates[kind])
    from ctypes import byref, c_double, c_void_p
    r = c_double()
    buf = torch.empty(256, dtype=torch.int64, device="cuda:0")
    assert wct.wct_probe_issue_rate(4, 1, 1, c_void_p(buf.data_ptr()), 2048, byref(r), None) == -1
    assert wct.wct_probe_issue_rate(0, 2, 1, c_void_p(buf.data_ptr()), 2048, byref(r), None) == -1  # too small
    assert "buffer" in wct.wct_probe_last_error().decode()


def test_atomic_add_rates(wct):
    say("atomic add rates")
    lds, _ = wct.probe_atomic_add("lds", blocks=512, iters=64)
    glob, _ = wct.probe_atomic_add("global", blocks=512, iters=16, buf_elems=512 * 256 * 2)
    assert 0 < lds < 4 * LANE_RATE and 0 < glob < 4 * LANE_RATE
