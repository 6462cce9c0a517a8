"""Helpers shared by the GPU parity tests (no arithmetic of the method lives here)."""
import sys

import numpy as np


def say(*a):
    """Name the case on stdout before a GPU step (flushed, so a fault still shows it)."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    den = np.linalg.norm(y)
    return float(np.linalg.norm(x - y) / (den if den > 0 else 1.0))


def make_plan(wct, wl, max_events=1):
    from paper_2104_08265_amd import synth
    planes = [synth.Plane(pl.n_wires, pl.n_ticks, pl.n_impacts, pl.half_wires, pl.resp_ticks, pl.kind)
              for pl in wl.planes]
    return wct.Plan(planes, synth.round_responses(wl), dtype=wl.dtype, max_events=max_events)


def device_depos(wct, wl, depos=None):
    import torch
    d = wl.depos if depos is None else depos
    dt = torch.float32 if wl.dtype == "f32" else torch.float64
    return wct.DeviceDepos.from_numpy(d, "cuda:0", dt)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)
