"""Transform variants and their autotuner.

* Every compiled variant that applies to a plane gives the convolution the runtime plan
  gives (same transform, different rounding: relative L2 1e-6 in FP32).
* wct_plan_tune picks a variant per plane and kind, writes the cache file, and a second
  plan reading the cache makes the same choices without timing.
"""
import numpy as np
import pytest

from gpu_util import make_plan, say
from paper_2104_08265_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    import torch
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


@pytest.mark.parametrize("name", ["config2", "config3"])
def test_variants_agree_with_runtime_plan(wct, name):
    import torch
    wl = synth.config2(n_depos=10) if name == "config2" else synth.config3(n_depos=10)
    plan = make_plan(wct, wl)
    rng = np.random.default_rng(3)  # a seeded sparse grid written on the host
    host = rng.random(plan.grid_elems)
    host[rng.random(plan.grid_elems) < 0.9] = 0
    g = torch.as_tensor(host).to("cuda:0", plan.torch_dtype)
    for p in range(plan.n_planes):
        for k in (0, 1):
            plan.set_fft(p, k, -1)
    ref = plan.convolve(g, 1).clone()
    for p in range(plan.n_planes):
        for k in (0, 1):
            for v in plan.fft_candidates(p, k)[:-1]:
                say(name, "plane", p, "kind", k, "variant", v)
                plan.set_fft(p, k, v)
                w = plan.convolve(g, 1)
                assert rel(w, ref) < 1e-6, (p, k, v)
            plan.set_fft(p, k, -1)
    plan.close()


def test_tune_and_cache(wct, tmp_path):
    import torch
    wl = synth.config2(n_depos=10)
    cache = tmp_path / "fft.tune"
    plan = make_plan(wct, wl)
    say("tune config2 geometry")
    choice = plan.tune(1, cache)
    lines = cache.read_text().strip().splitlines()
    # one line per distinct (geometry, kind): planes 0 and 1 share a geometry and a choice
    assert len(lines) == 2 * 2 and len({ln.split(" -> ")[0] for ln in lines}) == len(lines)
    assert choice[(0, 0)] == choice[(1, 0)] and choice[(0, 1)] == choice[(1, 1)]
    for (p, k), v in choice.items():
        assert v in plan.fft_candidates(p, k)
    plan2 = make_plan(wct, wl)
    assert plan2.tune(1, cache) == choice
    assert cache.read_text().strip().splitlines() == lines  # nothing appended
    g = torch.as_tensor(np.random.default_rng(5).random(plan.grid_elems)).to("cuda:0", plan.torch_dtype)
    assert rel(plan.convolve(g, 1), plan2.convolve(g, 1)) == 0.0
    plan.close()
    plan2.close()
