"""The host builds of the product's sampler and transform code under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU code is instrumented).

The sampler checker (tests/sampler_host) runs the kernels' binomial searches, Philox, erf
and normal-mode code on the CPU; the transform checker (tests/fft_host) runs the plan
builder and the Stockham butterflies.  Built with -fno-sanitize-recover, any
out-of-bounds access, signed overflow, misaligned or invalid shift aborts the run; the
outputs must still equal the oracle's (sampler) or the long-double DFT (transforms).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import fluct as OF
from test_sampler_host import edge_triples, triples

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2104_08265_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def build(tmp, src, name, extra):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp / name)
    r = subprocess.run([hipcc, "-std=c++17", "-O0", "-g", "--offload-arch=gfx950", "--cuda-host-only", *extra, *SAN,
                        "-I", CSRC, "-x", "hip", src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def run(exe, args, stdin=""):
    r = subprocess.run([exe, *args], input=stdin, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout


@pytest.fixture(scope="module")
def sampler(tmp_path_factory):
    return build(tmp_path_factory.mktemp("san_sampler"), os.path.join(HERE, "sampler_host", "sampler_host_check.hip"),
                 "sampler_san", ["-ffp-contract=off", "-DWCT_HOST_LOCKSTEP"])


@pytest.fixture(scope="module")
def fft(tmp_path_factory):
    return build(tmp_path_factory.mktemp("san_fft"), os.path.join(HERE, "fft_host", "fft_host_check.hip"),
                 "fft_san", [])


@pytest.mark.parametrize("mode", ["binom", "binom_lockstep"])
def test_sampler_clean_and_equal_oracle(sampler, mode):
    N1, p1, u1 = edge_triples()
    N2, p2, u2 = triples(3, 8000)
    N, p, u = np.concatenate([N1, N2]), np.concatenate([p1, p2]), np.concatenate([u1, u2])
    lines = "".join(f"{int(n)} {float(a).hex()} {float(b).hex()}\n" for n, a, b in zip(N, p, u))
    got = np.array([int(v) for v in run(sampler, [mode], lines).split()], np.int64)
    assert np.array_equal(got, OF.binomial(N, p, u))


def test_sampler_other_modes_clean(sampler):
    x = np.linspace(-7.0, 7.0, 301)
    out = run(sampler, ["erf"], "".join(f"{float(v).hex()}\n" for v in x)).split()
    assert len(out) == x.size


@pytest.mark.parametrize("n,policy,batch", [(625, 0, 1), (5000, 1, 1), (270, 2, 1), (30, 0, 4), (3600, 1, 1),
                                            (972, 0, 4)])
def test_transforms_clean(fft, n, policy, batch):
    out = run(fft, [str(n), str(policy), str(batch)]).split()
    assert float(out[0]) < 1e-14 and float(out[1]) < 1e-14 and float(out[2]) < 2e-6
