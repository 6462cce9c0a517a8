"""CPU check of the HIP path's transforms: the product's Stockham butterflies and plans run on
the host (tests/fft_host/fft_host_check.hip) against a direct long-double DFT, for every
transform length the configured geometries use and every radix policy."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LENGTHS = [2, 8, 16, 30, 625, 3125, 5000, 270, 2430, 3600, 810, 972, 1000, 4096]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("fft") / "fft_host_check")
    subprocess.run([hipcc, "-std=c++17", "-O2", "--offload-arch=gfx950", "-I",
                    os.path.join(ROOT, "paper_2104_08265_amd", "csrc"), "-x", "hip",
                    os.path.join(HERE, "fft_host", "fft_host_check.hip"), "-o", exe], check=True, capture_output=True)
    return exe


CASES = [(n, p) for n in LENGTHS for p in (0, 1, 2) if n <= 1000 or p == 0] + [(5000, 1), (3600, 1)]


@pytest.mark.parametrize("n,policy", CASES)
def test_transform_lengths(checker, n, policy):
    out = subprocess.run([checker, str(n), str(policy), "1"], capture_output=True, text=True, check=True).stdout.split()
    f64f, f64i, f32f, f32i = (float(v) for v in out[:4])
    radices = [int(v) for v in out[4:]]
    prod = 1
    for r in radices:
        prod *= r
    assert prod == n
    assert f64f < 1e-14 and f64i < 1e-14, out
    assert f32f < 1e-6 and f32i < 1e-6, out


@pytest.mark.parametrize("n", [270, 810, 972, 30])
def test_interleaved_batch_of_four(checker, n):
    out = subprocess.run([checker, str(n), "0", "4"], capture_output=True, text=True, check=True).stdout.split()
    assert float(out[0]) < 1e-14 and float(out[1]) < 1e-14 and float(out[2]) < 1e-6


def test_compiled_variants(checker):
    """Every compiled plan (fftvariants.hpp): forward with its table, inverse with the
    reversed radices, against the long-double DFT (column variants with power twiddles)."""
    lines = subprocess.run([checker, "variants"], capture_output=True, text=True, check=True).stdout.strip().splitlines()
    assert len(lines) >= 10
    for ln in lines:
        f = ln.split()
        ef, ei, ef32, ei32 = (float(v) for v in f[3:7])
        assert ef < 1e-14 and ei < 1e-14, ln
        assert ef32 < 2e-6 and ei32 < 2e-6, ln
