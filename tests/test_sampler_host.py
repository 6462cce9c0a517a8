"""CPU check of the HIP path's fluctuation arithmetic against the oracle.

tests/sampler_host/sampler_host_check.hip is the HIP path's sampler (fluct.hpp) built for
the host: the cheap tests, then the search of the cell's regime, as the raster kernels
combine them; and its Philox4x32-10 with the 53-bit uniforms.  Counts and words must
equal the oracle's (oracle/fluct.py, Sec. 4.3.1 binomial fluctuation) exactly, over
seeded triples (N, p, u) that cover both regimes, both sides of p = 1/2, the regime
switch N p' = 10, the inversion cap (N near 128), the ln(n!) table edge (N near 2^17),
u at 0 and next to 1, and p near 0 and 1.  The normal-approximation mode's Box-Muller
normals, deterministic sqrt, cos and sin, and counts must equal oracle/normal.py's.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import fluct as OF
from oracle import normal as ON

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("sampler") / "sampler_host_check")
    subprocess.run([hipcc, "-std=c++17", "-O2", "-ffp-contract=off", "--offload-arch=gfx950", "-DWCT_HOST_LOCKSTEP",
                    "-I",
                    os.path.join(ROOT, "paper_2104_08265_amd", "csrc"), "-x", "hip",
                    os.path.join(HERE, "sampler_host", "sampler_host_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def run_binom(exe, N, p, u, mode="binom"):
    lines = "".join(f"{int(n)} {float(a).hex()} {float(b).hex()}\n" for n, a, b in zip(N, p, u))
    out = subprocess.run([exe, mode], input=lines, capture_output=True, text=True, check=True).stdout.split()
    return np.array([int(v) for v in out], np.int64)


def triples(seed, n):
    rng = np.random.default_rng(seed)
    N = np.concatenate([rng.integers(1, 60, n // 4), rng.integers(1, 20000, n // 4),
                        np.exp(rng.uniform(0, np.log(2e5), n // 2)).astype(np.int64) + 1])
    p = np.exp(-rng.uniform(0, 14, N.size))
    p = np.where(rng.random(N.size) < 0.2, 1.0 - p, p)
    p = np.where(rng.random(N.size) < 0.1, rng.random(N.size), p)
    u = rng.random(N.size)
    near1 = rng.random(N.size) < 0.05
    u[near1] = 1.0 - np.exp(-rng.uniform(10, 36, near1.sum()))
    return N, p, u


def edge_triples():
    Ns = [1, 2, 3, 10, 11, 127, 128, 129, 130, 1000, 131071, 131072, 131073, 400_000]
    ps = [1e-300, 1e-12, 1e-6, 0.001, 0.05, 0.3, 0.5, np.nextafter(0.5, 1.0), 0.7, 0.999999, np.nextafter(1.0, 0.0)]
    us = [0.0, 1e-17, 0.25, 0.5, 0.75, 0.999, np.nextafter(1.0, 0.0)]
    N, p, u = np.meshgrid(Ns, ps, us, indexing="ij")
    N, p, u = N.ravel(), p.ravel(), u.ravel()
    # the regime switch: N p' = 10 exactly and one ulp to either side
    sw_N = np.array([20, 100, 1000, 12345, 10**6])
    sw_p = 10.0 / sw_N
    sw = [(n, q, v) for n, p0 in zip(sw_N, sw_p) for q in (np.nextafter(p0, 0), p0, np.nextafter(p0, 1))
          for v in (0.1, 0.5, 0.9)]
    N = np.concatenate([N, [t[0] for t in sw]])
    p = np.concatenate([p, [t[1] for t in sw]])
    u = np.concatenate([u, [t[2] for t in sw]])
    return N.astype(np.int64), p.astype(np.float64), u.astype(np.float64)


def test_counts_equal_oracle_edges(checker):
    N, p, u = edge_triples()
    got = run_binom(checker, N, p, u)
    ref = OF.binomial(N, p, u)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(int(N[i]), float(p[i]), float(u[i]), int(got[i]), int(ref[i])) for i in bad[:5]]


@pytest.mark.parametrize("seed", [1, 2])
def test_counts_equal_oracle_random(checker, seed):
    N, p, u = triples(seed, 40000)
    got = run_binom(checker, N, p, u)
    ref = OF.binomial(N, p, u)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(int(N[i]), float(p[i]), float(u[i]), int(got[i]), int(ref[i])) for i in bad[:5]]
    # both regimes and the cheap cases are exercised
    pp = np.minimum(p, 1 - p)
    assert np.sum(N * pp >= 10) > 2000 and np.sum((N * pp < 10) & (got > 0)) > 2000


def test_philox_words_and_uniforms_equal_oracle(checker):
    rng = np.random.default_rng(9)
    keys = [(0, 0), (2**32 - 1, 2**32 - 1), (0x12345678, 0x9ABCDEF0), (1, 0)]
    rows, ref_w, ref_u = [], [], []
    for k0, k1 in keys:
        c = rng.integers(0, 2**32, (500, 4), dtype=np.uint64)
        c[:2] = 0
        c[2:4] = 2**32 - 1
        w = OF.philox4x32_10(c[:, 0], c[:, 1], c[:, 2], c[:, 3], k0, k1)
        rows += [f"{a} {b} {cc} {d} {k0} {k1}\n" for a, b, cc, d in c.tolist()]
        ref_w.append(np.stack(w, 1).astype(np.uint64))
        ref_u.append(np.stack([OF.uniform53(w[0], w[1]), OF.uniform53(w[2], w[3])], 1))
    out = subprocess.run([checker, "philox"], input="".join(rows), capture_output=True, text=True, check=True).stdout
    got = [ln.split() for ln in out.strip().splitlines()]
    got_w = np.array([[int(v) for v in r[:4]] for r in got], np.uint64)
    got_u = np.array([[float.fromhex(v) for v in r[4:]] for r in got])
    assert np.array_equal(got_w, np.concatenate(ref_w))
    assert np.array_equal(got_u, np.concatenate(ref_u))


@pytest.mark.parametrize("seed", [3])
def test_counts_unchanged_by_lockstep_passes(checker, seed):
    """On the GPU the searches run with uniform control: a lane whose search has ended keeps
    taking passes (with its count fixed) while slower lanes of its wave search on.  Here
    each search continues for up to 8 extra passes after its own end; the counts must still
    equal the oracle's."""
    N, p, u = triples(seed, 40000)
    got = run_binom(checker, N, p, u, mode="binom_lockstep")
    ref = OF.binomial(N, p, u)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(int(N[i]), float(p[i]), float(u[i]), int(got[i]), int(ref[i])) for i in bad[:5]]
    Ne, pe, ue = edge_triples()
    assert np.array_equal(run_binom(checker, Ne, pe, ue, mode="binom_lockstep"), OF.binomial(Ne, pe, ue))


def test_normal_mode_equals_oracle(checker):
    rng = np.random.default_rng(12)
    n = 20000
    w = rng.integers(0, 2**32, (n, 4), dtype=np.uint64)
    w[:4, :2] = 0                # u1 = 1: r = 0
    w[4:8, :2] = 2**32 - 1       # u1 = 2^-53: the largest r
    w[8:12, 2:] = 0              # u2 = 0
    N = rng.integers(0, 2**31 - 1, n)
    N[:n // 2] = rng.integers(0, 1000, n // 2)
    pe = rng.random(n)
    po = rng.random(n)
    pe[:50], po[:50] = 0.0, 1.0
    pe[50:100] = 2.0 ** -rng.integers(10, 60, 50)
    po[100:200] = np.arange(100) / 100.0  # quadrant edges of the cos/sin argument
    rows = [f"{a} {b} {c} {d} {m} {x.hex()} {y.hex()}\n" for (a, b, c, d), m, x, y in
            zip(w.tolist(), N.tolist(), pe.tolist(), po.tolist())]
    out = subprocess.run([checker, "normal"], input="".join(rows), capture_output=True, text=True, check=True).stdout
    got = [ln.split() for ln in out.strip().splitlines()]
    assert len(got) == n
    ze, zo = ON.box_muller_words(w[:, 0], w[:, 1], w[:, 2], w[:, 3])
    c, s = ON.det_sincos2pi(po)
    ref = [ze, zo, ON.normal_count(N, pe, ze), ON.normal_count(N, po, zo), ON.det_sqrt(pe * 1e6), c, s]
    for col, r in enumerate(ref):
        g = np.array([float.fromhex(x[col]) if col not in (2, 3) else int(x[col]) for x in got])
        assert np.array_equal(g, r), (col, int(np.sum(g != r)))


def test_erf_equals_oracle(checker):
    """The device's det_erf stops its series once the remaining terms cannot change the sum;
    it must still return the oracle's 60-term value bit for bit, over the arguments the
    raster uses (|x| <= 4.2 / sqrt 2) and beyond the checkpoints' thresholds."""
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.uniform(-3.0, 3.0, 200000), rng.uniform(-1e-3, 1e-3, 2000),
                        np.linspace(-2.97, 2.97, 20001), [0.0, -0.0, 1e-300, -1e-300, 2.97, -2.97, 4.2, 6.0]])
    out = subprocess.run([checker, "erf"], input="".join(f"{float(v).hex()}\n" for v in x), capture_output=True,
                         text=True, check=True).stdout.split()
    got = np.array([float.fromhex(v) for v in out])
    ref = OF.det_erf(x)
    assert np.array_equal(got, ref), int(np.sum(got != ref))
