#!/usr/bin/env python3
"""Throughput of the LArTPC signal-simulation hot path on one MI355X.

One step = wct_simulate on one event of the three-plane workload (2400 + 2400 + 3456
wires x 9600 ticks, 10 impact rows per pitch, 1e5 depositions on 50 seeded straight
tracks, FP32, binomial fluctuation on): rasterisation with scatter adding, then the FFT
convolution with the pre-computed response spectrum.  Inputs are resident in HBM when
the timed region starts.  Prints one JSON line.

Extras on the same line: planes/s; per-kernel device times from HIP events recorded
around every kernel on the launch stream during the timed region; the roofline of the
dominant kernel; the forward+backward / forward time ratio of the differentiable mode
(one plane 256 wires x 1024 ticks, 2e4 track depositions, FP32); and the FP64 CPU
oracle timed on a bounded sample of the same workload on this host's cores.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_JSON = os.path.join(PROFILES, "hbm_traffic.json")

# The commands whose output --summarize reads (run from /tmp on the GPU host, R = repo root).
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d $R/gpurun_out/prof_cfg2 -o cfg2 -- "
             "python3 $R/bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras --raster-tile 128x48x5 "
             "--tune-cache $R/gpurun_out/fft.tune",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d $R/gpurun_out/pmc_fetch -o fetch -- "
             "python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --copy-calibration-mib 1024 "
             "--raster-tile 128x48x5 --tune-cache $R/gpurun_out/fft.tune",
    "write": "rocprofv3 --pmc WRITE_SIZE -f csv -d $R/gpurun_out/pmc_write -o write -- "
             "python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --copy-calibration-mib 1024 "
             "--raster-tile 128x48x5 --tune-cache $R/gpurun_out/fft.tune",
    "trace_showers": "rocprofv3 --kernel-trace --stats -f csv -d $R/gpurun_out/prof_cfg3 -o cfg3 -- "
                     "python3 $R/bench.py --showers-only --steps 3",
    "sq": "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_LDS_ATOMIC SQ_THREAD_CYCLES_VALU "
          "SQ_ACTIVE_INST_VALU SQ_WAVES SQ_LDS_BANK_CONFLICT -f csv -d $R/gpurun_out/pmc_sq -o sq -- "
          "python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --raster-tile 128x48x5 "
          "--tune-cache $R/gpurun_out/fft.tune",
    "atomic": "rocprofv3 --pmc TCC_ATOMIC TCP_TOTAL_ATOMIC_WITHOUT_RET -f csv -d $R/gpurun_out/pmc_atomic -o atomic -- "
              "python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --raster-tile 128x48x5 "
          "--tune-cache $R/gpurun_out/fft.tune",
}
COUNTERS_JSON = os.path.join(PROFILES, "raster_counters.json")


def family(kernel_name):
    """Kernel family (the names of the per-kernel table) of a device kernel symbol."""
    n = kernel_name.split("(")[0]
    if "k_tile<" in n:  # k_tile<T, mode, ...>: 0 mean, 1 binomial, 2 normal approximation
        mode = n.split("k_tile<", 1)[1].split(",")[1].strip()
        return {"0": "raster_tile_mean", "1": "raster_tile_fluct", "2": "raster_tile_normal"}.get(mode)
    if "k_big<" in n:
        return "raster_wide_rows"
    if "k_rows_r2c" in n:
        return "rows_r2c"
    if "k_colpass" in n and "adj" not in n:
        return "colpass"
    if "k_rows_c2r" in n and ", false," in n:
        return "rows_c2r"
    return None


def built_digest():
    """Digest of the sources the in-tree libwct.so was built from (written by the build)."""
    try:
        with open(os.path.join(ROOT, "paper_2104_08265_amd", "libwct.sha256")) as f:
            return f.read().strip()
    except OSError:
        return None


def log_line(path):
    """The bench JSON line inside a log file (a dict), or None."""
    with open(path) as f:
        for line in f:
            if line.startswith("{") and '"build"' in line:
                return json.loads(line)
    return None


def log_digest(path):
    """The "build" digest printed in a bench JSON line inside a log file."""
    line = log_line(path)
    return line.get("build") if line else None


def summarize(out_dir):
    """Write profiles/*.md and profiles/hbm_traffic.json from rocprofv3 CSV output."""
    import csv
    import glob
    import collections
    os.makedirs(PROFILES, exist_ok=True)
    stats = glob.glob(os.path.join(out_dir, "prof_cfg2", "*kernel_stats.csv"))[0]
    rows = list(csv.DictReader(open(stats)))
    lines = ["# Kernel time summary: three-plane track workload (1e5 depositions, fluctuation on, FP32)", "",
             "Command (from /tmp, R = repository root):", "", "    " + PROFILE_COMMANDS["trace"], "",
             "5 timed + 1 warm-up steps of wct_simulate, plus plan creation (k_resp_*).", "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:16]:
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    open(os.path.join(PROFILES, "simulate_3plane_1e5_kernel_stats.md"), "w").write("\n".join(lines) + "\n")
    shower = glob.glob(os.path.join(out_dir, "prof_cfg3", "*kernel_stats.csv"))
    if shower:
        rows = list(csv.DictReader(open(shower[0])))
        lines = ["# Kernel time summary: shower workload (two faces, 1e6 depositions, fluctuation on, FP32)", "",
                 "Command (from /tmp, R = repository root):", "", "    " + PROFILE_COMMANDS["trace_showers"], "",
                 "3 timed + 1 warm-up calls of wct_simulate (k_tile: one launch per call), plus plan creation "
                 "(k_resp_*) and the transform tuner's timing runs (the many short transform launches).", "",
                 "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
        for r in rows[:16]:
            name = r["Name"].split("(")[0].replace("void ", "")
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
        open(os.path.join(PROFILES, "simulate_showers_1e6_kernel_stats.md"), "w").write("\n".join(lines) + "\n")

    def counters(tag, counter):
        path = glob.glob(os.path.join(out_dir, f"pmc_{tag}", "*counter_collection.csv"))[0]
        acc = collections.defaultdict(lambda: [0.0, 0])
        copies = []
        seen = []  # (dispatch, family, KiB)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            kib = float(r["Counter_Value"])
            if r["Kernel_Name"] == "__amd_rocclr_copyBuffer":
                copies.append(kib)
            fam = family(r["Kernel_Name"])
            if fam:
                seen.append((int(r["Dispatch_Id"]), fam, kib))
        # the headline step's launches of its own kernels: the last of each family before
        # the mean raster the bench runs after the step (the tuners' launches come before
        # it, the noise, ADC and drift figures after it); the other families whole
        means = [d for d, fam, _ in seen if fam == "raster_tile_mean"]
        cut = min(means) if means else None
        step_fams = {"rows_r2c": 3, "colpass": 3, "rows_c2r": 3, "raster_tile_fluct": 1}
        keep = set()
        for fam, n in step_fams.items():
            ids = sorted({d for d, f, _ in seen if f == fam and (cut is None or d < cut)})
            keep.update((fam, d) for d in ids[-n:])
        for d, fam, kib in seen:
            if fam not in step_fams or (fam, d) in keep:
                acc[fam][0] += kib
                acc[fam][1] += 1
        # three 1 GiB device copies: the counter's reading for a known 1 GiB (= 1048576 KiB)
        big = sorted(copies)[-3:]
        scale = 1048576.0 / (sum(big) / len(big))
        return acc, scale

    fetch, fs = counters("fetch", "FETCH_SIZE")
    write, ws = counters("write", "WRITE_SIZE")
    digest = log_digest(os.path.join(out_dir, "pmc_fetch.log"))
    if digest is None or digest != log_digest(os.path.join(out_dir, "pmc_write.log")):
        raise SystemExit("the two counter runs do not name the same library build")
    # the raster's traffic depends on the tile shape the tuner chose in those runs
    tiles = [(log_line(os.path.join(out_dir, f"pmc_{t}.log")) or {}).get("raster_tile") for t in ("fetch", "write")]
    tile = tiles[0] if tiles[0] is not None and tiles[0] == tiles[1] else None
    traffic = {"build": digest, "fetch_scale": fs, "write_scale": ws, "kernels": {}, "raster_tile": tile,
               "commands": {k: PROFILE_COMMANDS[k] for k in ("fetch", "write")}}
    lines = ["# HBM traffic per kernel family: three-plane track workload, one step", "",
             "Commands (separate runs, from /tmp, R = repository root):", "",
             "    " + PROFILE_COMMANDS["fetch"], "    " + PROFILE_COMMANDS["write"], "",
             f"Calibration: three plain 1 GiB device copies read {1048576 / fs:.0f} KiB (FETCH_SIZE) and wrote "
             f"{1048576 / ws:.0f} KiB (WRITE_SIZE) per copy, so the counters are scaled by {fs:.4f} (fetch) "
             f"and {ws:.4f} (write).", "",
             (f"Raster tile shape of both runs (set with --raster-tile): {tile['rows']} x {tile['ticks']}, "
              f"{tile['blocks_per_cu']} blocks per CU; the bench reports the raster's traffic only when it runs "
              f"the same shape." if tile else "The two runs chose different raster tile shapes: the raster's "
              "traffic is not reported."), "",
             "| family | launches | fetch GB | write GB | total GB per launch |", "|---|---|---|---|---|"]
    for fam in sorted(set(fetch) | set(write)):
        f_b = fetch[fam][0] * 1024 * fs
        w_b = write[fam][0] * 1024 * ws
        n = max(fetch[fam][1], write[fam][1], 1)
        traffic["kernels"][fam] = {"fetch_bytes": f_b, "write_bytes": w_b, "launches": n,
                                   "bytes_per_launch": (f_b + w_b) / n}
        lines.append(f"| {fam} | {n} | {f_b / 1e9:.3f} | {w_b / 1e9:.3f} | {(f_b + w_b) / n / 1e9:.3f} |")
    open(os.path.join(PROFILES, "simulate_3plane_1e5_hbm_traffic.md"), "w").write("\n".join(lines) + "\n")
    json.dump(traffic, open(TRAFFIC_JSON, "w"), indent=1)
    print("\n".join(lines))
    summarize_counters(out_dir)


def summarize_counters(out_dir):
    """profiles/raster_counters.json and .md: per-launch instruction and atomic counters of
    each kernel family (the headline step plus the mean raster the bench runs after it)."""
    import csv
    import glob
    import collections
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    n_launch = {}
    digests = set()
    for tag in ("sq", "atomic"):
        paths = glob.glob(os.path.join(out_dir, f"pmc_{tag}", "*counter_collection.csv"))
        if not paths:
            return
        digests.add(log_digest(os.path.join(out_dir, f"pmc_{tag}.log")))
        last = {}
        rows = list(csv.DictReader(open(paths[0])))
        # the headline step's launches: the last of each family before the mean raster that
        # the bench runs after the step (the tuners run before it; the noise, ADC and drift
        # figures after it run the transform passes again)
        ids_mean = [int(r["Dispatch_Id"]) for r in rows if family(r["Kernel_Name"]) == "raster_tile_mean"]
        cut = min(ids_mean) if ids_mean else None
        for r in rows:
            fam = family(r["Kernel_Name"])
            did = int(r["Dispatch_Id"])
            if fam and (cut is None or did < cut or not fam.startswith(("rows_", "colpass", "raster_tile_fluct"))):
                last.setdefault(fam, []).append(did)
        want = {fam: set(sorted(set(ids))[-3:] if fam in ("rows_r2c", "colpass", "rows_c2r") else sorted(set(ids))[-1:])
                for fam, ids in last.items()}
        for r in rows:
            fam = family(r["Kernel_Name"])
            if fam and int(r["Dispatch_Id"]) in want[fam]:
                per[fam][r["Counter_Name"]] += float(r["Counter_Value"])
        if tag == "sq":
            n_launch = {fam: len(ids) for fam, ids in want.items()}
    if len(digests) != 1 or None in digests:
        raise SystemExit("the counter runs do not name the same library build")
    tiles = [(log_line(os.path.join(out_dir, f"pmc_{t}.log")) or {}).get("raster_tile") for t in ("sq", "atomic")]
    out = {"build": digests.pop(), "commands": {k: PROFILE_COMMANDS[k] for k in ("sq", "atomic")}, "kernels": {},
           "raster_tile": tiles[0] if tiles[0] is not None and tiles[0] == tiles[1] else None}
    names = ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_LDS_ATOMIC", "SQ_THREAD_CYCLES_VALU",
             "SQ_ACTIVE_INST_VALU", "SQ_WAVES", "SQ_LDS_BANK_CONFLICT", "TCC_ATOMIC", "TCP_TOTAL_ATOMIC_WITHOUT_RET"]
    lines = ["# Instruction and atomic counters per launch: three-plane track workload", "",
             "Commands (separate runs, from /tmp, R = repository root):", "",
             "    " + PROFILE_COMMANDS["sq"], "    " + PROFILE_COMMANDS["atomic"], "",
             "One headline step (raster_tile_fluct, the three transform passes) and the mean raster of the same "
             "event that the bench runs after it (raster_tile_mean).  VALU and SALU are wave instructions; "
             "lane use = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU).", "",
             "| family | launches | " + " | ".join(names) + " | lane use |", "|---" * (len(names) + 3) + "|"]
    for fam in sorted(per):
        n = max(n_launch.get(fam, 1), 1)
        vals = {k: per[fam].get(k, 0.0) / n for k in names}
        use = vals["SQ_THREAD_CYCLES_VALU"] / (64 * vals["SQ_ACTIVE_INST_VALU"]) if vals["SQ_ACTIVE_INST_VALU"] else None
        vals["lane_use"] = use
        vals["launches_counted"] = n
        out["kernels"][fam] = vals
        use_txt = f"{use:.2f}" if use is not None else "-"
        lines.append(f"| {fam} | {n} | " + " | ".join(f"{vals[k]:.3e}" for k in names) + f" | {use_txt} |")
    open(os.path.join(PROFILES, "simulate_3plane_1e5_counters.md"), "w").write("\n".join(lines) + "\n")
    json.dump(out, open(COUNTERS_JSON, "w"), indent=1)
    print("\n".join(lines))


def measured_counters(kernel, tile=None):
    """Per-launch counters of a kernel family from committed profiles, or None when the
    library changed since (or, for the raster tiles, when `tile` is not the tile shape the
    counter runs used)."""
    try:
        c = json.load(open(COUNTERS_JSON))
    except (OSError, ValueError):
        return None
    if c.get("build") is None or c.get("build") != built_digest():
        return None
    if kernel.startswith("raster_tile") and (tile is None or c.get("raster_tile") != tile):
        return None
    return c.get("kernels", {}).get(kernel)


def measured_traffic(kernel, tile=None):
    """HBM bytes per launch from committed counters, or None when the kernels changed since
    (or, for the raster tiles, when `tile` is not the tile shape the counter runs used)."""
    try:
        t = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if t.get("build") is None or t.get("build") != built_digest() or kernel not in t.get("kernels", {}):
        return None
    if kernel.startswith("raster_tile") and (tile is None or t.get("raster_tile") != tile):
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # lane operations per second: 256 CUs x 4 SIMD16 x 2.4 GHz


def raster_alu_ops(wl, sample_rows=3000, nsigma=3.0, seed=0):
    """Algorithmic lane operations of one fluctuated raster of the workload (a cost model).

    Per cell of a row's window: half a Philox4x32-10 block (10 rounds of two 32x32->64
    products and two xors, key bumps: 78 ops per block), the 53-bit uniform (7), the
    probability and address (3), the zero bound (6).  Cells that need the full sampler
    add, in the inversion regime (N p' < 10), the set-up (4), the square-and-multiply
    power (bit length + popcount of N) and 6 ops per search step (k steps, E[k] = N p');
    in the chop-down regime the set-up (3 table reads, two logs, one exp: 110) and 7 ops
    per side step (about 2 |k - m| + 1, E|k - m| ~ 0.8 sigma).  Expectations are taken
    over a seeded sample of the workload's rows and scaled to all rows.
    """
    import numpy as np
    from scipy.special import erf
    d = wl.depos
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(d.q), min(sample_rows, len(d.q)), replace=False)
    total = 0.0

    def axis(mu, sig, n):
        lo, hi = mu - nsigma * sig, mu + nsigma * sig
        k = np.arange(np.floor(lo), np.ceil(hi))
        k = k[(k >= 0) & (k < n)]
        e0, e1 = np.maximum(k, lo), np.minimum(k + 1, hi)
        return 0.5 * (erf((e1 - mu) / (sig * np.sqrt(2))) - erf((e0 - mu) / (sig * np.sqrt(2))))

    for j in idx:
        pl = wl.planes[int(d.plane[j])]
        a = axis(pl.n_impacts * float(d.p[j]), pl.n_impacts * float(d.sigma_p[j]), pl.n_impacts * pl.n_wires)
        b = axis(float(d.t[j]), float(d.sigma_t[j]), pl.n_ticks)
        p = np.outer(a, b).ravel()
        p = p[p > 0]
        N = np.floor(float(d.q[j]) + 0.5)
        if N <= 0 or p.size == 0:
            continue
        pp = np.minimum(p, 1 - p)
        mu = N * pp
        ops = p.size * (39 + 7 + 3 + 6)
        inv = mu < 10
        full_inv = inv * np.clip(mu, 0, 1) + inv * (mu >= 1) * (1 - np.clip(mu, 0, 1))  # P(not the zero bound)
        nbits = int(N).bit_length() + bin(int(N)).count("1")
        ops += float(np.sum(full_inv * (4 + nbits + 6 * mu)))
        chop = ~inv
        sig = np.sqrt(N * pp * (1 - pp))
        ops += float(np.sum(chop * (110 + 7 * (2 * 0.8 * sig + 1))))
        total += ops
    return total * len(d.q) / len(idx)


def algorithmic_bytes(plan, esize=4):
    """Bytes each kernel family must move per event (sum over planes) by design."""
    from paper_2104_08265_amd import wct
    out = {"rows_r2c": 0, "colpass": 0, "rows_c2r": 0, "raster_tile_fluct": 0, "raster_tile_mean": 0}
    for p, inf in enumerate(plan.info):
        nb = inf["n_impacts"] * inf["n_wires"]
        nw, nt, F, lw, I = inf["n_wires"], inf["n_ticks"], inf["F"], inf["lw"], inf["n_impacts"]
        c = 2 * esize  # one complex value
        out["rows_r2c"] += esize * nb * nt + c * nb * F          # read S, write S-hat
        if plan.get_fft(p, 1) == wct.WCT_WIRE_DIRECT:  # read S-hat and the 21 I coefficients, write M-hat
            out["colpass"] += c * nb * F + c * I * (2 * inf["half_wires"] + 1) * F + c * nw * F
        else:  # read S-hat and R~, write M-hat
            out["colpass"] += c * nb * F + c * I * lw * F + c * nw * F
        out["rows_c2r"] += c * nw * F + esize * nw * nt          # read M-hat, write M
        out["raster_tile_fluct"] += esize * nb * nt              # write S once
        out["raster_tile_mean"] += esize * nb * nt
    return out


def cpu_baseline(wl, n_sample_depos=3000):
    """The FP64 oracle on a bounded sample (about 10 s of work on one core), scaled to the
    whole event (depos/s)."""
    import numpy as np
    from oracle import convolve as OC
    from oracle import fluct as OF
    d = wl.depos
    # a seeded random sample of the depositions (all their depo-plane rows)
    ids = np.sort(np.random.default_rng(1).choice(np.unique(d.depo_id), n_sample_depos, replace=False))
    sub = d.select(np.isin(d.depo_id, ids))
    t0 = time.perf_counter()
    OF.raster_fluct(sub, wl.planes, seed=wl.seed)
    t_r = time.perf_counter() - t0
    # convolution: one impact phase of the smallest plane, scaled by phases and plane sizes
    pl = wl.planes[0]
    R = wl.responses[0]
    lw = OC._next_pow2(pl.n_wires + 2 * pl.half_wires)
    lt = OC._next_pow2(pl.n_ticks + pl.resp_ticks)
    S = np.zeros((lw, lt))
    S[: pl.n_wires, : pl.n_ticks] = 1.0
    ker = OC.response_kernel(R[:, :1], 1, lw, lt)[0]
    t0 = time.perf_counter()
    np.fft.irfft2(np.fft.rfft2(S) * np.fft.rfft2(ker), s=(lw, lt))
    t_c1 = time.perf_counter() - t0
    conv_units = 0.0
    for p in wl.planes:
        lwp = OC._next_pow2(p.n_wires + 2 * p.half_wires)
        conv_units += p.n_impacts * lwp / lw
    n_all = wl.n_depos
    t_event = t_r * n_all / len(ids) + t_c1 * conv_units
    return {
        "value": n_all / t_event, "unit": "depos/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle fluctuated raster of {len(ids)} of {n_all} depositions ({len(sub)} depo-plane rows, "
                   f"{t_r:.1f} s) + one impact phase of the {pl.n_wires}-wire plane's FFT convolution "
                   f"({t_c1:.1f} s), scaled to the full event ({t_event:.0f} s/event); numpy FP64, single thread"),
        "seconds_measured": t_r + t_c1,
    }


def window_cells(wl, nsigma=3.0):
    """Cells of all rows' truncated windows inside the grid: the mean raster's LDS adds
    (one per cell; rows wider than four tiles excepted, a small share)."""
    import numpy as np
    d = wl.depos
    total = 0
    for k, pl in enumerate(wl.planes):
        m = np.asarray(d.plane) == k
        u, su = pl.n_impacts * np.asarray(d.p, np.float64)[m], pl.n_impacts * np.asarray(d.sigma_p, np.float64)[m]
        t, st = np.asarray(d.t, np.float64)[m], np.asarray(d.sigma_t, np.float64)[m]
        nb = np.minimum(np.ceil(u + nsigma * su), pl.n_impacts * pl.n_wires) - np.maximum(np.floor(u - nsigma * su), 0)
        nt = np.minimum(np.ceil(t + nsigma * st), pl.n_ticks) - np.maximum(np.floor(t - nsigma * st), 0)
        total += int(np.sum(np.clip(nb, 0, None) * np.clip(nt, 0, None)))
    return total


def cpu_parallel_baseline(wl, n_sample_rows=30000):
    """A CPU-parallel leg on this host's cores: the fluctuated raster vectorised in NumPy
    (window weights by scipy's erf, counts by NumPy's binomial generator, scatter-add by
    bincount) over thread-pool chunks, and the FFT convolution by scipy.fft with
    workers = all cores; timed on a sample of rows and one full plane, scaled to the event.
    Not bit-identical to the draw stream of the GPU and the oracle (its own generator): a
    throughput baseline only."""
    import numpy as np
    import scipy.fft as sfft
    from concurrent.futures import ThreadPoolExecutor
    from scipy.special import erf
    cores = os.cpu_count() or 1
    d = wl.depos
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(d.q), min(n_sample_rows, len(d.q)), replace=False))

    def axis(mu, sig, n, width):
        lo, hi = mu - 3 * sig, mu + 3 * sig
        k0 = np.maximum(np.floor(lo), 0)
        k = k0[:, None] + np.arange(width)[None, :]
        e0, e1 = np.maximum(k, lo[:, None]), np.minimum(k + 1, hi[:, None])
        w = 0.5 * (erf((e1 - mu[:, None]) / (sig[:, None] * np.sqrt(2))) - erf((e0 - mu[:, None]) / (sig[:, None] * np.sqrt(2))))
        ok = (k < np.minimum(np.ceil(hi), n)[:, None]) & (e1 > e0)
        return k.astype(np.int64), np.where(ok, w, 0.0)

    def chunk(rows, seed):
        g = np.random.default_rng(seed)
        out = 0
        for k, pl in enumerate(wl.planes):
            r = rows[np.asarray(d.plane)[rows] == k]
            if r.size == 0:
                continue
            u, su = pl.n_impacts * d.p[r].astype(np.float64), pl.n_impacts * d.sigma_p[r].astype(np.float64)
            t, st = d.t[r].astype(np.float64), d.sigma_t[r].astype(np.float64)
            bi, a = axis(u, su, pl.n_impacts * pl.n_wires, int(np.ceil(6 * su.max())) + 2)
            ki, b = axis(t, st, pl.n_ticks, int(np.ceil(6 * st.max())) + 2)
            p = a[:, :, None] * b[:, None, :]
            n = g.binomial(np.floor(d.q[r].astype(np.float64) + 0.5).astype(np.int64)[:, None, None], p)
            cell = bi[:, :, None] * pl.n_ticks + ki[:, None, :]
            keep = n > 0
            out += int(np.bincount(cell[keep], weights=n[keep]).size)
        return out

    parts = np.array_split(idx, cores * 4)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(chunk, parts, range(len(parts))))
    t_r = time.perf_counter() - t0
    # convolution of the first plane: 10 impact phases, rfft2 of each padded phase grid
    # times the response kernel, summed, inverse (scipy.fft, all cores)
    pl = wl.planes[0]
    lw, lt = sfft.next_fast_len(pl.n_wires + pl.half_wires), sfft.next_fast_len(pl.n_ticks + pl.resp_ticks - 1)
    S = np.zeros((pl.n_impacts, lw, lt), np.float32)
    S[:, : pl.n_wires, : pl.n_ticks] = 1.0
    K = np.zeros((pl.n_impacts, lw, lt), np.float32)
    K[:, : 2 * pl.half_wires + 1, : pl.resp_ticks] = np.transpose(wl.responses[0], (1, 0, 2))
    t0 = time.perf_counter()
    acc = np.sum(sfft.rfft2(S, workers=cores) * sfft.rfft2(K, workers=cores), axis=0)
    sfft.irfft2(acc, s=(lw, lt), workers=cores)
    t_c = time.perf_counter() - t0
    cells = sum(p.n_impacts * p.n_wires for p in wl.planes) / pl.n_impacts / pl.n_wires
    t_event = t_r * len(d.q) / len(idx) + t_c * cells
    return {"value": wl.n_depos / t_event, "unit": "depos/s", "cores": cores, "kind": "cpu-parallel",
            "sample": (f"vectorised NumPy fluctuated raster of {len(idx)} of {len(d.q)} depo-plane rows in "
                       f"{cores} threads ({t_r:.2f} s) + scipy.fft convolution of the {pl.n_wires}-wire plane "
                       f"with workers={cores} ({t_c:.2f} s), scaled to the full event ({t_event:.2f} s/event); "
                       f"FP64 raster, FP32 transforms; its own random stream"),
            "seconds_measured": t_r + t_c}


PAPER_CONTEXT = {
    "note": "the paper's timings of the rasterisation step (2D sampling + fluctuation) on ~100k depositions "
            "(Sec. 3), other hardware, context only; no FFT convolution timing is published",
    "ref_cpu_serial_s": {"value": 3.57, "hardware": "AMD Threadripper 3960X, 1 thread", "source": "Table 2"},
    "ref_cuda_s": {"value": 1.22, "hardware": "NVIDIA V100 + host, one depo per launch", "source": "Table 2"},
    "kokkos_omp_1thread_s": {"value": 0.29, "hardware": "3960X, pre-computed RNG", "source": "Table 3"},
    "kokkos_cuda_s": {"value": 2.31, "hardware": "NVIDIA V100", "source": "Table 3"},
}


def fwd_bwd_ratio(wct, synth, steps=10):
    import torch
    wl = synth.config4()
    pl = wl.planes
    plan = wct.Plan(pl, synth.round_responses(wl), dtype="f32")
    dd = wct.DeviceDepos.from_numpy(wl.depos, "cuda:0", torch.float32)
    o = wct.opts(3.0, False, 1, wl.seed)
    wave = plan.simulate(dd, o)
    g = torch.randn_like(wave)
    for _ in range(3):
        plan.simulate(dd, o, wave)
        plan.simulate_backward(dd, o, g)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(steps):
        plan.simulate(dd, o, wave)
    e[1].record()
    for _ in range(steps):
        plan.simulate_backward(dd, o, g)
    e[2].record()
    torch.cuda.synchronize()
    tf = e[0].elapsed_time(e[1]) / steps
    tb = e[1].elapsed_time(e[2]) / steps
    plan.close()
    return {"fwd_ms": tf, "bwd_ms": tb, "ratio": (tf + tb) / tf,
            "workload": "256 wires x 1024 ticks, 2e4 track depositions, FP32, no fluctuation"}


def graph_of(fn):
    """Captures fn's launches (on torch's capture stream) into a HIP graph."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def batch_bench(wct, synth, sub_batch=16, reps=2):
    """The 64-event workload (three-plane geometry, log-uniform event sizes): per-event time of
    one batched call (sub-batches of `sub_batch` events: one persistent raster and one set of
    batched transform passes each) against a loop of one-event calls on each event's own rows,
    both eager and replayed from a HIP graph; outputs of the two are compared bit for bit."""
    import numpy as np
    import torch
    wl = synth.config5()
    n_ev = wl.n_events
    plan = wct.Plan(wl.planes, synth.round_responses(wl), dtype="f32", max_events=sub_batch)
    dd = wct.DeviceDepos.from_numpy(wl.depos, "cuda:0", torch.float32)
    starts = np.searchsorted(wl.depos.event, np.arange(n_ev + 1))
    we = plan.wave_elems
    wave_b = plan.new_wave(n_ev)
    wave_l = plan.new_wave(n_ev)
    plan.tune(1)
    plan.tune_raster(dd, wct.opts(wl.nsigma, True, 4, wl.seed))  # on the rows of the first four events
    torch.cuda.empty_cache()
    plan.workspace(wct.OP_SIMULATE, sub_batch, dd.n)
    o_all = wct.opts(wl.nsigma, True, n_ev, wl.seed)
    singles = [(dd.slice(int(starts[e]), int(starts[e + 1])), wct.opts(wl.nsigma, True, 1, wl.seed, event_base=e),
                wave_l[e * we:(e + 1) * we]) for e in range(n_ev)]

    def batched():
        plan.simulate(dd, o_all, wave_b)

    def loop():
        for d, o, w in singles:
            plan.simulate(d, o, w)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"events": n_ev, "depos": int(wl.n_depos), "sub_batch": sub_batch}
    out["batched_ms_per_event"] = timed(batched) / n_ev
    out["loop_ms_per_event"] = timed(loop) / n_ev
    out["bitwise_equal"] = bool(torch.equal(wave_b, wave_l))
    gb = graph_of(batched)
    out["batched_graph_ms_per_event"] = timed(gb.replay) / n_ev
    gl = graph_of(loop)
    out["loop_graph_ms_per_event"] = timed(gl.replay) / n_ev
    torch.cuda.synchronize()
    out["graph_replay_bitwise_equal"] = bool(torch.equal(wave_b, wave_l))
    del gb, gl
    # the library's own graph of the batched call (wct_simulate_graph: captured on the
    # first call, launched from the plan's cache after)
    wave_b.fill_(-1.0)
    out["batched_abi_graph_ms_per_event"] = timed(lambda: plan.simulate_graph(dd, o_all, wave_b)) / n_ev
    torch.cuda.synchronize()
    out["abi_graph_bitwise_equal"] = bool(torch.equal(wave_b, wave_l))
    plan.close()
    return out


def shower_bench(wct, synth, tune_cache=None, steps=3):
    """The shower workload (two faces x 800+800+960 wires x 6000 ticks, 1e6 depositions in
    20 EM-shower-like clusters, fluctuation on, FP32): time per event of wct_simulate, the
    per-kernel split, and the tile raster on the same lane-operation roofline as the
    three-plane workload."""
    import torch
    wl = synth.config3()
    plan = wct.Plan(wl.planes, synth.round_responses(wl), dtype="f32")
    plan.tune(1, tune_cache)
    dd = wct.DeviceDepos.from_numpy(wl.depos, "cuda:0", torch.float32)
    o = wct.opts(wl.nsigma, True, 1, wl.seed)
    tile = {v["index"]: v for v in wct.tile_variants()}[plan.tune_raster(dd, o, tune_cache)]
    alg = algorithmic_bytes(plan)
    wave = plan.new_wave(1)
    plan.workspace(wct.OP_SIMULATE, 1, dd.n)
    plan.simulate(dd, o, wave)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_reset()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.simulate(dd, o, wave)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kt = plan.profile_read()
    plan.profile(False)
    plan.close()
    kernels = {k: tot / steps for k, (tot, _) in sorted(kt.items(), key=lambda kv: -kv[1][0])}
    t_tile = kernels.get("raster_tile_fluct", 0.0)
    ops = raster_alu_ops(wl)
    passes = ("rows_r2c", "colpass", "rows_c2r")
    t_conv = sum(kernels.get(k, 0.0) for k in passes)
    conv_bytes = sum(alg[k] for k in passes)
    conv_gbs = conv_bytes / (t_conv * 1e-3) / 1e9
    return {"workload": "2 faces x (800+800+960 wires) x 6000 ticks, 10 impacts/pitch, 1e6 depositions in "
                        "20 seeded showers, binomial fluctuation on, FP32",
            "ms_per_event": ms, "depos_per_s": wl.n_depos / (ms * 1e-3),
            "t_raster_ms": sum(v for k, v in kernels.items() if k.startswith("raster")),
            "t_conv_ms": t_conv,
            "kernels_ms": kernels,
            "raster_tile": {"rows": tile["th"], "ticks": tile["tw"], "blocks_per_cu": tile["blocks_per_cu"]},
            "conv_roofline": {"bound": "hbm", "achieved": conv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": conv_gbs / HBM_PEAK_GBS, "alg_bytes": conv_bytes,
                              "per_pass": {k: {"ms": kernels.get(k), "GBps": alg[k] / (kernels[k] * 1e-3) / 1e9,
                                               "frac": alg[k] / (kernels[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                                           for k in passes if kernels.get(k)},
                              "note": "algorithmic bytes of the three transform passes (read S, S-hat, M-hat once, "
                                      "write each once) / their summed time"},
            "tile_raster_alu_frac": ops / (t_tile * 1e-3) / 1e12 / ALU_PEAK_TOPS if t_tile > 0 else None}


def issue_rates(wct):
    """The chip's sustained rates for the instruction kinds the kernels issue (the probe):
    lane operations per second and wave64 instructions per CU per 2.4 GHz cycle."""
    out = {}
    for kind in wct.ISSUE_KINDS:
        r = wct.probe_issue_rate(kind)
        out[kind] = {"lane_ops_per_s": r, "wave_instr_per_cu_cycle": r / (64 * 256 * 2.4e9)}
    out["probe"] = ("wct_probe_issue_rate: 16 independent chains per thread, 16 blocks of 256 threads per CU; "
                    "fma_f32_sgpr takes its multiplier from a scalar register, as the direct wire pass does")
    return out


def raster_atomics(wct, wl, t_mean_ms, t_fluct_ms, tile=None):
    """The raster's atomic adds against the chip's peaks (the probes): the mean raster makes
    one LDS add per window cell (counted on the host); the fluctuated raster's LDS and
    device-memory atomic instructions come from the committed counters of this build."""
    lds_peak, _ = wct.probe_atomic_add("lds", blocks=2048, iters=256)
    glob_peak, _ = wct.probe_atomic_add("global", blocks=2048, iters=32, buf_elems=2048 * 256 * 2)
    out = {"lds_peak_adds_per_s": lds_peak, "global_peak_adds_per_s": glob_peak,
           "probe": "wct_probe_atomic_add: 2048 blocks x 256 threads, a wave's 64 lanes on 64 consecutive floats; "
                    "device-memory adds over a 4 MiB buffer (L2)"}
    if t_mean_ms:
        cells = window_cells(wl)
        rate = cells / (t_mean_ms * 1e-3)
        out["mean_raster"] = {"lds_adds": cells, "ms": t_mean_ms, "adds_per_s": rate, "frac_of_lds_peak": rate / lds_peak}
    c = measured_counters("raster_tile_fluct", tile)
    if c and t_fluct_ms:
        lds_i = c["SQ_INSTS_LDS_ATOMIC"]
        out["fluct_raster"] = {"lds_atomic_instructions": lds_i,
                               "lds_atomic_lane_ops_upper": 64 * lds_i,
                               "frac_of_lds_peak_upper": 64 * lds_i / (t_fluct_ms * 1e-3) / lds_peak,
                               "l2_atomics": c["TCC_ATOMIC"],
                               "note": "counters of the committed profile for this build; lane ops bounded by 64 per "
                                       "wave instruction"}
    return out


def raster_issue(t_ms, alg_ops, tile=None):
    """Issued instructions of the fluctuated tile raster (committed counters of this build)
    against the cost model's lane operations."""
    c = measured_counters("raster_tile_fluct", tile)
    if not c or not t_ms:
        return None
    slots = 64 * c["SQ_INSTS_VALU"]
    return {"valu_instructions": c["SQ_INSTS_VALU"], "salu_instructions": c["SQ_INSTS_SALU"],
            "lds_instructions": c["SQ_INSTS_LDS"], "lane_use": c.get("lane_use"),
            "valu_lane_slots_per_alg_op": slots / alg_ops if alg_ops else None,
            "issued_per_s": (c["SQ_INSTS_VALU"] + c["SQ_INSTS_SALU"]) / (t_ms * 1e-3)}


def noise_cost(wct, synth, plan, dd, wl, wave, steps=3):
    """The headline step with each plane's noise (Eq. 1's N term) added: time per step and
    the inverse row transform's time with and without it."""
    import torch
    for p in range(len(wl.planes)):
        plan.set_noise(p, synth.noise_amplitude(plan.plane_info(p)["lt"], 300.0))
    on = wct.opts(wl.nsigma, True, 1, wl.seed, noise=True)
    plan.simulate(dd, on, wave)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_reset()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.simulate(dd, on, wave)
    e1.record()
    torch.cuda.synchronize()
    k = plan.profile_read()
    plan.profile(False)
    for p in range(len(wl.planes)):
        plan.set_noise(p, None)
    return {"ms_per_step": e0.elapsed_time(e1) / steps, "rows_c2r_ms": k["rows_c2r"][0] / steps,
            "spectrum": "synth.noise_amplitude(L_t, rms=300): shaped electronics-like noise, white floor 5%"}


def drift_cost(wct, synth, plan, reps=5):
    """wct_drift of the track workload's 1e5 3D depositions onto the three planes (FP32):
    mean time over `reps` calls from HIP events on the launch stream, and its HBM rate on
    algorithmic bytes (7 values read per deposition; 5 values and 3 ints written per row)."""
    import torch
    pts, det, prm, _ = synth.config2_points()
    dp = wct.DevicePoints.from_numpy(pts, "cuda:0", torch.float32)
    params = wct.drift_params(**prm)
    rows = plan.drift(dp, params)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.drift(dp, params, rows)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = dp.n * 4 * 7 + rows.n * (4 * 5 + 4 * 3)
    return {"ms": ms, "depositions": dp.n, "rows": rows.n, "alg_bytes": alg, "GBps": alg / (ms * 1e-3) / 1e9,
            "note": "launch-bound at this size (a few MB); drift speed 0.16 cm/us, D_L 6.2e-6 and D_T 1.32e-5 "
                    "cm^2/us, lifetime 10 ms"}


def adc_cost(plan, wave, reps=5):
    """ADC digitisation of the step's waveforms (wct_digitize, one 12-bit converter per
    plane): mean time over `reps` calls from HIP events on the launch stream, and its HBM
    rate on algorithmic bytes (each sample read once, its 16-bit code written once)."""
    import torch
    for p in range(plan.n_planes):
        plan.set_adc(p, 1.0 / 40.0, 400.0 if p < 2 else 900.0, 4095)
    adc = plan.digitize(wave, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.digitize(wave, 1, adc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = plan.wave_elems * (wave.element_size() + 2)
    return {"ms": ms, "alg_bytes": alg, "GBps": alg / (ms * 1e-3) / 1e9,
            "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "converter": "gain 1/40 count per unit of M, pedestal 400 (induction) / 900 (collection), 12 bits"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the backward-ratio and batching measurements")
    ap.add_argument("--showers-only", action="store_true",
                    help="time only the shower workload (two faces, 1e6 depositions) and print its JSON")
    ap.add_argument("--summarize", metavar="DIR", help="write profiles/ summaries from rocprofv3 output in DIR")
    ap.add_argument("--tune-cache", metavar="FILE", help="transform-variant choices: read from / appended to FILE")
    ap.add_argument("--raster-tile", metavar="RxTxB",
                    help="use this raster tile shape (rows x ticks x blocks per CU) instead of the tuner's choice "
                         "(the counter runs fix the shape their per-launch figures hold for)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (a known-size reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); events and planes shard "
              "across GPUs without communication, so per-GPU throughput is the single-GPU figure.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2104_08265_amd import synth, wct

    if args.showers_only:
        print(json.dumps(shower_bench(wct, synth, args.tune_cache, steps=args.steps)), flush=True)
        return
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    wl = synth.config2()
    plan = wct.Plan(wl.planes, synth.round_responses(wl), dtype="f32")
    dd = wct.DeviceDepos.from_numpy(wl.depos, "cuda:0", torch.float32)
    o = wct.opts(wl.nsigma, True, 1, wl.seed)
    fft_choice = plan.tune(1, args.tune_cache)  # transform variant per plane and axis, timed on this GPU
    tiles = {v["index"]: v for v in wct.tile_variants()}
    if args.raster_tile:
        want = tuple(int(x) for x in args.raster_tile.split("x"))
        tile = next(i for i, v in tiles.items() if v["dtype"] == "f32" and (v["th"], v["tw"], v["blocks_per_cu"]) == want)
        plan.set_tile(tile)
    else:
        tile = plan.tune_raster(dd, o, args.tune_cache)  # raster tile shape, timed on this event's rows
    tile_shape = {"rows": tiles[tile]["th"], "ticks": tiles[tile]["tw"], "blocks_per_cu": tiles[tile]["blocks_per_cu"]}
    variants = {v["index"]: v for v in wct.fft_variants()}
    fft_desc = {f"plane{p}_{'ticks' if k == 0 else 'wires'}":
                ("direct 21-wire sums" if v == wct.WCT_WIRE_DIRECT else "runtime" if v < 0
                 else f"{variants[v]['threads']} threads, radices {variants[v]['radices']}")
                for (p, k), v in sorted(fft_choice.items())}
    wave = plan.new_wave(1)
    plan.workspace(wct.OP_SIMULATE, 1, dd.n)
    for _ in range(args.warmup):
        plan.simulate(dd, o, wave)
    torch.cuda.synchronize()

    plan.profile(True)
    plan.profile_reset()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        plan.simulate(dd, o, wave)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    kt = plan.profile_read()
    # after the timed region: the mean raster of the same event (its LDS adds for the
    # atomic-throughput evidence), the normal-approximation raster (Box-Muller mode), then
    # the same step with noise added
    plan.profile_reset()
    plan.raster(dd, wct.opts(wl.nsigma, False, 1, wl.seed))
    torch.cuda.synchronize()
    t_mean = plan.profile_read().get("raster_tile_mean", (None, 0))[0]
    o_norm = wct.opts(wl.nsigma, wct.FLUCT_NORMAL, 1, wl.seed)
    plan.raster(dd, o_norm)
    plan.profile_reset()
    for _ in range(3):
        plan.raster(dd, o_norm)
    torch.cuda.synchronize()
    t_normal = plan.profile_read().get("raster_tile_normal", (None, 0))[0]
    t_normal = t_normal / 3 if t_normal is not None else None
    plan.profile(False)
    noise = noise_cost(wct, synth, plan, dd, wl, wave)
    adc = adc_cost(plan, wave)
    drift = drift_cost(wct, synth, plan)

    n_depos = wl.n_depos
    n_planes = len(wl.planes)
    alg = algorithmic_bytes(plan)
    kernels = {}
    for name, (tot, cnt) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        k = {"ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps}
        if name in alg and tot > 0:
            gbs = alg[name] * args.steps / (tot * 1e-3) / 1e9
            k.update({"alg_bytes_per_step": alg[name], "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS})
        mt = measured_traffic(name, tile_shape)
        if mt and tot > 0 and cnt > 0:  # counter bytes (FETCH_SIZE + WRITE_SIZE) per launch of this build
            cgbs = mt * cnt / (tot * 1e-3) / 1e9
            k.update({"counter_bytes_per_launch": mt, "counter_GBps": cgbs, "counter_hbm_frac": cgbs / HBM_PEAK_GBS})
        mc = measured_counters(name, tile_shape)
        if mc and tot > 0 and cnt > 0:  # VALU issue: SQ_INSTS_VALU wave instructions x 64 lanes per launch
            k["valu_issue_frac"] = mc["SQ_INSTS_VALU"] * 64 / ((tot / cnt) * 1e-3 * ALU_PEAK_TOPS * 1e12)
        kernels[name] = k
    t_raster = sum(v["ms_per_step"] for k, v in kernels.items() if k.startswith("raster"))
    t_conv = sum(v["ms_per_step"] for k, v in kernels.items() if k in ("rows_r2c", "colpass", "rows_c2r"))
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    # roofline of the dominant kernel: the fluctuated raster is bound by lane arithmetic
    # (Philox products and the FP64 sampler), the transform passes by HBM
    fft_dom = max(("rows_r2c", "colpass", "rows_c2r"), key=lambda k: kernels.get(k, {}).get("ms_per_step", 0))
    kd = kernels[fft_dom]
    roofline_fft = {"kernel": fft_dom, "bound": "hbm", "achieved": kd["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": kd["GBps"] / HBM_PEAK_GBS, "traffic": measured_traffic(fft_dom),
                    "alg_bytes_per_launch": alg[fft_dom] / n_planes,
                    "avg_launch_ms": kd["ms_per_step"] / kd["launches_per_step"],
                    "valu_issue_frac": kd.get("valu_issue_frac")}
    if dom == "raster_tile_fluct":
        ops = raster_alu_ops(wl)
        t = kernels[dom]["ms_per_step"] * 1e-3
        roofline = {"kernel": dom, "bound": "alu", "achieved": ops / t / 1e12, "peak": ALU_PEAK_TOPS,
                    "unit": "Tops/s", "frac": ops / t / 1e12 / ALU_PEAK_TOPS, "traffic": measured_traffic(dom, tile_shape),
                    "alg_ops_per_launch": ops, "avg_launch_ms": kernels[dom]["ms_per_step"],
                    "note": "algorithmic lane operations (bench.raster_alu_ops cost model) / mean launch time "
                            "from HIP events on the launch stream; peak = 256 CUs x 64 lanes x 2.4 GHz"}
    else:
        roofline = dict(roofline_fft)
    roofline_fft["note"] = "algorithmic bytes / mean launch time from HIP events on the launch stream"
    conv_bytes = sum(alg[k] for k in ("rows_r2c", "colpass", "rows_c2r"))
    grid_bytes = 4 * sum(i["n_impacts"] * i["n_wires"] * i["n_ticks"] for i in plan.info)
    wave_bytes = 4 * sum(i["n_wires"] * i["n_ticks"] for i in plan.info)

    out = {
        "metric": "depos/s + planes/s (raster+FFT conv) on 1 MI355X; fwd+bwd/fwd ratio; %HBM peak",
        "value": n_depos / (ms * 1e-3),
        "unit": "depos/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3 planes (2400+2400+3456 wires) x 9600 ticks, 10 impacts/pitch, 1e5 depositions "
                               "on 50 seeded tracks, binomial fluctuation on",
                   "n_depos": n_depos, "n_rows": dd.n, "planes": n_planes, "events": 1},
        "planes_per_s": n_planes / (ms * 1e-3),
        "t_raster_ms": t_raster,
        "t_conv_ms": t_conv,
        "conv_hbm_frac_algorithmic": (grid_bytes + wave_bytes) / (t_conv * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "conv_pass_bytes_GBps": conv_bytes / (t_conv * 1e-3) / 1e9,
        "dominant_kernel": dom,
        "kernels": kernels,
        "roofline": roofline,
        "roofline_fft": roofline_fft,
        "fft_plans": fft_desc,
        "raster_tile": tile_shape,
        "raster_atomics": raster_atomics(wct, wl, t_mean, kernels.get("raster_tile_fluct", {}).get("ms_per_step"),
                                         tile_shape),
        "raster_issue": raster_issue(kernels.get("raster_tile_fluct", {}).get("ms_per_step"),
                                     roofline.get("alg_ops_per_launch"), tile_shape),
        "issue_rates": issue_rates(wct),
        "noise": noise,
        "adc": adc,
        "drift": drift,
        "fluct_modes": {"tile_ms": {"mean": t_mean, "binomial": kernels.get("raster_tile_fluct", {}).get("ms_per_step"),
                                    "normal_box_muller": t_normal},
                        "note": "k_tile time of the same event per raster mode (tile shape tuned for the "
                                "binomial mode); the normal mode replaces each binomial count by its normal "
                                "approximation with Box-Muller normals (Sec. 4.3.1)"},
        "paper_context": PAPER_CONTEXT,
        "build": built_digest(),
    }
    plan.close()
    if not args.no_extras:
        out["fwd_bwd"] = fwd_bwd_ratio(wct, synth)
        out["batch"] = batch_bench(wct, synth)
        out["showers"] = shower_bench(wct, synth, args.tune_cache)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl)
        cb["cores_available"] = os.cpu_count()
        out["cpu_baseline"] = cb
        out["cpu_parallel"] = cpu_parallel_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
