"""Seeded synthetic workloads: depositions, plane geometries and wire responses.

This module generates inputs only.  It holds none of the simulation's arithmetic
(no rasterisation, no transform, no fluctuation): both the HIP path and the FP64
oracle receive the arrays produced here.

The paper's own inputs (cosmic-ray depositions from CORSIKA + Geant4 via LArSoft,
Sec. 4.3.2, and the real Wire-Cell field/electronics responses, Sec. 2) are not
available, so seeded stand-ins with the same structure are generated:

* straight tracks sampled densely along their length (cosmic-muon-like),
* electromagnetic-shower-like clusters (exponential depth, Gaussian lateral spread),
* uniform point clouds in the (pitch, tick) plane,
* per-plane responses R[k][i][tau] over 2K+1 wires x I impact positions x T_R ticks:
  unipolar (collection-like) or bipolar (induction-like), with per-(k, i) jitter so
  that no response is separable or mirror-symmetric.

Conventions (shared by every consumer): time in ticks, tick k covers [k, k+1);
pitch coordinate in wire pitches from the plane's lower grid edge, wire w sits at
p = w + 1/2, impact row b = I*w + i covers [b/I, (b+1)/I) in pitch units.
R[k][i][tau] is the response of wire w to unit charge in impact row I*(w+k)+i,
tau ticks after arrival.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2104082650

F32 = "f32"
F64 = "f64"


@dataclass
class Plane:
    """One readout plane: N_w wires x N_t ticks, I impacts per pitch, response extent."""

    n_wires: int
    n_ticks: int
    n_impacts: int = 10
    half_wires: int = 10  # K: response spans wires -K..K
    resp_ticks: int = 200  # T_R
    kind: str = "collection"  # or "induction"

    @property
    def n_rows(self) -> int:
        return self.n_impacts * self.n_wires


@dataclass
class Depos:
    """Structure-of-arrays depo-plane rows (one row per deposition per plane)."""

    q: np.ndarray
    t: np.ndarray
    p: np.ndarray
    sigma_t: np.ndarray
    sigma_p: np.ndarray
    plane: np.ndarray
    event: np.ndarray
    depo_id: np.ndarray

    def __len__(self) -> int:
        return int(self.q.shape[0])

    def astype(self, dtype) -> "Depos":
        return Depos(*(a.astype(dtype) for a in (self.q, self.t, self.p, self.sigma_t, self.sigma_p)),
                     self.plane, self.event, self.depo_id)

    def select(self, mask) -> "Depos":
        return Depos(*(a[mask] for a in (self.q, self.t, self.p, self.sigma_t, self.sigma_p,
                                          self.plane, self.event, self.depo_id)))

    @staticmethod
    def concat(parts: list["Depos"]) -> "Depos":
        return Depos(*(np.concatenate([getattr(d, f) for d in parts]) for f in
                       ("q", "t", "p", "sigma_t", "sigma_p", "plane", "event", "depo_id")))


@dataclass
class Workload:
    name: str
    planes: list
    responses: list  # one float64 array [2K+1][I][T_R] per plane
    depos: Depos
    dtype: str = F32
    fluctuate: bool = False
    nsigma: float = 3.0
    seed: int = 0
    n_events: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n_depos(self) -> int:
        """Physical depositions (rows sharing (event, depo_id) are one deposition)."""
        key = self.depos.event.astype(np.int64) * (1 << 32) + self.depos.depo_id.astype(np.int64)
        return int(np.unique(key).size)


# ----------------------------------------------------------------------------
# responses
# ----------------------------------------------------------------------------

def make_response(plane: Plane, rng: np.random.Generator) -> np.ndarray:
    """Seeded synthetic response R[k][i][tau], k = -K..K stored at index k+K.

    Charge in impact row I*(w+k)+i sits at x = k + (i+1/2)/I - 1/2 pitches from wire
    w.  Transverse fall-off g(x) = exp(-x^2/2).  Time shape: collection
    (tau/ts)^4 exp(-tau/ts), ts = 8(1+0.1 eps) ticks; induction -(tau-100)/sr *
    exp(-(tau-100)^2/(2 sr^2)), sr = 10(1+0.1 eps) ticks, mean over tau removed.
    eps ~ N(0,1) per (k, i).
    """
    K, I, T = plane.half_wires, plane.n_impacts, plane.resp_ticks
    k = np.arange(-K, K + 1, dtype=np.float64)[:, None, None]
    i = np.arange(I, dtype=np.float64)[None, :, None]
    tau = np.arange(T, dtype=np.float64)[None, None, :]
    x = k + (i + 0.5) / I - 0.5
    eps = rng.standard_normal((2 * K + 1, I, 1))
    g = np.exp(-0.5 * x * x)
    if plane.kind == "collection":
        ts = 8.0 * (1.0 + 0.1 * eps)
        f = (tau / ts) ** 4 * np.exp(-tau / ts)
    elif plane.kind == "induction":
        sr = 10.0 * (1.0 + 0.1 * eps)
        d = (tau - 0.5 * T) / sr
        f = -d * np.exp(-0.5 * d * d)
        f = f - f.mean(axis=2, keepdims=True)
    else:
        raise ValueError(plane.kind)
    return np.ascontiguousarray(g * f)


# ----------------------------------------------------------------------------
# charge laws
# ----------------------------------------------------------------------------

def lognormal_charge(rng, n, mean):
    """Lognormal with sigma_ln = 0.5 and the stated mean."""
    return rng.lognormal(math.log(mean) - 0.125, 0.5, n)


MOYAL_MEAN = 0.5772156649015329 + math.log(2.0)


def moyal_charge(rng, n, mean):
    """Landau-like (Moyal) charge: X = -ln Z^2, Z ~ N(0,1); Q = max(0, mean + 0.25 mean (X - E X))."""
    z = rng.standard_normal(n)
    x = -np.log(z * z)
    return np.maximum(0.0, mean + 0.25 * mean * (x - MOYAL_MEAN))


# ----------------------------------------------------------------------------
# 3D detectors and projection onto wire planes
# ----------------------------------------------------------------------------

@dataclass
class Detector:
    """A drift volume x in [0, x_max], y in [0, H], z in [0, W] read by planes of given angles."""

    x_max: float
    height: float
    width: float
    angles_deg: tuple
    pitch_cm: float
    planes: list
    cm_per_tick: float = 0.08  # 1.6 mm/us drift speed x 0.5 us ticks
    t0_max: float = 0.0

    def project(self, xyz: np.ndarray, t0: np.ndarray):
        """Per plane: pitch coordinate (pitches), time (ticks), sigma_t, sigma_p."""
        x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
        frac = np.clip(x / self.x_max, 0.0, 1.0)
        t = t0 + x / self.cm_per_tick
        st = 1.0 + 2.0 * np.sqrt(frac)
        sp = 0.3 + 1.7 * np.sqrt(frac)
        out = []
        for ang, pl in zip(self.angles_deg, self.planes):
            a = math.radians(ang)
            p = ((z - 0.5 * self.width) * math.cos(a) + (y - 0.5 * self.height) * math.sin(a)) / self.pitch_cm \
                + 0.5 * pl.n_wires
            out.append((p, t, st, sp))
        return out

    def inside_all(self, xyz, margin):
        ok = np.ones(len(xyz), bool)
        for (p, _, _, _), pl in zip(self.project(xyz, np.zeros(len(xyz))), self.planes):
            ok &= (p > margin) & (p < pl.n_wires - margin)
        return ok


def detector_uboone_like(n_ticks=9600, wires=(2400, 2400, 3456)) -> Detector:
    planes = [Plane(wires[0], n_ticks, kind="induction"), Plane(wires[1], n_ticks, kind="induction"),
              Plane(wires[2], n_ticks, kind="collection")]
    pitch = 0.3
    width = pitch * wires[2]
    # choose H so the +-60 degree planes exactly span the box
    height = (pitch * wires[0] - width * 0.5) / math.sin(math.radians(60.0))
    x_max = 256.0 * min(1.0, n_ticks / 9600.0)  # drift length shrinks with a shorter readout window
    return Detector(x_max=x_max, height=height, width=width, angles_deg=(60.0, -60.0, 0.0),
                    pitch_cm=pitch, planes=planes, t0_max=max(0.0, n_ticks - x_max / 0.08 - 100.0))


def detector_dune_like(n_ticks=6000, wires=(800, 800, 960)) -> Detector:
    planes = [Plane(wires[0], n_ticks, kind="induction"), Plane(wires[1], n_ticks, kind="induction"),
              Plane(wires[2], n_ticks, kind="collection")]
    pitch = 0.47
    x_max = 360.0 * min(1.0, n_ticks / 6000.0)
    return Detector(x_max=x_max, height=300.0 * min(1.0, wires[2] / 960.0), width=pitch * wires[2],
                    angles_deg=(35.7, -35.7, 0.0), pitch_cm=pitch, planes=planes,
                    t0_max=max(0.0, n_ticks - x_max / 0.08 - 100.0))


def _rows_from_points(det: Detector, xyz, t0, q, event, depo_ids, plane_offset=0) -> Depos:
    parts = []
    for j, (p, t, st, sp) in enumerate(det.project(xyz, t0)):
        n = len(q)
        parts.append(Depos(q.copy(), t, p, st, sp, np.full(n, plane_offset + j, np.int32),
                           np.full(n, event, np.int32), depo_ids.astype(np.int32)))
    return Depos.concat(parts)


def _isotropic(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def track_points(rng, det: Detector, n_tracks: int, n_points: int, lmin=10.0, lmax=200.0):
    """n_points spread evenly (in length) over n_tracks straight tracks inside the box."""
    ext = np.array([det.x_max, det.height, det.width])
    lmax = min(lmax, 0.95 * float(ext.min()))  # small test boxes: tracks still fit
    lmin = min(lmin, 0.5 * lmax)
    L = rng.uniform(lmin, lmax, n_tracks)
    d = _isotropic(rng, n_tracks)
    start = np.empty((n_tracks, 3))
    for a in range(3):
        span = L * d[:, a]
        lo = np.maximum(0.0, -span)
        hi = np.minimum(ext[a], ext[a] - span)
        start[:, a] = rng.uniform(lo, hi)
    t0 = rng.uniform(0.0, det.t0_max, n_tracks)
    # equal step along every track: step = sum(L) / n_points
    cum = np.concatenate([[0.0], np.cumsum(L)])
    s = (np.arange(n_points) + 0.5) * (cum[-1] / n_points)
    tid = np.clip(np.searchsorted(cum, s, side="right") - 1, 0, n_tracks - 1)
    along = s - cum[tid]
    xyz = start[tid] + along[:, None] * d[tid]
    return xyz, t0[tid]


def shower_points(rng, det: Detector, n_showers: int, n_points: int, depth_cm=14.0, lateral_cm=2.0,
                  margin=80.0):
    """EM-shower-like clusters: exponential depth along a random axis, Gaussian lateral spread."""
    ext = np.array([det.x_max, det.height, det.width])
    verts = []
    while len(verts) < n_showers:
        cand = rng.uniform(0.0, 1.0, (64, 3)) * ext
        cand[:, 0] = rng.uniform(0.05 * det.x_max, 0.95 * det.x_max, 64)
        for c in cand[det.inside_all(cand, margin)]:
            if len(verts) < n_showers:
                verts.append(c)
    verts = np.array(verts)
    axes = _isotropic(rng, n_showers)
    t0 = rng.uniform(0.0, det.t0_max, n_showers)
    sid = np.arange(n_points) % n_showers
    d = axes[sid]
    # orthonormal frame per shower
    helper = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(d, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(d, e1)
    depth = rng.exponential(depth_cm, n_points)
    l1 = rng.normal(0.0, lateral_cm, n_points)
    l2 = rng.normal(0.0, lateral_cm, n_points)
    xyz = verts[sid] + depth[:, None] * d + l1[:, None] * e1 + l2[:, None] * e2
    xyz[:, 0] = np.clip(xyz[:, 0], 0.0, det.x_max)
    return xyz, t0[sid], sid


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def _rng(c):
    return np.random.Generator(np.random.PCG64(SEED_BASE + c))


def _finish(depos: Depos, dtype: str) -> Depos:
    """Round the float inputs to the working precision once; both sides widen from these."""
    if dtype == F32:
        return depos.astype(np.float32)
    return depos.astype(np.float64)


def uniform_points(rng, plane_idx: int, plane: Plane, n: int, mean_q=5000.0, event=0) -> Depos:
    p = rng.uniform(0.0, plane.n_wires, n)
    t = rng.uniform(0.0, plane.n_ticks, n)
    q = lognormal_charge(rng, n, mean_q)
    st = rng.uniform(1.0, 3.0, n)
    sp = rng.uniform(0.3, 2.0, n)
    return Depos(q, t, p, st, sp, np.full(n, plane_idx, np.int32), np.full(n, event, np.int32),
                 np.arange(n, dtype=np.int32))


def config1(n_depos=1000, n_wires=256, n_ticks=1024) -> Workload:
    """One collection plane 256 wires x 1024 ticks, 1000 uniform points, FP64, no fluctuation."""
    rng = _rng(1)
    pl = Plane(n_wires, n_ticks, kind="collection")
    resp = [make_response(pl, rng)]
    d = uniform_points(rng, 0, pl, n_depos)
    return Workload("config1", [pl], resp, _finish(d, F64), dtype=F64, fluctuate=False, seed=1)


def config2(n_depos=100_000, n_tracks=50, n_ticks=9600, wires=(2400, 2400, 3456), dtype=F32,
            fluctuate=True) -> Workload:
    """Three planes (2400+2400+3456 wires x 9600 ticks), 1e5 depos on 50 tracks, FP32, fluctuation on."""
    rng = _rng(2)
    det = detector_uboone_like(n_ticks, wires)
    resp = [make_response(pl, rng) for pl in det.planes]
    xyz, t0 = track_points(rng, det, n_tracks, n_depos)
    q = moyal_charge(rng, n_depos, 6000.0)
    d = _rows_from_points(det, xyz, t0, q, 0, np.arange(n_depos))
    return Workload("config2", det.planes, resp, _finish(d, dtype), dtype=dtype, fluctuate=fluctuate, seed=2)


@dataclass
class Points:
    """3D depositions before the drift (structure of arrays): position (cm; x is the
    distance to the readout planes), time (us), electrons, initial extents (cm)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    t0: np.ndarray
    q: np.ndarray
    sigma_l: np.ndarray
    sigma_t: np.ndarray
    event: np.ndarray
    depo_id: np.ndarray

    def astype(self, dtype) -> "Points":
        f = lambda a: a.astype(dtype)
        return Points(f(self.x), f(self.y), f(self.z), f(self.t0), f(self.q), f(self.sigma_l), f(self.sigma_t),
                      self.event, self.depo_id)


def drift_params(det: Detector, tick_us=0.5, diffusion_l=6.2e-6, diffusion_t=13.2e-6, lifetime_us=10000.0):
    """Drift constants of a detector as plain numbers: liquid-argon-like longitudinal and
    transverse diffusion (cm^2/us) and electron lifetime, the detector's drift speed
    (cm_per_tick / tick), and per plane its wire-normal angle (radians), pitch, the pitch
    coordinate of y = z = 0 (the projection of Detector.project) and a zero time offset."""
    angles = [math.radians(a) for a in det.angles_deg]
    offsets = [0.5 * pl.n_wires - (0.5 * det.width * math.cos(a) + 0.5 * det.height * math.sin(a)) / det.pitch_cm
               for a, pl in zip(angles, det.planes)]
    return {"drift_speed": det.cm_per_tick / tick_us, "diffusion_l": diffusion_l, "diffusion_t": diffusion_t,
            "lifetime": lifetime_us, "tick": tick_us, "angles": tuple(angles),
            "pitches": tuple(det.pitch_cm for _ in angles), "wire_offsets": tuple(offsets),
            "time_offsets": tuple(0.0 for _ in angles)}


def config2_points(n_depos=100_000, n_tracks=50, n_ticks=9600, wires=(2400, 2400, 3456), dtype=F32):
    """The three-plane track workload before the drift: 1e5 3D depositions on 50 seeded
    straight tracks in the drift volume, initial extents 0.03-0.06 cm.  Returns (points,
    detector, drift constants, responses)."""
    rng = _rng(6)
    det = detector_uboone_like(n_ticks, wires)
    resp = [make_response(pl, rng) for pl in det.planes]
    xyz, t0 = track_points(rng, det, n_tracks, n_depos)
    q = moyal_charge(rng, n_depos, 6000.0)
    prm = drift_params(det)
    pts = Points(xyz[:, 0], xyz[:, 1], xyz[:, 2], t0 * prm["tick"], q, rng.uniform(0.03, 0.06, n_depos),
                 rng.uniform(0.03, 0.06, n_depos), np.zeros(n_depos, np.int32), np.arange(n_depos, dtype=np.int32))
    return pts.astype(np.float32 if dtype == F32 else np.float64), det, prm, resp


def config3(n_depos=1_000_000, n_showers=20, n_ticks=6000, wires=(800, 800, 960), dtype=F32,
            fluctuate=True) -> Workload:
    """Two faces x (800+800+960 wires) x 6000 ticks, 1e6 depos in 20 showers, FP32, fluctuation on."""
    rng = _rng(3)
    det = detector_dune_like(n_ticks, wires)
    planes = list(det.planes) + [Plane(pl.n_wires, pl.n_ticks, kind=pl.kind) for pl in det.planes]
    resp = [make_response(pl, rng) for pl in planes]
    xyz, t0, sid = shower_points(rng, det, n_showers, n_depos)
    q = lognormal_charge(rng, n_depos, 3000.0)
    face = sid % 2
    parts = []
    ids = np.arange(n_depos)
    for f in (0, 1):
        m = face == f
        parts.append(_rows_from_points(det, xyz[m], t0[m], q[m], 0, ids[m], plane_offset=3 * f))
    d = Depos.concat(parts)
    return Workload("config3", planes, resp, _finish(d, dtype), dtype=dtype, fluctuate=fluctuate, seed=3)


def config4(n_depos=20_000, n_tracks=20, n_wires=256, n_ticks=1024) -> Workload:
    """Config-1 geometry, 2e4 depos on straight tracks in the (pitch, tick) plane, FP32, no fluctuation.

    extra["target_depos"] holds the seeded perturbation used to simulate the target waveform:
    Q x N(1, 0.05), t + N(0, 0.5) ticks, p + N(0, 0.2) pitches.
    """
    rng = _rng(4)
    pl = Plane(n_wires, n_ticks, kind="collection")
    resp = [make_response(pl, rng)]
    a = rng.uniform([0, 0], [n_wires, n_ticks], (n_tracks, 2))
    b = rng.uniform([0, 0], [n_wires, n_ticks], (n_tracks, 2))
    tid = np.arange(n_depos) % n_tracks
    s = rng.uniform(0.0, 1.0, n_depos)
    pt = a[tid] + s[:, None] * (b[tid] - a[tid])
    q = lognormal_charge(rng, n_depos, 5000.0)
    st = rng.uniform(1.0, 3.0, n_depos)
    sp = rng.uniform(0.3, 2.0, n_depos)
    d = Depos(q, pt[:, 1], pt[:, 0], st, sp, np.zeros(n_depos, np.int32), np.zeros(n_depos, np.int32),
              np.arange(n_depos, dtype=np.int32))
    tgt = Depos(q * rng.normal(1.0, 0.05, n_depos), pt[:, 1] + rng.normal(0.0, 0.5, n_depos),
                pt[:, 0] + rng.normal(0.0, 0.2, n_depos), st, sp, d.plane, d.event, d.depo_id)
    return Workload("config4", [pl], resp, _finish(d, F32), dtype=F32, fluctuate=False, seed=4,
                    extra={"target_depos": _finish(tgt, F32)})


def event_depo_counts(rng, n_events, lo=1e2, hi=2e5):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_events))).astype(np.int64)


def config5(n_events=64, lo=1e2, hi=2e5, n_ticks=9600, wires=(2400, 2400, 3456), dtype=F32,
            fluctuate=True) -> Workload:
    """64 events on the config-2 geometry, depo counts log-uniform in [1e2, 2e5], tracks or showers."""
    rng = _rng(5)
    det = detector_uboone_like(n_ticks, wires)
    resp = [make_response(pl, rng) for pl in det.planes]
    counts = event_depo_counts(rng, n_events, lo, hi)
    parts = []
    kinds = []
    for e, n in enumerate(counts):
        n = int(n)
        if rng.uniform() < 0.5:
            xyz, t0 = track_points(rng, det, max(1, math.ceil(n / 2000)), n)
            q = moyal_charge(rng, n, 6000.0)
            kinds.append("track")
        else:
            xyz, t0, _ = shower_points(rng, det, max(1, math.ceil(n / 50_000)), n, margin=60.0)
            q = lognormal_charge(rng, n, 3000.0)
            kinds.append("shower")
        parts.append(_rows_from_points(det, xyz, t0, q, e, np.arange(n)))
    d = Depos.concat(parts)
    return Workload("config5", det.planes, resp, _finish(d, dtype), dtype=dtype, fluctuate=fluctuate, seed=5,
                    n_events=n_events, extra={"counts": counts, "kinds": kinds})


def tiny(n_wires=6, n_ticks=40, half_wires=2, resp_ticks=12, n_impacts=10, n_depos=12, seed=7, dtype=F64,
         kind="collection", sigma_scale=1.0) -> Workload:
    """A tiny single-plane workload for brute-force checks."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 100 + seed))
    pl = Plane(n_wires, n_ticks, n_impacts=n_impacts, half_wires=half_wires, resp_ticks=resp_ticks, kind=kind)
    resp = [make_response(pl, rng)]
    p = rng.uniform(-0.5, n_wires + 0.5, n_depos)
    t = rng.uniform(-2.0, n_ticks + 2.0, n_depos)
    q = lognormal_charge(rng, n_depos, 2000.0)
    st = rng.uniform(0.6, 2.0, n_depos) * sigma_scale
    sp = rng.uniform(0.1, 0.6, n_depos) * sigma_scale
    d = Depos(q, t, p, st, sp, np.zeros(n_depos, np.int32), np.zeros(n_depos, np.int32),
              np.arange(n_depos, dtype=np.int32))
    return Workload("tiny", [pl], resp, _finish(d, dtype), dtype=dtype, seed=seed)


def round_responses(wl: Workload):
    """Responses as the plan consumes them: rounded to the working precision once."""
    dt = np.float32 if wl.dtype == F32 else np.float64
    return [np.ascontiguousarray(r.astype(dt)) for r in wl.responses]


def noise_amplitude(lt: int, rms: float, shaping_ticks: float = 2.0, white: float = 0.05) -> np.ndarray:
    """Synthetic noise amplitude spectrum A[k], k = 0..L_t/2, of an L_t-point tick transform.

    Shape (a stand-in for electronics noise after a shaping amplifier; the paper gives no
    spectrum): s(f) = (f / f0) exp(1 - f / f0) + white, f = k / L_t cycles per tick,
    f0 = 1 / (2 pi shaping_ticks), zero at DC; scaled so that the noise waveform's RMS is
    `rms` (Parseval: rms^2 = (A[0]^2 + 2 sum A[k]^2 + A[L/2]^2) / L^2).
    """
    F = lt // 2 + 1
    f = np.arange(F) / lt
    f0 = 1.0 / (2.0 * np.pi * shaping_ticks)
    s = (f / f0) * np.exp(1.0 - f / f0) + white
    s[0] = 0.0
    power = (s[0] ** 2 + 2.0 * np.sum(s[1:-1] ** 2) + s[-1] ** 2) / lt ** 2
    return s * (rms / np.sqrt(power))
