"""ctypes binding of libwct.so: the C ABI of include/wct.h with the same call names.

Argument marshalling only: every step of the simulation runs in the library's HIP
kernels.  Device memory and streams come from PyTorch (tensors' data pointers and the
current HIP stream).  Importing this module loads the library and raises ImportError if
it has not been built (python -m paper_2104_08265_amd.build).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

# torch is imported first so that its bundled HIP runtime is the one in the process:
# libwct.so's dependency on libamdhip64.so.7 then resolves (by soname) to that same
# runtime, and torch's device pointers and streams are valid in the library's calls.
import torch  # noqa: F401  (load order matters)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwct.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2104_08265_amd.build`")
lib = ctypes.CDLL(LIB_PATH)

WCT_F32, WCT_F64 = 0, 1
WCT_WIRE_DIRECT = -2  # wct_plan_set_fft kind 1: direct sums over the response's 21 wires
WCT_OK, WCT_E_INVALID, WCT_E_WORKSPACE, WCT_E_DEVICE, WCT_E_UNSUPPORTED, WCT_E_NOMEM = 0, -1, -2, -3, -4, -5
OP_RASTER, OP_CONVOLVE, OP_SIMULATE, OP_BACKWARD = 0, 1, 2, 3
STATUS = {0: "WCT_OK", -1: "WCT_E_INVALID", -2: "WCT_E_WORKSPACE", -3: "WCT_E_DEVICE", -4: "WCT_E_UNSUPPORTED",
          -5: "WCT_E_NOMEM"}


class wct_plane_desc(ctypes.Structure):
    _fields_ = [("n_wires", c_int32), ("n_ticks", c_int32), ("n_impacts", c_int32), ("half_wires", c_int32),
                ("resp_ticks", c_int32), ("response", c_void_p)]


class wct_plan_desc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("n_planes", c_int32), ("planes", POINTER(wct_plane_desc)),
                ("max_events", c_int32), ("device", c_int32)]


class wct_depos(ctypes.Structure):
    _fields_ = [("n", c_int64), ("q", c_void_p), ("t", c_void_p), ("p", c_void_p), ("sigma_t", c_void_p),
                ("sigma_p", c_void_p), ("plane", c_void_p), ("event", c_void_p), ("depo_id", c_void_p)]


MAX_PLANES = 8


class wct_depos3d(ctypes.Structure):
    _fields_ = [("n", c_int64), ("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("t0", c_void_p), ("q", c_void_p),
                ("sigma_l", c_void_p), ("sigma_t", c_void_p), ("event", c_void_p), ("depo_id", c_void_p)]


class wct_drift_params(ctypes.Structure):
    _fields_ = [("drift_speed", c_double), ("diffusion_l", c_double), ("diffusion_t", c_double),
                ("lifetime", c_double), ("tick", c_double), ("angle", c_double * MAX_PLANES),
                ("pitch", c_double * MAX_PLANES), ("wire_offset", c_double * MAX_PLANES),
                ("time_offset", c_double * MAX_PLANES)]


class wct_depos_out(ctypes.Structure):
    _fields_ = [("q", c_void_p), ("t", c_void_p), ("p", c_void_p), ("sigma_t", c_void_p), ("sigma_p", c_void_p),
                ("plane", c_void_p), ("event", c_void_p), ("depo_id", c_void_p)]


class wct_opts(ctypes.Structure):
    _fields_ = [("nsigma", c_double), ("fluctuate", c_int32), ("n_events", c_int32), ("seed", c_uint64),
                ("event_base", c_int32), ("noise", c_int32)]


PlanP = c_void_p


def _sig(name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


wct_plan_create = _sig("wct_plan_create", c_int32, [POINTER(wct_plan_desc), POINTER(c_void_p)])
wct_plan_destroy = _sig("wct_plan_destroy", None, [PlanP])
wct_grid_elems = _sig("wct_grid_elems", c_int64, [PlanP])
wct_wave_elems = _sig("wct_wave_elems", c_int64, [PlanP])
wct_plane_info = _sig("wct_plane_info", c_int32, [PlanP, c_int32, POINTER(c_int64)])
wct_workspace_bytes = _sig("wct_workspace_bytes", c_size_t, [PlanP, c_int32, c_int32, c_int64])
wct_raster = _sig("wct_raster", c_int32, [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_void_p, c_void_p, c_size_t,
                                         c_void_p])
wct_raster_noalloc = _sig("wct_raster_noalloc", c_int32, [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_void_p,
                                                         c_void_p])
NOALLOC_SCRATCH_BYTES = 128 << 20  # WCT_NOALLOC_SCRATCH_BYTES
wct_probe_atomic_add = _sig("wct_probe_atomic_add", c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int64,
                                                              POINTER(c_double), c_void_p])
wct_probe_issue_rate = _sig("wct_probe_issue_rate", c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int64,
                                                              POINTER(c_double), c_void_p])
wct_probe_last_error = _sig("wct_probe_last_error", c_char_p, [])
wct_convolve = _sig("wct_convolve", c_int32, [PlanP, c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p])
wct_simulate = _sig("wct_simulate", c_int32, [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_void_p, c_void_p,
                                             c_size_t, c_void_p])
wct_simulate_graph = _sig("wct_simulate_graph", c_int32, [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_void_p,
                                                         c_void_p, c_size_t, c_void_p])
wct_simulate_backward = _sig("wct_simulate_backward", c_int32,
                             [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
wct_last_error = _sig("wct_last_error", c_char_p, [])
wct_abi_version = _sig("wct_abi_version", c_int32, [])
wct_profile_enable = _sig("wct_profile_enable", c_int32, [PlanP, c_int32])
wct_profile_reset = _sig("wct_profile_reset", c_int32, [PlanP])
wct_profile_count = _sig("wct_profile_count", c_int32, [PlanP])
wct_profile_get = _sig("wct_profile_get", c_int32, [PlanP, c_int32, c_char_p, c_size_t, POINTER(c_double),
                                                   POINTER(c_int64)])
wct_fluct_spec_version = _sig("wct_fluct_spec_version", c_int32, [])
wct_fft_variant_count = _sig("wct_fft_variant_count", c_int32, [])
wct_fft_variant_info = _sig("wct_fft_variant_info", c_int32, [c_int32, POINTER(c_int32)])
wct_plan_get_fft = _sig("wct_plan_get_fft", c_int32, [PlanP, c_int32, c_int32, POINTER(c_int32)])
wct_plan_set_fft = _sig("wct_plan_set_fft", c_int32, [PlanP, c_int32, c_int32, c_int32])
wct_tile_variant_count = _sig("wct_tile_variant_count", c_int32, [])
wct_tile_variant_info = _sig("wct_tile_variant_info", c_int32, [c_int32, POINTER(c_int32)])
wct_plan_get_tile = _sig("wct_plan_get_tile", c_int32, [PlanP, POINTER(c_int32)])
wct_plan_set_tile = _sig("wct_plan_set_tile", c_int32, [PlanP, c_int32])
wct_tune_raster_workspace_bytes = _sig("wct_tune_raster_workspace_bytes", c_size_t, [PlanP, c_int32, c_int64])
wct_plan_tune_raster = _sig("wct_plan_tune_raster", c_int32, [PlanP, POINTER(wct_depos), POINTER(wct_opts), c_char_p,
                                                             c_void_p, c_size_t, c_void_p])
wct_plan_set_noise = _sig("wct_plan_set_noise", c_int32, [PlanP, c_int32, POINTER(c_double), c_int64])
wct_drift = _sig("wct_drift", c_int32, [PlanP, POINTER(wct_depos3d), POINTER(wct_drift_params),
                                         POINTER(wct_depos_out), c_void_p])
wct_plan_set_adc = _sig("wct_plan_set_adc", c_int32, [PlanP, c_int32, c_double, c_double, c_int32])
wct_digitize = _sig("wct_digitize", c_int32, [PlanP, c_void_p, c_int32, c_void_p, c_void_p])
wct_tune_workspace_bytes = _sig("wct_tune_workspace_bytes", c_size_t, [PlanP, c_int32])
wct_plan_tune = _sig("wct_plan_tune", c_int32, [PlanP, c_int32, c_char_p, c_void_p, c_size_t, c_void_p])


def probe_atomic_add(where, blocks=2048, iters=256, buf_elems=None, device=0):
    """Peak float atomic adds per second: where = "lds" (into LDS) or "global" (into device
    memory, performed at L2).  A measurement call: allocates a buffer and synchronises."""
    torch = _torch()
    n = blocks * 256 if buf_elems is None else int(buf_elems)
    buf = torch.zeros(n, dtype=torch.float32, device=f"cuda:{device}")
    rate = c_double()
    code = wct_probe_atomic_add(0 if where == "lds" else 1, blocks, iters, _ptr(buf), n, ctypes.byref(rate),
                                c_void_p(torch.cuda.current_stream(device).cuda_stream))
    if code != 0:
        raise WctError(code, f"wct_probe_atomic_add: {wct_probe_last_error().decode()}")
    return rate.value, buf


ISSUE_KINDS = ("fma_f32_vgpr", "fma_f32_sgpr", "fma_f64", "mad_u64_u32")


def probe_issue_rate(kind, blocks=None, iters=2048, device=0):
    """Lane operations per second of one instruction kind (ISSUE_KINDS, or its index): 16
    independent chains per thread over 16 blocks of 256 threads per CU.  A measurement
    call: allocates a buffer and synchronises."""
    torch = _torch()
    k = ISSUE_KINDS.index(kind) if isinstance(kind, str) else int(kind)
    if blocks is None:
        blocks = 16 * torch.cuda.get_device_properties(device).multi_processor_count
    buf = torch.empty(blocks * 256, dtype=torch.int64, device=f"cuda:{device}")
    rate = c_double()
    code = wct_probe_issue_rate(k, blocks, iters, _ptr(buf), buf.numel() * 8, ctypes.byref(rate),
                                c_void_p(torch.cuda.current_stream(device).cuda_stream))
    if code != 0:
        raise WctError(code, f"wct_probe_issue_rate: {wct_probe_last_error().decode()}")
    return rate.value


def tile_variants():
    """Compiled raster tile variants: list of dicts (index, dtype, th, tw, blocks_per_cu)."""
    out = []
    buf = (c_int32 * 4)()
    for k in range(wct_tile_variant_count()):
        check(wct_tile_variant_info(k, buf), "wct_tile_variant_info")
        out.append({"index": k, "dtype": "f64" if buf[0] else "f32", "th": buf[1], "tw": buf[2],
                    "blocks_per_cu": buf[3]})
    return out


def fft_variants():
    """Compiled transform variants: list of dicts (index, kind, dtype, threads, n, radices)."""
    out = []
    buf = (c_int32 * 12)()
    for k in range(wct_fft_variant_count()):
        check(wct_fft_variant_info(k, buf), "wct_fft_variant_info")
        v = list(buf)
        out.append({"index": k, "kind": v[0], "dtype": "f64" if v[1] else "f32", "threads": v[2], "n": v[3],
                    "radices": v[5:5 + v[4]]})
    return out


class WctError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}: {last_error()}")


def last_error() -> str:
    return (wct_last_error() or b"").decode()


def check(code, what="wct call"):
    if code != WCT_OK:
        raise WctError(code, what)
    return code


# ---------------------------------------------------------------------------
# torch-facing helpers (torch supplies device memory and the stream)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dt(dtype):
    torch = _torch()
    return torch.float32 if dtype == WCT_F32 else torch.float64


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


class DeviceDepos:
    """Depo-plane rows resident on the device (structure of arrays)."""

    def __init__(self, q, t, p, sigma_t, sigma_p, plane=None, event=None, depo_id=None):
        self.q, self.t, self.p, self.sigma_t, self.sigma_p = q, t, p, sigma_t, sigma_p
        self.plane, self.event, self.depo_id = plane, event, depo_id
        self.n = int(q.shape[0])
        for a in (t, p, sigma_t, sigma_p):
            if a.shape[0] != self.n or a.dtype != q.dtype or a.device != q.device or not a.is_contiguous():
                raise ValueError("depo float arrays must share length, dtype and device and be contiguous")
        for a in (plane, event, depo_id):
            if a is not None and (a.shape[0] != self.n or str(a.dtype) != "torch.int32" or not a.is_contiguous()):
                raise ValueError("plane/event/depo_id must be contiguous int32 of the same length")

    @staticmethod
    def from_numpy(d, device, dtype):
        """From an object with numpy fields q, t, p, sigma_t, sigma_p, plane, event, depo_id."""
        torch = _torch()
        f = lambda a: torch.as_tensor(a).to(device=device, dtype=dtype).contiguous()
        i = lambda a: torch.as_tensor(a.astype("int32")).to(device=device).contiguous()
        return DeviceDepos(f(d.q), f(d.t), f(d.p), f(d.sigma_t), f(d.sigma_p), i(d.plane), i(d.event), i(d.depo_id))

    def slice(self, a, b):
        """Rows a..b-1 as views (no copy)."""
        f = lambda x: x[a:b]
        return DeviceDepos(f(self.q), f(self.t), f(self.p), f(self.sigma_t), f(self.sigma_p), f(self.plane),
                           f(self.event), f(self.depo_id))

    def c(self):
        return wct_depos(self.n, _ptr(self.q), _ptr(self.t), _ptr(self.p), _ptr(self.sigma_t), _ptr(self.sigma_p),
                         _ptr(self.plane), _ptr(self.event), _ptr(self.depo_id))


class DevicePoints:
    """3D depositions resident on the device (wct_depos3d): x, y, z, t0, q, sigma_l, sigma_t
    in the plan dtype, event and depo_id int32 (or None)."""

    FIELDS = ("x", "y", "z", "t0", "q", "sigma_l", "sigma_t")

    def __init__(self, **arrays):
        for f in self.FIELDS + ("event", "depo_id"):
            setattr(self, f, arrays.get(f))
        self.n = int(self.x.shape[0])
        for f in self.FIELDS:
            a = getattr(self, f)
            if a.shape[0] != self.n or a.dtype != self.x.dtype or not a.is_contiguous():
                raise ValueError("point arrays must share length and dtype and be contiguous")

    @staticmethod
    def from_numpy(pts, device, dtype):
        torch = _torch()
        f = lambda a: torch.as_tensor(a).to(device=device, dtype=dtype).contiguous()
        i = lambda a: None if a is None else torch.as_tensor(a.astype("int32")).to(device=device).contiguous()
        return DevicePoints(**{k: f(getattr(pts, k)) for k in DevicePoints.FIELDS},
                            event=i(getattr(pts, "event", None)), depo_id=i(getattr(pts, "depo_id", None)))

    def c(self):
        return wct_depos3d(self.n, *(_ptr(getattr(self, f)) for f in self.FIELDS), _ptr(self.event),
                           _ptr(self.depo_id))


def drift_params(drift_speed, diffusion_l, diffusion_t, lifetime, tick, angles, pitches, wire_offsets,
                 time_offsets):
    """wct_drift_params from plain numbers (per-plane sequences: angle in radians, pitch,
    wire offset in pitches, time offset)."""
    prm = wct_drift_params(float(drift_speed), float(diffusion_l), float(diffusion_t), float(lifetime), float(tick))
    for k, (a, p, o, d) in enumerate(zip(angles, pitches, wire_offsets, time_offsets)):
        prm.angle[k], prm.pitch[k], prm.wire_offset[k], prm.time_offset[k] = a, p, o, d
    return prm


FLUCT_MEAN, FLUCT_BINOMIAL, FLUCT_NORMAL = 0, 1, 2


def opts(nsigma=3.0, fluctuate=False, n_events=1, seed=0, event_base=0, noise=False):
    """Run options; the call simulates events event_base .. event_base + n_events - 1.

    fluctuate: False / 0 the mean charge, True / 1 binomial counts, 2 (FLUCT_NORMAL) their
    normal approximation with Box-Muller normals; noise: wct_simulate adds the planes'
    noise (Plan.set_noise)."""
    return wct_opts(float(nsigma), int(fluctuate), int(n_events), int(seed) & 0xFFFFFFFFFFFFFFFF,
                    int(event_base), int(bool(noise)))


class Plan:
    """A wct_plan plus torch-allocated workspaces.

    planes: sequence of objects with n_wires, n_ticks, n_impacts, half_wires, resp_ticks;
    responses: one host array [2K+1][I][T_R] per plane (converted to the plan dtype).
    """

    def __init__(self, planes, responses, dtype="f32", max_events=1, device=0):
        import numpy as np
        self.dtype = WCT_F32 if dtype in ("f32", WCT_F32) else WCT_F64
        npdt = np.float32 if self.dtype == WCT_F32 else np.float64
        self._resp = [np.ascontiguousarray(np.asarray(r, dtype=npdt)) for r in responses]
        descs = (wct_plane_desc * len(planes))()
        for k, (pl, r) in enumerate(zip(planes, self._resp)):
            K = (r.shape[0] - 1) // 2
            if r.shape != (2 * K + 1, pl.n_impacts, r.shape[2]):
                raise ValueError("response shape must be [2K+1][I][T_R]")
            descs[k] = wct_plane_desc(pl.n_wires, pl.n_ticks, pl.n_impacts, K, r.shape[2],
                                      r.ctypes.data_as(c_void_p))
        self.device = int(device)
        self.max_events = int(max_events)
        desc = wct_plan_desc(self.dtype, len(planes), descs, self.max_events, self.device)
        h = c_void_p()
        check(wct_plan_create(ctypes.byref(desc), ctypes.byref(h)), "wct_plan_create")
        self.h = h
        self.n_planes = len(planes)
        self.grid_elems = int(wct_grid_elems(h))
        self.wave_elems = int(wct_wave_elems(h))
        self.info = [self.plane_info(k) for k in range(self.n_planes)]
        self._ws = None

    def plane_info(self, plane):
        out = (c_int64 * 10)()
        check(wct_plane_info(self.h, plane, out), "wct_plane_info")
        keys = ["n_wires", "n_ticks", "n_impacts", "half_wires", "resp_ticks", "lw", "lt", "F", "grid_off",
                "wave_off"]
        return dict(zip(keys, [int(v) for v in out]))

    @property
    def torch_dtype(self):
        return _dt(self.dtype)

    def workspace(self, op, n_events, n_rows=0):
        torch = _torch()
        need = int(wct_workspace_bytes(self.h, op, n_events, n_rows))
        if need == 0:
            raise WctError(WCT_E_INVALID, "wct_workspace_bytes")
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws, need

    def _stream(self):
        torch = _torch()
        return c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def new_grid(self, n_events=1):
        torch = _torch()
        return torch.empty(n_events * self.grid_elems, dtype=self.torch_dtype, device=f"cuda:{self.device}")

    def new_wave(self, n_events=1):
        torch = _torch()
        return torch.empty(n_events * self.wave_elems, dtype=self.torch_dtype, device=f"cuda:{self.device}")

    def raster(self, depos: DeviceDepos, o: wct_opts, grid=None):
        grid = self.new_grid(o.n_events) if grid is None else grid
        ws, nb = self.workspace(OP_RASTER, o.n_events, depos.n)
        d = depos.c()
        check(wct_raster(self.h, ctypes.byref(d), ctypes.byref(o), _ptr(grid), _ptr(ws), nb, self._stream()),
              "wct_raster")
        return grid

    def raster_noalloc(self, depos: DeviceDepos, o: wct_opts, grid):
        """wct_raster with the library's static scratch: allocates nothing (grid given)."""
        d = depos.c()
        check(wct_raster_noalloc(self.h, ctypes.byref(d), ctypes.byref(o), _ptr(grid), self._stream()),
              "wct_raster_noalloc")
        return grid

    def convolve(self, grid, n_events=1, wave=None):
        wave = self.new_wave(n_events) if wave is None else wave
        ws, nb = self.workspace(OP_CONVOLVE, n_events, 0)
        check(wct_convolve(self.h, _ptr(grid), n_events, _ptr(wave), _ptr(ws), nb, self._stream()), "wct_convolve")
        return wave

    def simulate(self, depos: DeviceDepos, o: wct_opts, wave=None):
        wave = self.new_wave(o.n_events) if wave is None else wave
        ws, nb = self.workspace(OP_SIMULATE, o.n_events, depos.n)
        d = depos.c()
        check(wct_simulate(self.h, ctypes.byref(d), ctypes.byref(o), _ptr(wave), _ptr(ws), nb, self._stream()),
              "wct_simulate")
        return wave

    def simulate_graph(self, depos: DeviceDepos, o: wct_opts, wave=None):
        """simulate() replayed from the plan's graph for these arguments (captured on first use)."""
        wave = self.new_wave(o.n_events) if wave is None else wave
        ws, nb = self.workspace(OP_SIMULATE, o.n_events, depos.n)
        d = depos.c()
        check(wct_simulate_graph(self.h, ctypes.byref(d), ctypes.byref(o), _ptr(wave), _ptr(ws), nb, self._stream()),
              "wct_simulate_graph")
        return wave

    def simulate_backward(self, depos: DeviceDepos, o: wct_opts, grad_wave):
        torch = _torch()
        outs = [torch.empty(depos.n, dtype=self.torch_dtype, device=f"cuda:{self.device}") for _ in range(5)]
        ws, nb = self.workspace(OP_BACKWARD, o.n_events, depos.n)
        d = depos.c()
        check(wct_simulate_backward(self.h, ctypes.byref(d), ctypes.byref(o), _ptr(grad_wave), *[_ptr(x) for x in outs],
                                    _ptr(ws), nb, self._stream()), "wct_simulate_backward")
        return outs

    def get_fft(self, plane, kind):
        """Transform variant of a plane's tick (kind 0) or wire (kind 1) transforms; -1 = runtime plan."""
        v = c_int32()
        check(wct_plan_get_fft(self.h, plane, kind, ctypes.byref(v)), "wct_plan_get_fft")
        return v.value

    def set_fft(self, plane, kind, variant):
        check(wct_plan_set_fft(self.h, plane, kind, variant), "wct_plan_set_fft")

    def tile_candidates(self):
        """Raster tile variants of this plan's dtype (indices of tile_variants())."""
        dt = "f64" if self.dtype == WCT_F64 else "f32"
        return [v["index"] for v in tile_variants() if v["dtype"] == dt]

    def get_tile(self):
        v = c_int32()
        check(wct_plan_get_tile(self.h, ctypes.byref(v)), "wct_plan_get_tile")
        return v.value

    def set_tile(self, variant):
        check(wct_plan_set_tile(self.h, variant), "wct_plan_set_tile")

    def tune_raster(self, depos: DeviceDepos, o: wct_opts, cache_path=None):
        """Pick the fastest raster tile variant for these rows (optionally via a cache file)."""
        torch = _torch()
        need = int(wct_tune_raster_workspace_bytes(self.h, o.n_events, depos.n))
        if need == 0:
            raise WctError(WCT_E_INVALID, "wct_tune_raster_workspace_bytes")
        ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        d = depos.c()
        path = None if cache_path is None else str(cache_path).encode()
        check(wct_plan_tune_raster(self.h, ctypes.byref(d), ctypes.byref(o), path, _ptr(ws), need, self._stream()),
              "wct_plan_tune_raster")
        return self.get_tile()

    def set_noise(self, plane, amp):
        """Noise amplitude spectrum of a plane (host array of F = L_t/2 + 1 values), or None."""
        if amp is None:
            check(wct_plan_set_noise(self.h, plane, None, 0), "wct_plan_set_noise")
            return
        a = np.ascontiguousarray(amp, dtype=np.float64)
        check(wct_plan_set_noise(self.h, plane, a.ctypes.data_as(POINTER(c_double)), a.size), "wct_plan_set_noise")

    def drift(self, pts: "DevicePoints", prm: "wct_drift_params", out: "DeviceDepos" = None):
        """Rows of the drifted depositions on every plane (wct_drift), plane-major."""
        torch = _torch()
        n = self.n_planes * pts.n
        if pts.x.dtype != self.torch_dtype:
            raise WctError(WCT_E_INVALID, "points must be in the plan dtype")
        if out is None:
            dev = pts.x.device
            f = lambda: torch.empty(n, dtype=self.torch_dtype, device=dev)
            i = lambda: torch.empty(n, dtype=torch.int32, device=dev)
            out = DeviceDepos(f(), f(), f(), f(), f(), i(), i(), i())
        elif out.n != n:
            raise WctError(WCT_E_INVALID, "out must hold n_planes x n rows")
        o = wct_depos_out(_ptr(out.q), _ptr(out.t), _ptr(out.p), _ptr(out.sigma_t), _ptr(out.sigma_p),
                          _ptr(out.plane), _ptr(out.event), _ptr(out.depo_id))
        d = pts.c()
        check(wct_drift(self.h, ctypes.byref(d), ctypes.byref(prm), ctypes.byref(o), self._stream()), "wct_drift")
        return out

    def set_adc(self, plane, gain, baseline, max_code):
        """ADC converter of a plane: code = min(max(floor(M gain + baseline + 1/2), 0), max_code)."""
        check(wct_plan_set_adc(self.h, plane, float(gain), float(baseline), int(max_code)), "wct_plan_set_adc")

    def digitize(self, wave, n_events=1, adc=None):
        """ADC codes of n_events events of `wave` (uint16 values, held in an int16 tensor of
        the waveform's element count; view them as uint16 on the host)."""
        torch = _torch()
        n = n_events * self.wave_elems
        if wave.numel() < n:
            raise WctError(WCT_E_INVALID, "wave holds fewer than n_events events")
        if adc is None:
            adc = torch.empty(n, dtype=torch.int16, device=f"cuda:{self.device}")
        elif adc.numel() < n or adc.element_size() != 2:
            raise WctError(WCT_E_INVALID, "adc must hold n_events events of 16-bit codes")
        check(wct_digitize(self.h, _ptr(wave), n_events, _ptr(adc), self._stream()), "wct_digitize")
        return adc

    def tune(self, n_events=1, cache_path=None):
        """Pick the fastest transform variant per plane and kind (optionally via a cache file)."""
        torch = _torch()
        need = int(wct_tune_workspace_bytes(self.h, n_events))
        if need == 0:
            raise WctError(WCT_E_INVALID, "wct_tune_workspace_bytes")
        ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        path = None if cache_path is None else str(cache_path).encode()
        check(wct_plan_tune(self.h, n_events, path, _ptr(ws), need, self._stream()), "wct_plan_tune")
        return {(p, k): self.get_fft(p, k) for p in range(self.n_planes) for k in (0, 1)}

    def fft_candidates(self, plane, kind):
        """Variants applicable to a plane's transform of this kind, runtime plan (-1) last."""
        info = self.plane_info(plane)
        n = info["lt"] // 2 if kind == 0 else info["lw"]
        kinds = (0,) if kind == 0 else (1, 2)  # wire transforms: whole or half chunks per block
        comp = [v["index"] for v in fft_variants()
                if v["kind"] in kinds and v["dtype"] == ("f64" if self.dtype == WCT_F64 else "f32")
                and v["n"] == n]
        # wires: the direct sum over the response's 21 wires when the response has them
        direct = [WCT_WIRE_DIRECT] if kind == 1 and info["half_wires"] == 10 else []
        return comp + direct + [-1]

    def profile(self, enable=True):
        check(wct_profile_enable(self.h, int(bool(enable))), "wct_profile_enable")

    def profile_reset(self):
        check(wct_profile_reset(self.h), "wct_profile_reset")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last reset (synchronises)."""
        n = wct_profile_count(self.h)
        if n < 0:
            check(n, "wct_profile_count")
        out = {}
        buf = ctypes.create_string_buffer(128)
        for k in range(n):
            ms = c_double()
            cnt = c_int64()
            check(wct_profile_get(self.h, k, buf, 128, ctypes.byref(ms), ctypes.byref(cnt)), "wct_profile_get")
            out[buf.value.decode()] = (ms.value, cnt.value)
        return out

    def grid_view(self, grid, event=0):
        """Per-plane [N_b][N_t] views of one event of a packed grid."""
        out = []
        base = event * self.grid_elems
        for inf in self.info:
            n = inf["n_impacts"] * inf["n_wires"] * inf["n_ticks"]
            out.append(grid[base + inf["grid_off"]: base + inf["grid_off"] + n].view(
                inf["n_impacts"] * inf["n_wires"], inf["n_ticks"]))
        return out

    def wave_view(self, wave, event=0):
        out = []
        base = event * self.wave_elems
        for inf in self.info:
            n = inf["n_wires"] * inf["n_ticks"]
            out.append(wave[base + inf["wave_off"]: base + inf["wave_off"] + n].view(inf["n_wires"], inf["n_ticks"]))
        return out

    def close(self):
        if getattr(self, "h", None):
            wct_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
