"""The C ABI library: loads, exports every declared symbol, rejects bad arguments (no GPU needed)."""
import ctypes
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wct.h")


def declared_functions():
    import glob
    src = "".join(open(h).read() for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wct_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = declared_functions()
    for n in ("wct_raster", "wct_convolve", "wct_simulate", "wct_simulate_graph", "wct_simulate_backward",
              "wct_plan_create",
              "wct_plan_destroy", "wct_workspace_bytes", "wct_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(wct):
    for n in declared_functions():
        assert hasattr(wct.lib, n), f"{n} declared in wct.h but not exported"


def test_versions(wct):
    assert wct.wct_abi_version() == 8
    assert wct.wct_fluct_spec_version() == 2


def test_null_and_invalid_arguments(wct):
    from ctypes import byref, c_int64, c_void_p
    assert wct.wct_raster(None, None, None, None, None, 0, None) == wct.WCT_E_INVALID
    assert "plan is NULL" in wct.last_error()
    assert wct.wct_convolve(None, None, 1, None, None, 0, None) == wct.WCT_E_INVALID
    assert wct.wct_simulate(None, None, None, None, None, 0, None) == wct.WCT_E_INVALID
    assert wct.wct_simulate_backward(None, None, None, None, None, None, None, None, None, None, 0,
                                     None) == wct.WCT_E_INVALID
    assert wct.wct_workspace_bytes(None, 0, 1, 10) == 0
    assert wct.wct_grid_elems(None) == -1 and wct.wct_wave_elems(None) == -1
    out = (c_int64 * 10)()
    assert wct.wct_plane_info(None, 0, out) == wct.WCT_E_INVALID
    assert wct.wct_profile_enable(None, 1) == wct.WCT_E_INVALID
    wct.wct_plan_destroy(None)
    h = c_void_p()
    assert wct.wct_plan_create(None, byref(h)) == wct.WCT_E_INVALID
    # bad descriptors are rejected before any device call
    desc = wct.wct_plan_desc(7, 1, None, 1, 0)
    assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_INVALID and not h.value
    desc = wct.wct_plan_desc(wct.WCT_F32, 0, None, 1, 0)
    assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_INVALID
    assert "n_planes" in wct.last_error()
    desc = wct.wct_plan_desc(wct.WCT_F32, 1, None, 1, 0)
    assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_INVALID
    planes = (wct.wct_plane_desc * 1)()
    desc = wct.wct_plan_desc(wct.WCT_F32, 1, planes, 0, 0)
    assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_INVALID
    assert "max_events" in wct.last_error()


def test_plan_limits_answer_before_any_device_call(wct, monkeypatch):
    """Buffers of max_events events past 2^60 bytes, and a WCT_PLAN_MEM_CAP that is not a
    byte count, are refused from the description alone (no GPU needed)."""
    import numpy as np
    from ctypes import byref, c_void_p
    resp = np.zeros((21, 10, 200), np.float32)
    planes = (wct.wct_plane_desc * 1)()
    planes[0] = wct.wct_plane_desc(2400, 9600, 10, 10, 200, resp.ctypes.data_as(c_void_p))
    h = c_void_p()
    desc = wct.wct_plan_desc(wct.WCT_F32, 1, planes, 2 ** 31 - 1, 0)
    assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_UNSUPPORTED and not h.value
    assert "2^60" in wct.last_error()
    desc = wct.wct_plan_desc(wct.WCT_F32, 1, planes, 1, 0)
    for bad in ("12kB", "-5", ""):
        monkeypatch.setenv("WCT_PLAN_MEM_CAP", bad)
        assert wct.wct_plan_create(byref(desc), byref(h)) == wct.WCT_E_INVALID and not h.value
        assert "WCT_PLAN_MEM_CAP" in wct.last_error()


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The product path has no fallback: importing the binding without libwct.so raises."""
    pkg = tmp_path / "paper_2104_08265_amd"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    shutil.copy(os.path.join(ROOT, "paper_2104_08265_amd", "wct.py"), pkg / "wct.py")
    r = subprocess.run([sys.executable, "-c", "import paper_2104_08265_amd.wct"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0 and "is not built" in r.stderr


def test_build_flags_keep_packed_fp32_out_and_contraction_off_for_fluctuation():
    from paper_2104_08265_amd import build as B
    assert "-packed-fp32-ops" in B.COMMON
    for src in ("raster.hip", "drift.hip", "adc.hip"):
        assert "-ffp-contract=off" in B.SOURCES[src], src
