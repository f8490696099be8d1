"""The C-ABI library loads without a GPU, exports every entry point that
include/mcrt.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

from paper_1512_02110_amd import mcrt, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mc_\w+)\s*\(", text, flags=re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mcrt.LIB_PATH):
        pytest.skip("libmcrt.so not built")
    return mcrt.load_library()


def test_header_declares_the_entry_points():
    assert {"mc_render", "mc_grad_beta", "mc_trace_paths", "mc_error_string",
            "mc_device_count"} <= declared_functions()


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", mcrt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared_functions() - exported
    assert not missing, missing
    for name in declared_functions():
        assert hasattr(lib, name)


def test_struct_layouts_match_header():
    # sizes fixed by the header: grid 40, camera 176, params 88, stats 96,
    # event 40, path 64 bytes
    assert C.sizeof(mcrt.McGrid) == 40
    assert C.sizeof(mcrt.McCamera) == 3 * 8 + 9 * 8 + 4 * 8 + 8
    assert C.sizeof(mcrt.McParams) == 5 * 8 + 4 * 8 + 4 * 4
    assert C.sizeof(mcrt.McStats) == 10 * 8 + 2 * 8
    assert mcrt.EVENT_DTYPE.itemsize == 40 and mcrt.PATH_DTYPE.itemsize == 64


def test_error_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert mcrt.error_string(code)
    assert mcrt.error_string(-99) == "unknown status code"


def _call_render(lib, s, **kw):
    params = mcrt.make_params(s, **kw)
    return lib.mc_render(C.byref(mcrt.make_grid(s)), C.c_void_p(16), len(s.cameras),
                         mcrt.make_cameras(s.cameras), C.byref(params), C.c_void_p(16), None, None)


def test_invalid_arguments_rejected_before_device(lib):
    s = scenes.config1(n_photons=10)
    bad = [dict(g=1.0), dict(albedo=2.0), dict(sun_zenith=math.pi / 2), dict(rr_weight=0.0),
           dict(max_events=0)]
    for b in bad:
        t = s.replace(**{k: v for k, v in b.items() if k in ("g", "albedo", "sun_zenith")})
        kw = {k: v for k, v in b.items() if k in ("rr_weight", "max_events")}
        assert _call_render(lib, t, **kw) == mcrt.MC_ERR_INVALID_ARG
    p = mcrt.make_params(s)
    p.transport = 7
    assert lib.mc_render(C.byref(mcrt.make_grid(s)), C.c_void_p(16), 4, mcrt.make_cameras(s.cameras),
                         C.byref(p), C.c_void_p(16), None, None) == mcrt.MC_ERR_INVALID_ARG
    g = mcrt.make_grid(s)
    g.nx = 0
    assert lib.mc_render(C.byref(g), C.c_void_p(16), 4, mcrt.make_cameras(s.cameras),
                         C.byref(mcrt.make_params(s)), C.c_void_p(16), None, None) == mcrt.MC_ERR_INVALID_ARG
    assert lib.mc_render(C.byref(mcrt.make_grid(s)), C.c_void_p(16), 0, mcrt.make_cameras(s.cameras),
                         C.byref(mcrt.make_params(s)), C.c_void_p(16), None, None) == mcrt.MC_ERR_INVALID_ARG
    assert lib.mc_render(C.byref(mcrt.make_grid(s)), None, 4, mcrt.make_cameras(s.cameras),
                         C.byref(mcrt.make_params(s)), C.c_void_p(16), None, None) == mcrt.MC_ERR_INVALID_ARG
    cams = mcrt.make_cameras(s.cameras)
    cams[1].fx = -1.0
    assert lib.mc_render(C.byref(mcrt.make_grid(s)), C.c_void_p(16), 4, cams,
                         C.byref(mcrt.make_params(s)), C.c_void_p(16), None, None) == mcrt.MC_ERR_INVALID_ARG


def test_no_device_reported_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    s = scenes.config1(n_photons=10)
    assert lib.mc_device_count() == 0
    assert _call_render(lib, s) == mcrt.MC_ERR_NO_DEVICE
    with pytest.raises(RuntimeError):
        mcrt.mc_render(s, None)
