"""Python binding of libmcrt.so (the gfx950 HIP renderer).

Argument marshalling only: every step of the renderer runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the library
is missing or no GPU is visible the calls raise; there is no CPU fallback.

Entry points (same names as the C ABI in include/mcrt.h):
    mc_render(scene, beta, ...)      -> images (float64 tensor on the GPU), stats
    mc_grad_beta(scene, beta, dl, ...) -> dL/dbeta (float64 tensor), stats
    mc_render_tape(scene, beta, ...) -> images, stats, Tape (or None): a render that keeps its rays
    mc_grad_beta(..., tape=t)        -> the gradient of that render from its rays (no replay)
    mc_trace_paths(scene, beta, first_pid, count, max_rec, ...)
    MCRender: torch.autograd.Function (forward = render, backward = surrogate gradient)
    MCRenderMixture: the same for one channel of an air + aerosol mixture (backward =
        dL/d beta_aer, full or surrogate)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmcrt.so")

MC_OK, MC_ERR_INVALID_ARG, MC_ERR_NO_DEVICE, MC_ERR_HIP, MC_ERR_OUT_OF_MEMORY = 0, -1, -2, -3, -4
MC_ERR_SCRATCH_LIMIT = -5
MC_FP32, MC_FP64, MC_MIXED = 0, 1, 2
MC_TALLY_F64, MC_TALLY_KAHAN32 = 0, 1
# "mixed": photons in FP64, connection rays walked in FP32 (beta given in FP64)
TRANSPORTS = {"fp32": MC_FP32, "fp64": MC_FP64, "mixed": MC_MIXED}
TALLIES = {"f64": MC_TALLY_F64, "kahan32": MC_TALLY_KAHAN32}


class McGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class McCamera(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("R", C.c_double * 9), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class McParams(C.Structure):
    _fields_ = [("albedo", C.c_double), ("g", C.c_double), ("sun_zenith", C.c_double),
                ("sun_azimuth", C.c_double), ("rr_weight", C.c_double),
                ("n_photons", C.c_uint64), ("seed", C.c_uint64), ("photon_offset", C.c_uint64),
                ("n_photons_norm", C.c_uint64), ("max_events", C.c_uint32),
                ("transport", C.c_int32), ("tally", C.c_int32), ("tape_limit", C.c_int32)]


STAT_FIELDS = ["photons", "events", "le_jobs", "vox_free", "vox_conn", "esc_top", "esc_bottom",
               "esc_side", "rr_killed", "capped"]


TIMING_FIELDS = ["transport_ms", "tape_ms"]


class Stats(dict):
    """The counters of a call (a dict, compared as one); `.timing` holds the
    device times the library measured with HIP events."""
    timing: dict = {}


def _stats(st) -> "Stats":
    out = Stats(st.as_dict())
    out.timing = st.timing()
    return out


class McStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_FIELDS] + [(n, C.c_double) for n in TIMING_FIELDS]

    def as_dict(self):
        """The counters (deterministic for a given photon range)."""
        return {n: int(getattr(self, n)) for n in STAT_FIELDS}

    def timing(self):
        """Device times (ms) the library measured with HIP events."""
        return {n: float(getattr(self, n)) for n in TIMING_FIELDS}


EVENT_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("z", "<f8"), ("w", "<f8"),
                        ("voxel", "<i4"), ("pad_", "<i4")])
PATH_DTYPE = np.dtype([("n_events", "<i4"), ("fate", "<i4"), ("exit_pos", "<f8", (3,)),
                       ("exit_dir", "<f8", (3,)), ("exit_w", "<f8")])

EXPORTS = ["mc_render", "mc_render_moments", "mc_grad_beta", "mc_trace_paths", "mc_error_string",
           "mc_device_count", "mc_render_tape", "mc_grad_beta_tape", "mc_tape_free", "mc_release_memory",
           "mc_voxel_scatter", "mc_voxel_render", "mc_voxel_grad", "mc_voxel_conditioning", "mc_regularizer",
           "mc_image_residual", "mc_gd_step", "mc_camera_noise", "mc_recovery_error", "mc_recover",
           "mc_bmc_render", "mc_render_mixture", "mc_grad_mixture", "mc_render_frozen", "mc_render_noalloc",
           "mc_capture_gathers"]


class McError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({error_string(code)})")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmcrt.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError(f"{path} is missing: build it with `python -m paper_1512_02110_amd.build`")
        # torch first: its HIP runtime is then the one the library binds to
        # (a second copy loaded ahead of torch's is not safe in one process)
        import torch  # noqa: F401
        L = C.CDLL(path)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.mc_render.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                C.POINTER(McParams), vp, C.POINTER(McStats), vp]
        L.mc_capture_gathers.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera), C.POINTER(McParams),
                                         vp, C.c_uint32, C.c_uint32, C.c_uint32, vp, vp, C.POINTER(C.c_uint32),
                                         C.POINTER(McStats), vp]
        L.mc_render_noalloc.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                        C.POINTER(McParams), vp, C.POINTER(McStats), vp]
        L.mc_render_moments.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                        C.POINTER(McParams), vp, vp, C.POINTER(McStats), vp]
        L.mc_grad_beta.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                   C.POINTER(McParams), vp, vp, C.POINTER(McStats), vp]
        L.mc_trace_paths.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                     C.POINTER(McParams), C.c_uint64, C.c_uint32, C.c_uint32,
                                     vp, vp, vp, vp]
        L.mc_render_tape.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                     C.POINTER(McParams), vp, C.POINTER(McStats), vp, C.POINTER(vp)]
        L.mc_grad_beta_tape.argtypes = [vp, C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                        C.POINTER(McParams), vp, vp, C.POINTER(McStats), vp]
        L.mc_tape_free.argtypes = [vp, vp]
        L.mc_release_memory.argtypes = []
        L.mc_voxel_scatter.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera),
                                       C.POINTER(McParams), vp, C.POINTER(McStats), vp]
        L.mc_voxel_render.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera), C.c_int, vp, vp, vp]
        L.mc_voxel_grad.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera), C.c_int, vp, vp, vp,
                                    vp, vp]
        L.mc_bmc_render.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera), C.POINTER(McParams),
                                    C.c_uint32, vp, vp, C.POINTER(McStats), vp]
        L.mc_render_frozen.argtypes = [C.POINTER(McGrid), vp, vp, C.c_int, C.POINTER(McCamera),
                                       C.POINTER(McParams), vp, C.POINTER(McStats), vp]
        L.mc_render_mixture.argtypes = [C.POINTER(McGrid), vp, vp, C.c_double, C.c_int, C.POINTER(McCamera),
                                        C.POINTER(McParams), vp, vp, C.POINTER(McStats), vp]
        L.mc_grad_mixture.argtypes = [C.POINTER(McGrid), vp, vp, C.c_double, C.c_int, C.POINTER(McCamera),
                                      C.POINTER(McParams), vp, C.c_int, vp, C.POINTER(McStats), vp]
        L.mc_voxel_conditioning.argtypes = [C.POINTER(McGrid), C.c_int, C.POINTER(McCamera), C.c_int, vp, vp, vp]
        L.mc_regularizer.argtypes = [C.POINTER(McGrid), vp, vp, C.c_double, vp, vp, vp]
        L.mc_image_residual.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp]
        L.mc_gd_step.argtypes = [C.c_int64, vp, vp, C.c_double, vp]
        L.mc_camera_noise.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp]
        L.mc_recovery_error.argtypes = [C.c_int64, vp, vp, dp, vp]
        L.mc_recover.argtypes = [C.POINTER(McGrid), vp, C.c_int, C.POINTER(McCamera), C.POINTER(McParams), C.c_int,
                                 vp, vp, vp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, dp, vp]
        for f in ("mc_render", "mc_render_moments", "mc_grad_beta", "mc_trace_paths", "mc_device_count",
                  "mc_render_tape", "mc_grad_beta_tape", "mc_tape_free", "mc_release_memory",
                  "mc_voxel_scatter", "mc_voxel_render", "mc_voxel_grad", "mc_voxel_conditioning",
                  "mc_regularizer", "mc_image_residual", "mc_gd_step", "mc_camera_noise", "mc_recovery_error",
                  "mc_recover", "mc_bmc_render", "mc_render_mixture", "mc_grad_mixture", "mc_render_frozen"):
            getattr(L, f).restype = C.c_int
        L.mc_device_count.argtypes = []
        L.mc_error_string.argtypes = [C.c_int]
        L.mc_error_string.restype = C.c_char_p
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return load_library().mc_error_string(int(code)).decode()


def _check(fn, rc):
    if rc != MC_OK:
        raise McError(fn, rc)


def make_grid(s) -> McGrid:
    return McGrid(int(s.nx), int(s.ny), int(s.nz), 0, float(s.dx), float(s.dy), float(s.dz))


def make_cameras(cameras):
    arr = (McCamera * max(1, len(cameras)))()
    for i, c in enumerate(cameras):
        arr[i].pos[:] = [float(v) for v in c.pos]
        arr[i].R[:] = [float(v) for v in c.R]
        arr[i].fx, arr[i].fy = float(c.fx), float(c.fy)
        arr[i].cx, arr[i].cy = float(c.cx), float(c.cy)
        arr[i].width, arr[i].height = int(c.width), int(c.height)
    return arr


def make_params(s, n_photons=None, seed=None, photon_offset=0, n_photons_norm=0,
                max_events=100000, rr_weight=0.1, transport="fp32", tally="f64", tape_limit=0) -> McParams:
    return McParams(float(s.albedo), float(s.g), float(s.sun_zenith), float(s.sun_azimuth),
                    float(rr_weight), int(s.n_photons if n_photons is None else n_photons),
                    int(s.seed if seed is None else seed), int(photon_offset), int(n_photons_norm),
                    int(max_events), TRANSPORTS[transport], TALLIES[tally], int(tape_limit))


def n_pixels(s) -> int:
    return sum(int(c.width) * int(c.height) for c in s.cameras)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the renderer runs only on the HIP device")
    return torch


def _stream(torch, stream):
    return (stream if stream is not None else torch.cuda.current_stream()).cuda_stream


def beta_tensor(s, transport="fp32", beta=None, device="cuda"):
    """Device copy of the scene's extinction in the dtype the transport reads."""
    torch = _torch()
    b = s.beta if beta is None else beta
    dt = torch.float32 if transport == "fp32" else torch.float64  # (mixed: FP64 beta)
    if isinstance(b, torch.Tensor):
        return b.detach().to(device=device, dtype=dt).contiguous().reshape(-1)
    return torch.as_tensor(np.ascontiguousarray(b).reshape(-1), dtype=dt, device=device)


def _check_beta(torch, s, beta, transport):
    want = torch.float32 if transport == "fp32" else torch.float64
    if not (beta.is_cuda and beta.dtype == want and beta.is_contiguous() and beta.numel() == s.n_vox):
        raise ValueError(f"beta must be a contiguous {want} CUDA tensor of {s.n_vox} voxels")


def mc_render(s, beta, transport="fp32", tally="f64", stats=True, out=None, stream=None, **kw):
    """Forward render.  Returns (images [n_pix] float64 on the GPU, stats dict or None)."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    n = n_pixels(s)
    img = out if out is not None else torch.empty(n, dtype=torch.float64, device=beta.device)
    st = McStats() if stats else None
    rc = load_library().mc_render(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                  make_cameras(s.cameras),
                                  C.byref(make_params(s, transport=transport, tally=tally, **kw)),
                                  C.c_void_p(img.data_ptr()), C.byref(st) if stats else None,
                                  C.c_void_p(_stream(torch, stream)))
    _check("mc_render", rc)
    return img, (_stats(st) if stats else None)


def mc_render_noalloc(s, beta, transport="fp32", tally="f64", stats=True, out=None, stream=None, **kw):
    """mc_render through the entry point that allocates nothing in the library (its
    scratch is a fixed 64 MiB device array).  Returns (images, stats or None); `out`
    (a float64 CUDA tensor of the pixel count) avoids the allocation of the images."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    n = n_pixels(s)
    img = out if out is not None else torch.empty(n, dtype=torch.float64, device=beta.device)
    st = McStats() if stats else None
    rc = load_library().mc_render_noalloc(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                          make_cameras(s.cameras),
                                          C.byref(make_params(s, transport=transport, tally=tally, **kw)),
                                          C.c_void_p(img.data_ptr()), C.byref(st) if stats else None,
                                          C.c_void_p(_stream(torch, stream)))
    _check("mc_render_noalloc", rc)
    return img, (_stats(st) if stats else None)


def mc_capture_gathers(s, beta, first_step, n_steps, max_waves, stream=None, **kw):
    """The gather capture (a diagnostic of the FP32 render): returns (indices
    [max_waves, n_steps, 64] int32 tensor, steps per wavefront [max_waves], the
    launch's wavefronts, stats); see include/mcrt.h."""
    torch = _torch()
    _check_beta(torch, s, beta, "fp32")
    img = torch.empty(n_pixels(s), dtype=torch.float64, device=beta.device)
    idx = torch.full((max_waves, n_steps, 64), -1, dtype=torch.int32, device=beta.device)
    steps = torch.zeros(max_waves, dtype=torch.int32, device=beta.device)
    nw = C.c_uint32(0)
    st = McStats()
    rc = load_library().mc_capture_gathers(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                           make_cameras(s.cameras), C.byref(make_params(s, **kw)),
                                           C.c_void_p(img.data_ptr()), int(first_step), int(n_steps), int(max_waves),
                                           C.c_void_p(idx.data_ptr()), C.c_void_p(steps.data_ptr()), C.byref(nw),
                                           C.byref(st), C.c_void_p(_stream(torch, stream)))
    _check("mc_capture_gathers", rc)
    return idx, steps, int(nw.value), _stats(st)


def mc_render_moments(s, beta, transport="fp32", tally="f64", stats=True, stream=None, **kw):
    """Forward render with per-pixel second moments.  Returns (images, images_m2, stats);
    the Monte Carlo variance of a pixel is about images_m2 - images**2 / N."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    n = n_pixels(s)
    img = torch.empty(n, dtype=torch.float64, device=beta.device)
    m2 = torch.empty(n, dtype=torch.float64, device=beta.device)
    st = McStats() if stats else None
    rc = load_library().mc_render_moments(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()),
                                          len(s.cameras), make_cameras(s.cameras),
                                          C.byref(make_params(s, transport=transport, tally=tally, **kw)),
                                          C.c_void_p(img.data_ptr()), C.c_void_p(m2.data_ptr()),
                                          C.byref(st) if stats else None, C.c_void_p(_stream(torch, stream)))
    _check("mc_render_moments", rc)
    return img, m2, (_stats(st) if stats else None)


class Tape:
    """The rays a render kept (mc_render_tape) for mc_grad_beta(..., tape=...).
    Holds device memory of the library until free() (or garbage collection)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise ValueError("the tape has been freed")
        return self._h

    def free(self, stream=None):
        if self._h:
            torch = _torch()
            h, self._h = self._h, None
            _check("mc_tape_free", load_library().mc_tape_free(C.c_void_p(h), C.c_void_p(_stream(torch, stream))))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mc_release_memory():
    """Return the device memory the library keeps pooled for reuse (call when idle)."""
    _torch().cuda.synchronize()
    _check("mc_release_memory", load_library().mc_release_memory())


def mc_render_tape(s, beta, transport="fp32", tally="f64", stats=True, out=None, stream=None, **kw):
    """Forward render that keeps its connection rays for the gradient.  Returns (images,
    stats or None, Tape or None); None when the grid does not need a tape or the rays do
    not fit (the images are rendered either way).  Waits for the stream."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    n = n_pixels(s)
    img = out if out is not None else torch.empty(n, dtype=torch.float64, device=beta.device)
    st = McStats() if stats else None
    h = C.c_void_p()
    rc = load_library().mc_render_tape(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                       make_cameras(s.cameras),
                                       C.byref(make_params(s, transport=transport, tally=tally, **kw)),
                                       C.c_void_p(img.data_ptr()), C.byref(st) if stats else None,
                                       C.c_void_p(_stream(torch, stream)), C.byref(h))
    _check("mc_render_tape", rc)
    return img, (_stats(st) if stats else None), (Tape(h.value) if h.value else None)


def mc_grad_beta(s, beta, dl_dimages, transport="fp32", tally="f64", stats=True, out=None,
                 stream=None, tape=None, **kw):
    """Surrogate gradient dL/dbeta for image gradient dl_dimages (float64 [n_pix]); with
    `tape` (from mc_render_tape with the same scene, beta and parameters), from the
    render's rays instead of a replay of the photons."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    dl = dl_dimages.detach().to(device=beta.device, dtype=torch.float64).contiguous().reshape(-1)
    if dl.numel() != n_pixels(s):
        raise ValueError("dl_dimages has the wrong number of pixels")
    g = out if out is not None else torch.empty(s.n_vox, dtype=torch.float64, device=beta.device)
    st = McStats() if stats else None
    args = (C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras), make_cameras(s.cameras),
            C.byref(make_params(s, transport=transport, tally=tally, **kw)), C.c_void_p(dl.data_ptr()),
            C.c_void_p(g.data_ptr()), C.byref(st) if stats else None, C.c_void_p(_stream(torch, stream)))
    if tape is not None:
        rc = load_library().mc_grad_beta_tape(C.c_void_p(tape.handle), *args)
        _check("mc_grad_beta_tape", rc)
    else:
        rc = load_library().mc_grad_beta(*args)
        _check("mc_grad_beta", rc)
    return g, (_stats(st) if stats else None)


def mc_bmc_render(s, beta, n_per_pixel, transport="fp32", with_m2=False, stats=True, stream=None, **kw):
    """Backward Monte Carlo images (Sec. 2.1.4, Eq. ble).  Returns (images, stats[, m2])."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    n = n_pixels(s)
    img = torch.empty(n, dtype=torch.float64, device=beta.device)
    m2 = torch.empty(n, dtype=torch.float64, device=beta.device) if with_m2 else None
    st = McStats() if stats else None
    rc = load_library().mc_bmc_render(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                      make_cameras(s.cameras), C.byref(make_params(s, transport=transport, **kw)),
                                      int(n_per_pixel), C.c_void_p(img.data_ptr()), _ptr(m2),
                                      C.byref(st) if stats else None, C.c_void_p(_stream(torch, stream)))
    _check("mc_bmc_render", rc)
    out = (img, _stats(st) if stats else None)
    return out + (m2,) if with_m2 else out


def mc_render_frozen(s, beta_sample, beta_eval, transport="fp32", stats=True, stream=None, **kw):
    """Frozen-event images: photons through beta_sample, local estimates through
    beta_eval scaled by beta_eval / beta_sample at the collision (both GPU tensors in
    the transport's dtype).  Returns (images, stats)."""
    torch = _torch()
    _check_beta(torch, s, beta_sample, transport)
    _check_beta(torch, s, beta_eval, transport)
    img = torch.empty(n_pixels(s), dtype=torch.float64, device=beta_sample.device)
    st = McStats() if stats else None
    rc = load_library().mc_render_frozen(C.byref(make_grid(s)), C.c_void_p(beta_sample.data_ptr()),
                                         C.c_void_p(beta_eval.data_ptr()), len(s.cameras), make_cameras(s.cameras),
                                         C.byref(make_params(s, transport=transport, **kw)),
                                         C.c_void_p(img.data_ptr()), C.byref(st) if stats else None,
                                         C.c_void_p(_stream(torch, stream)))
    _check("mc_render_frozen", rc)
    return img, (_stats(st) if stats else None)


def _mix_fields(torch, s, beta_air, beta_aer):
    for name, t in (("beta_air", beta_air), ("beta_aer", beta_aer)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == s.n_vox):
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor of {s.n_vox} values")


def mc_render_mixture(s, beta_air, beta_aer, sigma=1.0, transport="fp32", with_m2=False, stats=True, stream=None,
                      **kw):
    """One channel of the air + aerosol mixture: extinction beta_air + sigma * beta_aer
    (float64 GPU tensors), the scene's albedo and g for the aerosol, Rayleigh air.
    Returns (images, stats[, m2])."""
    torch = _torch()
    _mix_fields(torch, s, beta_air, beta_aer)
    n = n_pixels(s)
    img = torch.empty(n, dtype=torch.float64, device=beta_air.device)
    m2 = torch.empty(n, dtype=torch.float64, device=beta_air.device) if with_m2 else None
    st = McStats() if stats else None
    rc = load_library().mc_render_mixture(C.byref(make_grid(s)), _ptr(beta_air), _ptr(beta_aer), float(sigma),
                                          len(s.cameras), make_cameras(s.cameras),
                                          C.byref(make_params(s, transport=transport, **kw)), _ptr(img), _ptr(m2),
                                          C.byref(st) if stats else None, C.c_void_p(_stream(torch, stream)))
    _check("mc_render_mixture", rc)
    out = (img, _stats(st) if stats else None)
    return out + (m2,) if with_m2 else out


def mc_grad_mixture(s, beta_air, beta_aer, dl_dimages, sigma=1.0, full=True, grad=None, transport="fp32",
                    stats=True, stream=None, **kw):
    """dL/d beta_aer (reference aerosol field) of the mixture render with the same
    arguments, ADDED to grad (a new zero tensor when None): the surrogate with the
    in-scatter field frozen (full=False) or the full derivative with the photon
    paths' scores (full=True).  Returns (grad, stats)."""
    torch = _torch()
    _mix_fields(torch, s, beta_air, beta_aer)
    n = n_pixels(s)
    if not (isinstance(dl_dimages, torch.Tensor) and dl_dimages.is_cuda and dl_dimages.dtype == torch.float64
            and dl_dimages.is_contiguous() and dl_dimages.numel() == n):
        raise ValueError(f"dl_dimages must be a contiguous float64 GPU tensor of {n} values")
    g = grad if grad is not None else torch.zeros(s.n_vox, dtype=torch.float64, device=beta_air.device)
    _mix_fields(torch, s, beta_air, g)
    st = McStats() if stats else None
    rc = load_library().mc_grad_mixture(C.byref(make_grid(s)), _ptr(beta_air), _ptr(beta_aer), float(sigma),
                                        len(s.cameras), make_cameras(s.cameras),
                                        C.byref(make_params(s, transport=transport, **kw)), _ptr(dl_dimages),
                                        int(bool(full)), _ptr(g), C.byref(st) if stats else None,
                                        C.c_void_p(_stream(torch, stream)))
    _check("mc_grad_mixture", rc)
    return g, (_stats(st) if stats else None)


def mc_render_rgb(s, beta_air_rgb, beta_aer, sigma_rgb, transport="fp32", stream=None, **kw):
    """RGB images of the mixture (Eq. channelBeta): one mc_render_mixture call per
    channel with that channel's air field and aerosol cross-section ratio.
    Returns a list of three (images, stats)."""
    return [mc_render_mixture(s, beta_air_rgb[c], beta_aer, sigma_rgb[c], transport=transport, stream=stream, **kw)
            for c in range(3)]


def mc_grad_rgb(s, beta_air_rgb, beta_aer, dl_rgb, sigma_rgb, full=True, grad=None, transport="fp32", stream=None,
                **kw):
    """Gradient of an RGB image loss with respect to the reference aerosol field
    (the image term of Eq. divCost1): the three channels' mc_grad_mixture calls
    added into one tensor.  Returns grad."""
    torch = _torch()
    g = grad if grad is not None else torch.zeros(s.n_vox, dtype=torch.float64, device=beta_aer.device)
    for c in range(3):
        mc_grad_mixture(s, beta_air_rgb[c], beta_aer, dl_rgb[c], sigma_rgb[c], full=full, grad=g,
                        transport=transport, stats=False, stream=stream, **kw)
    return g


def mc_voxel_scatter(s, beta, transport="fp32", stats=True, out=None, stream=None, **kw):
    """Voxelised model (Sec. 3): j_c(k) of Eq. (Jc) from photons without local
    estimation.  Returns (j: float64 [n_cams * n_vox] on the GPU, camera-major; stats)."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    j = out if out is not None else torch.empty(len(s.cameras) * s.n_vox, dtype=torch.float64,
                                                 device=beta.device)
    st = McStats() if stats else None
    rc = load_library().mc_voxel_scatter(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                         make_cameras(s.cameras),
                                         C.byref(make_params(s, transport=transport, **kw)),
                                         C.c_void_p(j.data_ptr()), C.byref(st) if stats else None,
                                         C.c_void_p(_stream(torch, stream)))
    _check("mc_voxel_scatter", rc)
    return j, (_stats(st) if stats else None)


def _voxel_inputs(torch, s, beta, j):
    if not (beta.is_cuda and beta.dtype == torch.float64 and beta.is_contiguous() and beta.numel() == s.n_vox):
        raise ValueError(f"beta must be a contiguous float64 CUDA tensor of {s.n_vox} voxels")
    j = j.detach().to(device=beta.device, dtype=torch.float64).contiguous().reshape(-1)
    if j.numel() != len(s.cameras) * s.n_vox:
        raise ValueError("j must hold one value per camera and voxel")
    return j


def mc_voxel_render(s, beta, j, rays_per_side=2, out=None, stream=None):
    """Images of the voxelised model, Eq. (Icpixel), for float64 beta and j."""
    torch = _torch()
    j = _voxel_inputs(torch, s, beta, j)
    img = out if out is not None else torch.empty(n_pixels(s), dtype=torch.float64, device=beta.device)
    rc = load_library().mc_voxel_render(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                        make_cameras(s.cameras), int(rays_per_side), C.c_void_p(j.data_ptr()),
                                        C.c_void_p(img.data_ptr()), C.c_void_p(_stream(torch, stream)))
    _check("mc_voxel_render", rc)
    return img


def _dev64(torch, x, device, n=None, name="array"):
    t = x.detach().to(device=device, dtype=torch.float64).contiguous().reshape(-1)
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must hold {n} values")
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t is not None else 0)


def mc_voxel_grad(s, beta, j, dl_dimages, rays_per_side=2, cam_weights=None, out=None, stream=None):
    """dL/dbeta of the voxelised images with j frozen (Eqs. Jaco1, TcofJaco1, DivTc); with
    cam_weights ([camera][voxel], e.g. mc_voxel_conditioning's q) every camera's term is weighted."""
    torch = _torch()
    j = _voxel_inputs(torch, s, beta, j)
    dl = _dev64(torch, dl_dimages, beta.device, n_pixels(s), "dl_dimages")
    q = None if cam_weights is None else _dev64(torch, cam_weights, beta.device, j.numel(), "cam_weights")
    g = out if out is not None else torch.empty(s.n_vox, dtype=torch.float64, device=beta.device)
    rc = load_library().mc_voxel_grad(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()), len(s.cameras),
                                      make_cameras(s.cameras), int(rays_per_side), C.c_void_p(j.data_ptr()),
                                      C.c_void_p(dl.data_ptr()), _ptr(q), C.c_void_p(g.data_ptr()),
                                      C.c_void_p(_stream(torch, stream)))
    _check("mc_voxel_grad", rc)
    return g


def mc_voxel_conditioning(s, rays_per_side=2, stream=None):
    """(counts, q) [n_cams * n_vox]: sub-pixel rays per camera and voxel, and q = 1/counts."""
    torch = _torch()
    n = len(s.cameras) * s.n_vox
    counts = torch.empty(n, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    rc = load_library().mc_voxel_conditioning(C.byref(make_grid(s)), len(s.cameras), make_cameras(s.cameras),
                                              int(rays_per_side), _ptr(counts), _ptr(q),
                                              C.c_void_p(_stream(torch, stream)))
    _check("mc_voxel_conditioning", rc)
    return counts, q


def mc_regularizer(s, beta, w_layer=None, eta=1.0, grad=None, stream=None):
    """(Psi as a 1-element tensor, grad with eta dPsi/dbeta added) of the Laplacian regulariser."""
    torch = _torch()
    b = _dev64(torch, beta, "cuda", s.n_vox, "beta")
    w = None if w_layer is None else _dev64(torch, w_layer, "cuda", s.nz, "w_layer")
    g = grad if grad is not None else torch.zeros(s.n_vox, dtype=torch.float64, device="cuda")
    val = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = load_library().mc_regularizer(C.byref(make_grid(s)), _ptr(b), _ptr(w), float(eta), _ptr(g), _ptr(val),
                                       C.c_void_p(_stream(torch, stream)))
    _check("mc_regularizer", rc)
    return val, g


def mc_image_residual(images, measured, mask=None, stream=None):
    """(dl = 2 mask^2 (images - measured), loss = |mask (images - measured)|^2)."""
    torch = _torch()
    i = _dev64(torch, images, "cuda")
    m = _dev64(torch, measured, "cuda", i.numel(), "measured")
    k = None if mask is None else _dev64(torch, mask, "cuda", i.numel(), "mask")
    dl = torch.empty_like(i)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = load_library().mc_image_residual(i.numel(), _ptr(i), _ptr(m), _ptr(k), _ptr(dl), _ptr(loss),
                                          C.c_void_p(_stream(torch, stream)))
    _check("mc_image_residual", rc)
    return dl, loss


def mc_gd_step(beta, grad, delta, stream=None):
    """In place: beta = max(beta - delta grad, 0) (beta: contiguous float64 CUDA tensor)."""
    torch = _torch()
    if not (beta.is_cuda and beta.dtype == torch.float64 and beta.is_contiguous()):
        raise ValueError("beta must be a contiguous float64 CUDA tensor")
    g = _dev64(torch, grad, beta.device, beta.numel(), "grad")
    _check("mc_gd_step", load_library().mc_gd_step(beta.numel(), _ptr(beta), _ptr(g), float(delta),
                                                   C.c_void_p(_stream(torch, stream))))
    return beta


def mc_camera_noise(images, normals, mask=None, stream=None):
    """Eq. (noise): (grey levels, scale as a 1-element tensor)."""
    torch = _torch()
    i = _dev64(torch, images, "cuda")
    z = _dev64(torch, normals, "cuda", i.numel(), "normals")
    k = None if mask is None else _dev64(torch, mask, "cuda", i.numel(), "mask")
    out = torch.empty_like(i)
    scale = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = load_library().mc_camera_noise(i.numel(), _ptr(i), _ptr(k), _ptr(z), _ptr(out), _ptr(scale),
                                        C.c_void_p(_stream(torch, stream)))
    _check("mc_camera_noise", rc)
    return out, scale


def mc_recovery_error(beta_hat, beta_true, stream=None):
    """(delta_mass, eps) of Sec. 7."""
    torch = _torch()
    b = _dev64(torch, beta_hat, "cuda")
    t = _dev64(torch, beta_true, "cuda", b.numel(), "beta_true")
    out = (C.c_double * 2)()
    _check("mc_recovery_error", load_library().mc_recovery_error(b.numel(), _ptr(b), _ptr(t), out,
                                                                 C.c_void_p(_stream(torch, stream))))
    return float(out[0]), float(out[1])


def mc_recover(s, beta0, measured, delta, n_gd, n_outer, rays_per_side=2, eta=0.0, w_layer=None, mask=None,
               conditioned=True, transport="fp32", stream=None, **kw):
    """The surrogate gradient-descent loop of Sec. 5.2 on the voxelised model.
    Returns (beta float64 tensor, cost numpy array [n_outer * n_gd])."""
    torch = _torch()
    b = _dev64(torch, beta0, "cuda", s.n_vox, "beta0").clone()
    m = _dev64(torch, measured, "cuda", n_pixels(s), "measured")
    k = None if mask is None else _dev64(torch, mask, "cuda", n_pixels(s), "mask")
    w = None if w_layer is None else _dev64(torch, w_layer, "cuda", s.nz, "w_layer")
    cost = (C.c_double * max(1, n_outer * n_gd))()
    rc = load_library().mc_recover(C.byref(make_grid(s)), _ptr(b), len(s.cameras), make_cameras(s.cameras),
                                   C.byref(make_params(s, transport=transport, **kw)), int(rays_per_side),
                                   _ptr(m), _ptr(k), _ptr(w), float(eta), float(delta), int(n_gd), int(n_outer),
                                   int(conditioned), cost, C.c_void_p(_stream(torch, stream)))
    _check("mc_recover", rc)
    return b, np.array(cost[:n_outer * n_gd])


def mc_trace_paths(s, beta, first_pid, count, max_rec, transport="fp32", with_pix=True,
                   stream=None, device=False, **kw):
    """Per-photon event records.  Returns numpy (events[count, max_rec], paths[count],
    pix[count, max_rec, n_cams] or None); unrecorded slots hold zeros / -2.  With
    device=True the records stay on the GPU: (events as raw bytes, a dict of path fields
    n_events, fate [count] int32, exit_pos [count, 3], exit_w [count] float64, and pix
    [count, max_rec, n_cams] int32 or None), all torch tensors."""
    torch = _torch()
    _check_beta(torch, s, beta, transport)
    dev = beta.device
    ev = torch.zeros(max(1, count * max_rec * EVENT_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    paths = torch.zeros(max(1, count * PATH_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    pix = (torch.full((max(1, count * max_rec * len(s.cameras)),), -2, dtype=torch.int32, device=dev)
           if with_pix else None)
    rc = load_library().mc_trace_paths(C.byref(make_grid(s)), C.c_void_p(beta.data_ptr()),
                                       len(s.cameras), make_cameras(s.cameras),
                                       C.byref(make_params(s, transport=transport, **kw)),
                                       int(first_pid), int(count), int(max_rec),
                                       C.c_void_p(ev.data_ptr() if max_rec > 0 else 0),
                                       C.c_void_p(pix.data_ptr() if with_pix else 0),
                                       C.c_void_p(paths.data_ptr()), C.c_void_p(_stream(torch, stream)))
    _check("mc_trace_paths", rc)
    if device:
        pi = paths[:count * PATH_DTYPE.itemsize].view(torch.int32).reshape(count, PATH_DTYPE.itemsize // 4)
        pf = paths[:count * PATH_DTYPE.itemsize].view(torch.float64).reshape(count, PATH_DTYPE.itemsize // 8)
        fields = {"n_events": pi[:, 0], "fate": pi[:, 1], "exit_pos": pf[:, 1:4], "exit_w": pf[:, 7]}
        px = pix[:count * max_rec * len(s.cameras)].reshape(count, max_rec, len(s.cameras)) if with_pix else None
        return ev, fields, px
    ev_np = ev.cpu().numpy()[:count * max_rec * EVENT_DTYPE.itemsize].view(EVENT_DTYPE)
    p_np = paths.cpu().numpy()[:count * PATH_DTYPE.itemsize].view(PATH_DTYPE)
    pix_np = (pix.cpu().numpy()[:count * max_rec * len(s.cameras)].reshape(count, max_rec, len(s.cameras))
              if with_pix else None)
    return ev_np.reshape(count, max_rec), p_np, pix_np


class MCRender:
    """torch.autograd.Function wrapper: images = render(beta); the backward
    pass returns the surrogate gradient (frozen in-scatter, Sec. 5.2) on the
    events of the same photon stream (or of `grad_seed` when given)."""

    @staticmethod
    def apply(beta, scene, transport="fp32", tally="f64", grad_seed=None, **kw):
        return _autograd_fn().apply(beta, scene, transport, tally, grad_seed, kw)


_fn = None


def _autograd_fn():
    global _fn
    if _fn is None:
        torch = _torch()

        class _MCRender(torch.autograd.Function):
            @staticmethod
            def forward(ctx, beta, scene, transport, tally, grad_seed, kw):
                b = beta_tensor(scene, transport, beta=beta, device=beta.device)
                ctx.tape = None
                if ctx.needs_input_grad[0] and grad_seed is None:
                    # keep the render's rays: the backward pass then needs no replay
                    img, _, ctx.tape = mc_render_tape(scene, b, transport=transport, tally=tally, stats=False,
                                                      **kw)
                else:
                    img, _ = mc_render(scene, b, transport=transport, tally=tally, stats=False, **kw)
                ctx.save_for_backward(b)
                ctx.scene, ctx.transport, ctx.tally, ctx.grad_seed, ctx.kw = scene, transport, tally, grad_seed, kw
                ctx.beta_dtype, ctx.beta_shape = beta.dtype, beta.shape
                return img

            @staticmethod
            def backward(ctx, g_img):
                (b,) = ctx.saved_tensors
                kw = dict(ctx.kw)
                if ctx.grad_seed is not None:
                    kw["seed"] = ctx.grad_seed
                g, _ = mc_grad_beta(ctx.scene, b, g_img, transport=ctx.transport, tally=ctx.tally,
                                    stats=False, tape=ctx.tape, **kw)
                if ctx.tape is not None:
                    ctx.tape.free()
                    ctx.tape = None
                return g.to(ctx.beta_dtype).reshape(ctx.beta_shape), None, None, None, None, None

        _fn = _MCRender
    return _fn


class MCRenderMixture:
    """torch.autograd.Function wrapper for one channel of the air + aerosol
    mixture (Eq. channelBeta): images = mc_render_mixture(beta_air,
    beta_aer, sigma); the backward pass returns dL/d beta_aer from
    mc_grad_mixture on the same photons, the full derivative (full=True,
    default) or the surrogate with the in-scatter field frozen.  beta_air is
    a constant (no gradient)."""

    @staticmethod
    def apply(beta_aer, scene, beta_air, sigma=1.0, full=True, transport="fp32", **kw):
        return _mixture_fn().apply(beta_aer, scene, beta_air, float(sigma), bool(full), transport, kw)


_mix_fn = None


def _mixture_fn():
    global _mix_fn
    if _mix_fn is None:
        torch = _torch()

        class _MCRenderMixture(torch.autograd.Function):
            @staticmethod
            def forward(ctx, beta_aer, scene, beta_air, sigma, full, transport, kw):
                aer = beta_aer.detach().to(dtype=torch.float64).contiguous().reshape(-1)
                air = beta_air.detach().to(device=aer.device, dtype=torch.float64).contiguous().reshape(-1)
                img, _ = mc_render_mixture(scene, air, aer, sigma, transport=transport, stats=False, **kw)
                ctx.save_for_backward(air, aer)
                ctx.scene, ctx.sigma, ctx.full, ctx.transport, ctx.kw = scene, sigma, full, transport, kw
                ctx.aer_dtype, ctx.aer_shape = beta_aer.dtype, beta_aer.shape
                return img

            @staticmethod
            def backward(ctx, g_img):
                air, aer = ctx.saved_tensors
                dl = g_img.detach().to(dtype=torch.float64).contiguous().reshape(-1)
                g, _ = mc_grad_mixture(ctx.scene, air, aer, dl, ctx.sigma, full=ctx.full, transport=ctx.transport,
                                       stats=False, **ctx.kw)
                return g.to(ctx.aer_dtype).reshape(ctx.aer_shape), None, None, None, None, None, None

        _mix_fn = _MCRenderMixture
    return _mix_fn

