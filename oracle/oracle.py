"""ctypes wrapper of the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.  The GPU library never loads it, and this
module imports nothing from the GPU package.  Scenes are passed duck-typed
(attributes nx, ny, nz, dx, dy, dz, beta, cameras, albedo, g, sun_zenith,
sun_azimuth, n_photons, seed).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "mcrt_oracle.c")]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-fno-fast-math", "-ffp-contract=off", "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Cam(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("R", C.c_double * 9), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("albedo", C.c_double), ("g", C.c_double), ("sun_zenith", C.c_double),
                ("sun_azimuth", C.c_double), ("rr_weight", C.c_double),
                ("n_photons", C.c_uint64), ("seed", C.c_uint64), ("photon_offset", C.c_uint64),
                ("n_photons_norm", C.c_uint64), ("max_events", C.c_uint32), ("pad_", C.c_int32)]


STAT_FIELDS = ["photons", "events", "le_jobs", "vox_free", "vox_conn", "esc_top", "esc_bottom",
               "esc_side", "rr_killed", "capped"]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_FIELDS]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n in STAT_FIELDS}


class Event(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("w", C.c_double),
                ("voxel", C.c_int32), ("pad_", C.c_int32)]


class Path(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("fate", C.c_int32), ("exit_pos", C.c_double * 3),
                ("exit_dir", C.c_double * 3), ("exit_w", C.c_double)]


EVENT_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("z", "<f8"), ("w", "<f8"),
                        ("voxel", "<i4"), ("pad_", "<i4")])
PATH_DTYPE = np.dtype([("n_events", "<i4"), ("fate", "<i4"), ("exit_pos", "<f8", (3,)),
                       ("exit_dir", "<f8", (3,)), ("exit_w", "<f8")])
FATES = {0: "top", 1: "bottom", 2: "side", 3: "rr", 4: "cap"}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.oracle_render.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.POINTER(Params),
                                    dp, dp, C.POINTER(Stats)]
        L.oracle_render_frozen.argtypes = [C.POINTER(Grid), dp, dp, C.c_int, C.POINTER(Cam),
                                           C.POINTER(Params), dp, C.POINTER(Stats)]
        L.oracle_grad_beta.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam),
                                       C.POINTER(Params), dp, dp, C.POINTER(Stats)]
        L.oracle_trace_paths.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam),
                                         C.POINTER(Params), C.c_uint64, C.c_uint32, C.c_uint32,
                                         C.c_void_p, C.c_void_p, C.c_void_p]
        for f in ("oracle_render", "oracle_render_frozen", "oracle_grad_beta", "oracle_trace_paths"):
            getattr(L, f).restype = C.c_int
        L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
        L.oracle_philox4x32_10.restype = None
        L.oracle_uniform.argtypes = [C.c_uint32]
        L.oracle_uniform.restype = C.c_double
        L.oracle_hg_phase.argtypes = [C.c_double, C.c_double]
        L.oracle_hg_phase.restype = C.c_double
        L.oracle_hg_sample.argtypes = [C.c_double, C.c_double]
        L.oracle_hg_sample.restype = C.c_double
        L.oracle_scatter_direction.argtypes = [dp, C.c_double, C.c_double, dp]
        L.oracle_scatter_direction.restype = None
        L.oracle_optical_depth.argtypes = [C.POINTER(Grid), dp, dp, dp, C.POINTER(C.c_int64)]
        L.oracle_optical_depth.restype = C.c_double
        L.oracle_pixel_solid_angle.argtypes = [C.POINTER(Cam), C.c_int, C.c_int]
        L.oracle_pixel_solid_angle.restype = C.c_double
        L.oracle_voxel_scatter.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.POINTER(Params),
                                           dp, C.POINTER(Stats)]
        L.oracle_voxel_transmittance.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), dp]
        L.oracle_voxel_render.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.c_int, dp, dp]
        L.oracle_voxel_grad.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.c_int, dp, dp, dp, dp]
        L.oracle_voxel_conditioning.argtypes = [C.POINTER(Grid), C.c_int, C.POINTER(Cam), C.c_int, dp, dp]
        L.oracle_voxel_conditioning.restype = C.c_int
        L.oracle_laplacian_reg.argtypes = [C.POINTER(Grid), dp, dp, dp]
        L.oracle_laplacian_reg.restype = C.c_double
        L.oracle_camera_noise.argtypes = [C.c_int64, dp, dp, dp, dp]
        L.oracle_camera_noise.restype = C.c_double
        L.oracle_recovery_error.argtypes = [C.c_int64, dp, dp, dp]
        L.oracle_recovery_error.restype = None
        L.oracle_recover.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.POINTER(Params), C.c_int,
                                     dp, dp, dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, dp]
        L.oracle_recover.restype = C.c_int
        L.oracle_bmc_render.argtypes = [C.POINTER(Grid), dp, C.c_int, C.POINTER(Cam), C.POINTER(Params),
                                        C.c_uint32, dp, dp, C.POINTER(Stats)]
        L.oracle_bmc_render.restype = C.c_int
        L.oracle_render_mix.argtypes = [C.POINTER(Grid), dp, dp, C.c_double, C.c_int, C.POINTER(Cam),
                                        C.POINTER(Params), dp, dp, C.POINTER(Stats)]
        L.oracle_render_mix.restype = C.c_int
        L.oracle_grad_mix.argtypes = [C.POINTER(Grid), dp, dp, C.c_double, C.c_int, C.POINTER(Cam),
                                      C.POINTER(Params), dp, C.c_int, dp, C.POINTER(Stats)]
        L.oracle_grad_mix.restype = C.c_int
        L.oracle_rayleigh_phase.argtypes = [C.c_double]
        L.oracle_rayleigh_phase.restype = C.c_double
        L.oracle_rayleigh_sample.argtypes = [C.c_double]
        L.oracle_rayleigh_sample.restype = C.c_double
        for f in ("oracle_voxel_scatter", "oracle_voxel_transmittance", "oracle_voxel_render",
                  "oracle_voxel_grad"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(s) -> Grid:
    return Grid(int(s.nx), int(s.ny), int(s.nz), 0, float(s.dx), float(s.dy), float(s.dz))


def make_cams(cameras):
    arr = (Cam * max(1, len(cameras)))()
    for i, c in enumerate(cameras):
        arr[i].pos[:] = [float(v) for v in c.pos]
        arr[i].R[:] = [float(v) for v in c.R]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[i].width, arr[i].height = int(c.width), int(c.height)
    return arr


def make_params(s, n_photons=None, seed=None, photon_offset=0, n_photons_norm=0,
                max_events=100000, rr_weight=0.1) -> Params:
    return Params(float(s.albedo), float(s.g), float(s.sun_zenith), float(s.sun_azimuth),
                  float(rr_weight), int(s.n_photons if n_photons is None else n_photons),
                  int(s.seed if seed is None else seed), int(photon_offset), int(n_photons_norm),
                  int(max_events), 0)


def _beta(s, beta=None):
    b = s.beta if beta is None else beta
    return np.ascontiguousarray(b, dtype=np.float64).reshape(-1)


def _n_pix(cameras):
    return sum(int(c.width) * int(c.height) for c in cameras)


def split_images(flat, cameras):
    out, o = [], 0
    for c in cameras:
        n = int(c.width) * int(c.height)
        out.append(flat[o:o + n].reshape(int(c.height), int(c.width)))
        o += n
    return out


def render(s, beta=None, with_m2=False, **kw):
    """Returns (images_flat, stats_dict[, m2_flat])."""
    b = _beta(s, beta)
    img = np.zeros(_n_pix(s.cameras))
    m2 = np.zeros_like(img) if with_m2 else None
    st = Stats()
    rc = lib().oracle_render(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                             C.byref(make_params(s, **kw)), _dptr(img),
                             _dptr(m2) if with_m2 else None, C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_render failed: {rc}")
    return (img, st.as_dict(), m2) if with_m2 else (img, st.as_dict())


def render_frozen(s, beta_sample, beta_eval, **kw):
    bs, be = _beta(s, beta_sample), _beta(s, beta_eval)
    img = np.zeros(_n_pix(s.cameras))
    st = Stats()
    rc = lib().oracle_render_frozen(C.byref(make_grid(s)), _dptr(bs), _dptr(be), len(s.cameras),
                                    make_cams(s.cameras), C.byref(make_params(s, **kw)), _dptr(img),
                                    C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_render_frozen failed: {rc}")
    return img, st.as_dict()


def grad_beta(s, dl_dimages, beta=None, **kw):
    b = _beta(s, beta)
    dl = np.ascontiguousarray(dl_dimages, dtype=np.float64).reshape(-1)
    if dl.size != _n_pix(s.cameras):
        raise ValueError("dl_dimages size mismatch")
    grad = np.zeros(b.size)
    st = Stats()
    rc = lib().oracle_grad_beta(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                C.byref(make_params(s, **kw)), _dptr(dl), _dptr(grad), C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_grad_beta failed: {rc}")
    return grad, st.as_dict()


def render_mix(s, beta_air, beta_aer, sigma=1.0, with_m2=False, **kw):
    """Air + aerosol mixture render of one channel: extinction beta_air +
    sigma * beta_aer, the scene's albedo and g for the aerosol.  Returns
    (images_flat, stats_dict[, m2_flat])."""
    ba, bs = _beta(s, beta_air), _beta(s, beta_aer)
    img = np.zeros(_n_pix(s.cameras))
    m2 = np.zeros_like(img) if with_m2 else None
    st = Stats()
    rc = lib().oracle_render_mix(C.byref(make_grid(s)), _dptr(ba), _dptr(bs), float(sigma), len(s.cameras),
                                 make_cams(s.cameras), C.byref(make_params(s, **kw)), _dptr(img),
                                 _dptr(m2) if with_m2 else None, C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_render_mix failed: {rc}")
    return (img, st.as_dict(), m2) if with_m2 else (img, st.as_dict())


def grad_mix(s, dl_dimages, beta_air, beta_aer, sigma=1.0, full=False, grad=None, **kw):
    """dL/d beta_aer of the mixture (surrogate, or full with path scores),
    added to grad (a new zero array when None).  Returns (grad, stats)."""
    ba, bs = _beta(s, beta_air), _beta(s, beta_aer)
    dl = np.ascontiguousarray(dl_dimages, dtype=np.float64).reshape(-1)
    if dl.size != _n_pix(s.cameras):
        raise ValueError("dl_dimages size mismatch")
    g = np.zeros(ba.size) if grad is None else grad
    st = Stats()
    rc = lib().oracle_grad_mix(C.byref(make_grid(s)), _dptr(ba), _dptr(bs), float(sigma), len(s.cameras),
                               make_cams(s.cameras), C.byref(make_params(s, **kw)), _dptr(dl), int(bool(full)),
                               _dptr(g), C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_grad_mix failed: {rc}")
    return g, st.as_dict()


def rayleigh_phase(cos_angle):
    return lib().oracle_rayleigh_phase(float(cos_angle))


def rayleigh_sample(u):
    return lib().oracle_rayleigh_sample(float(u))


def trace_paths(s, first_pid, count, max_rec, beta=None, with_pix=True, **kw):
    """Returns (events[count, max_rec] structured, paths[count] structured,
    pix[count, max_rec, n_cams] or None)."""
    b = _beta(s, beta)
    ev = np.zeros((count, max_rec), dtype=EVENT_DTYPE)
    paths = np.zeros(count, dtype=PATH_DTYPE)
    pix = np.full((count, max_rec, len(s.cameras)), -2, dtype=np.int32) if with_pix else None
    rc = lib().oracle_trace_paths(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                  C.byref(make_params(s, **kw)), int(first_pid), int(count),
                                  int(max_rec), ev.ctypes.data, pix.ctypes.data if with_pix else None,
                                  paths.ctypes.data)
    if rc != 0:
        raise OracleError(f"oracle_trace_paths failed: {rc}")
    return ev, paths, pix


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(x):
    return lib().oracle_uniform(int(x) & 0xFFFFFFFF)


def hg_phase(g, cos_angle):
    return lib().oracle_hg_phase(float(g), float(cos_angle))


def hg_sample(g, u):
    return lib().oracle_hg_sample(float(g), float(u))


def scatter_direction(w, mu, phi):
    wi = np.ascontiguousarray(w, dtype=np.float64)
    wo = np.zeros(3)
    lib().oracle_scatter_direction(_dptr(wi), float(mu), float(phi), _dptr(wo))
    return wo


def optical_depth(s, p0, p1, beta=None):
    b = _beta(s, beta)
    a0 = np.ascontiguousarray(p0, dtype=np.float64)
    a1 = np.ascontiguousarray(p1, dtype=np.float64)
    nv = C.c_int64(0)
    tau = lib().oracle_optical_depth(C.byref(make_grid(s)), _dptr(b), _dptr(a0), _dptr(a1), C.byref(nv))
    return tau, int(nv.value)


def pixel_solid_angle(cam, row, col):
    return lib().oracle_pixel_solid_angle(make_cams([cam]), int(row), int(col))


def normalisation(s, n_photons=None):
    """Per-pixel mu0 A_top / (N Omega_p) as the oracle applies it."""
    import math
    N = s.n_photons if n_photons is None else n_photons
    base = math.cos(s.sun_zenith) * s.nx * s.dx * s.ny * s.dy / N
    out = []
    for c in s.cameras:
        om = np.array([[pixel_solid_angle(c, r, q) for q in range(c.width)] for r in range(c.height)])
        out.append((base / om).reshape(-1))
    return np.concatenate(out)


# Voxelised forward model (Sec. 3): arrays [camera][voxel] are returned as
# (n_cams, n_vox) numpy arrays.

def voxel_scatter(s, beta=None, **kw):
    """j_c(k) of Eq. (Jc) from a FMC run without local estimation; (j, stats)."""
    b = _beta(s, beta)
    j = np.zeros(len(s.cameras) * b.size)
    st = Stats()
    rc = lib().oracle_voxel_scatter(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                    C.byref(make_params(s, **kw)), _dptr(j), C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_voxel_scatter failed: {rc}")
    return j.reshape(len(s.cameras), b.size), st.as_dict()


def voxel_transmittance(s, beta=None):
    b = _beta(s, beta)
    T = np.zeros(len(s.cameras) * b.size)
    rc = lib().oracle_voxel_transmittance(C.byref(make_grid(s)), _dptr(b), len(s.cameras),
                                          make_cams(s.cameras), _dptr(T))
    if rc != 0:
        raise OracleError(f"oracle_voxel_transmittance failed: {rc}")
    return T.reshape(len(s.cameras), b.size)


def voxel_render(s, j, n_rays_side, beta=None):
    """Images of Eq. (Icpixel) with n x n sub-pixel rays (flat, like render)."""
    b = _beta(s, beta)
    jj = np.ascontiguousarray(j, dtype=np.float64).reshape(-1)
    if jj.size != len(s.cameras) * b.size:
        raise ValueError("j must hold one value per camera and voxel")
    img = np.zeros(_n_pix(s.cameras))
    rc = lib().oracle_voxel_render(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                   int(n_rays_side), _dptr(jj), _dptr(img))
    if rc != 0:
        raise OracleError(f"oracle_voxel_render failed: {rc}")
    return img


def voxel_grad(s, j, dl_dimages, n_rays_side, beta=None, q=None):
    """dL/dbeta of the voxelised images for dL/di = dl_dimages, j frozen;
    with q ([camera][voxel]) each camera's term is weighted (conditioning)."""
    b = _beta(s, beta)
    jj = np.ascontiguousarray(j, dtype=np.float64).reshape(-1)
    dl = np.ascontiguousarray(dl_dimages, dtype=np.float64).reshape(-1)
    if jj.size != len(s.cameras) * b.size or dl.size != _n_pix(s.cameras):
        raise ValueError("size mismatch")
    qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    g = np.zeros(b.size)
    rc = lib().oracle_voxel_grad(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                 int(n_rays_side), _dptr(jj), _dptr(dl), _dptr(qq) if qq is not None else None,
                                 _dptr(g))
    if rc != 0:
        raise OracleError(f"oracle_voxel_grad failed: {rc}")
    return g


# Recovery (Secs. 5.2, 6, 7).

def voxel_conditioning(s, n_rays_side):
    """(counts, q): sub-pixel rays per camera and voxel, and q = 1/counts (0 where none)."""
    n = len(s.cameras) * s.nx * s.ny * s.nz
    counts, q = np.zeros(n), np.zeros(n)
    rc = lib().oracle_voxel_conditioning(C.byref(make_grid(s)), len(s.cameras), make_cams(s.cameras),
                                         int(n_rays_side), _dptr(counts), _dptr(q))
    if rc != 0:
        raise OracleError(f"oracle_voxel_conditioning failed: {rc}")
    shape = (len(s.cameras), s.nx * s.ny * s.nz)
    return counts.reshape(shape), q.reshape(shape)


def laplacian_reg(s, beta=None, w_layer=None):
    """(Psi, dPsi/dbeta) of the Laplacian regulariser."""
    b = _beta(s, beta)
    w = None if w_layer is None else np.ascontiguousarray(w_layer, dtype=np.float64)
    g = np.zeros(b.size)
    psi = lib().oracle_laplacian_reg(C.byref(make_grid(s)), _dptr(b), _dptr(w) if w is not None else None,
                                     _dptr(g))
    return psi, g


def camera_noise(images, normals, mask=None):
    """Eq. (noise): (grey levels, scale)."""
    im = np.ascontiguousarray(images, dtype=np.float64).reshape(-1)
    nz = np.ascontiguousarray(normals, dtype=np.float64).reshape(-1)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.float64).reshape(-1)
    out = np.zeros(im.size)
    scale = lib().oracle_camera_noise(im.size, _dptr(im), _dptr(m) if m is not None else None, _dptr(nz),
                                      _dptr(out))
    return out, scale


def recovery_error(beta_hat, beta_true):
    """(delta_mass, eps) of Sec. 7."""
    a = np.ascontiguousarray(beta_hat, dtype=np.float64).reshape(-1)
    t = np.ascontiguousarray(beta_true, dtype=np.float64).reshape(-1)
    out = np.zeros(2)
    lib().oracle_recovery_error(a.size, _dptr(a), _dptr(t), _dptr(out))
    return float(out[0]), float(out[1])


def recover(s, beta0, measured, n_rays_side, delta, n_gd, n_outer, eta=0.0, w_layer=None, mask=None,
            conditioned=True, **kw):
    """The surrogate gradient-descent loop; returns (beta, cost[n_outer * n_gd]).
    conditioned: False/0 none, True/1 Q_c = 1/count, 2 Q_c = count."""
    b = np.array(beta0, dtype=np.float64).reshape(-1).copy()
    meas = np.ascontiguousarray(measured, dtype=np.float64).reshape(-1)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.float64).reshape(-1)
    w = None if w_layer is None else np.ascontiguousarray(w_layer, dtype=np.float64)
    cost = np.zeros(max(1, n_outer * n_gd))
    rc = lib().oracle_recover(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                              C.byref(make_params(s, **kw)), int(n_rays_side), _dptr(meas),
                              _dptr(m) if m is not None else None, _dptr(w) if w is not None else None,
                              float(eta), float(delta), int(n_gd), int(n_outer), int(conditioned),
                              _dptr(cost))
    if rc != 0:
        raise OracleError(f"oracle_recover failed: {rc}")
    return b, cost[:n_outer * n_gd]


def bmc_render(s, n_per_pixel, beta=None, with_m2=False, **kw):
    """Backward Monte Carlo images (Sec. 2.1.4, Eq. ble): (images_flat, stats[, m2_flat]),
    m2 = mean squared packet sum per pixel."""
    b = _beta(s, beta)
    img = np.zeros(_n_pix(s.cameras))
    m2 = np.zeros_like(img) if with_m2 else None
    st = Stats()
    rc = lib().oracle_bmc_render(C.byref(make_grid(s)), _dptr(b), len(s.cameras), make_cams(s.cameras),
                                 C.byref(make_params(s, **kw)), int(n_per_pixel), _dptr(img),
                                 _dptr(m2) if with_m2 else None, C.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_bmc_render failed: {rc}")
    return (img, st.as_dict(), m2) if with_m2 else (img, st.as_dict())

