"""Seeded synthetic scenes: extinction grids, in-situ pinhole cameras, sun and
photon budget.

This module only *describes inputs*.  It holds none of the renderer's
arithmetic (no transport, no phase function, no transmittance, no image
normalisation), so both the HIP library and the CPU oracle can be fed from it
without sharing any of the method.

Geometry follows the voxelised model of the paper (Sec. 3): the domain is
[0, nx*dx] x [0, ny*dy] x [0, nz*dz] km with z up, the extinction beta is
constant inside each voxel and is sampled at voxel centres.  The voxel vector
is column-stacked with x fastest: k = ix + nx*(iy + ny*iz).

The paper's own scenes (Atm1-4, Sec. 4) come from an external data set that
is not available here; the fields below are seeded synthetic stand-ins with
cloud-like structure (a Gaussian blob, thresholded fractal value noise and a
multi-cloud field).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Camera:
    """Pinhole camera.  ``R`` maps world to camera coordinates (rows are the
    camera's x-right, y-down and z-forward axes); a world point X projects to
    column u = fx*qx/qz + cx and row v = fy*qy/qz + cy with q = R (X - pos)."""

    pos: tuple
    R: tuple  # 9 floats, row-major
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def n_pix(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    beta: np.ndarray  # float64, shape (nx*ny*nz,), x fastest
    cameras: List[Camera]
    albedo: float
    g: float
    sun_zenith: float  # rad, zenith angle of the direction towards the sun
    sun_azimuth: float  # rad, from +x towards +y
    n_photons: int
    seed: int = 0
    name: str = ""

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_cams(self) -> int:
        return len(self.cameras)

    @property
    def image_shapes(self):
        return [(c.height, c.width) for c in self.cameras]

    @property
    def n_pix_total(self) -> int:
        return sum(c.n_pix for c in self.cameras)

    def beta3d(self) -> np.ndarray:
        """beta viewed as [iz][iy][ix]."""
        return self.beta.reshape(self.nz, self.ny, self.nx)

    def with_beta(self, beta: np.ndarray) -> "Scene":
        s = dataclasses.replace(self)
        s.beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
        return s

    def replace(self, **kw) -> "Scene":
        s = dataclasses.replace(self, **kw)
        if "beta" in kw:
            s.beta = np.ascontiguousarray(kw["beta"], dtype=np.float64).reshape(-1)
        return s


# ----------------------------------------------------------------------------
# cameras

def upward_camera(x: float, y: float, z: float, width: int, height: int,
                  fov_deg: float) -> Camera:
    """Ground camera looking straight up (+z).  With R = I the image column
    grows with +x and the row with +y.  ``fov_deg`` is the full field of view
    across the image width; square pixels."""
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(pos=(float(x), float(y), float(z)),
                  R=(1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0),
                  fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height))


def camera_lattice(n_side: int, lx: float, ly: float, width: int, height: int,
                   fov_deg: float, z: float = 0.0) -> List[Camera]:
    """n_side x n_side ground cameras at ((i+1/2)/n_side) of the footprint."""
    cams = []
    for j in range(n_side):
        for i in range(n_side):
            cams.append(upward_camera((i + 0.5) / n_side * lx, (j + 0.5) / n_side * ly,
                                      z, width, height, fov_deg))
    return cams


# ----------------------------------------------------------------------------
# extinction fields

def voxel_centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * d


def gaussian_blob(nx, ny, nz, dx, dy, dz, peak, sigma, centre) -> np.ndarray:
    """peak * exp(-|X - centre|^2 / (2 sigma^2)) at voxel centres."""
    x = voxel_centres(nx, dx)[None, None, :]
    y = voxel_centres(ny, dy)[None, :, None]
    z = voxel_centres(nz, dz)[:, None, None]
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return peak * np.exp(-r2 / (2.0 * sigma * sigma))


def _smoothstep(f):
    return f * f * (3.0 - 2.0 * f)


def value_noise(nx, ny, nz, dx, dy, dz, seed, octaves=4, base_cells=4) -> np.ndarray:
    """Fractal 3D value noise in [0, 1] at voxel centres, shape [nz][ny][nx].

    Octave o uses a lattice of spacing L_max / (base_cells * 2**o), lattice
    values uniform in [0,1) drawn from ``np.random.default_rng(seed)`` (one
    generator, octaves drawn in order), smoothstep-weighted trilinear
    interpolation and amplitude 2**-o.  The sum is divided by the sum of the
    amplitudes."""
    rng = np.random.default_rng(seed)
    L = np.array([nx * dx, ny * dy, nz * dz])
    lmax = float(L.max())
    coords = [voxel_centres(nx, dx), voxel_centres(ny, dy), voxel_centres(nz, dz)]
    total = np.zeros((nz, ny, nx))
    amp_sum = 0.0
    for o in range(octaves):
        spacing = lmax / (base_cells * 2 ** o)
        ncell = [int(math.ceil(L[a] / spacing - 1e-9)) for a in range(3)]
        lat = rng.random((ncell[2] + 1, ncell[1] + 1, ncell[0] + 1))
        idx, wts = [], []
        for a in range(3):
            p = coords[a] / spacing
            i0 = np.minimum(np.floor(p).astype(np.int64), ncell[a] - 1)
            idx.append(i0)
            wts.append(_smoothstep(p - i0))
        ix, iy, iz = idx
        wx, wy, wz = wts
        ix = ix[None, None, :]
        iy = iy[None, :, None]
        iz = iz[:, None, None]
        wx = wx[None, None, :]
        wy = wy[None, :, None]
        wz = wz[:, None, None]
        acc = np.zeros((nz, ny, nx))
        for cz in (0, 1):
            fz = wz if cz else 1.0 - wz
            for cy in (0, 1):
                fy = wy if cy else 1.0 - wy
                for cx in (0, 1):
                    fx = wx if cx else 1.0 - wx
                    acc = acc + fz * fy * fx * lat[iz + cz, iy + cy, ix + cx]
        amp = 0.5 ** o
        total += amp * acc
        amp_sum += amp
    return total / amp_sum


def threshold_scale(n: np.ndarray, thresh: float, beta_max: float) -> np.ndarray:
    """beta_max * max(0, n - thresh) / (max(n) - thresh)."""
    top = float(n.max())
    if top <= thresh:
        return np.zeros_like(n)
    return beta_max * np.maximum(0.0, n - thresh) / (top - thresh)


def multi_cloud(nx, ny, nz, dx, dy, dz, seed, n_clouds=8) -> np.ndarray:
    """Fractal noise (seeded) modulated by a sum of seeded anisotropic
    Gaussian envelopes (horizontal sigma 0.4-1.0 km, vertical 0.3-0.6 km),
    rescaled to [0, 1]."""
    noise = value_noise(nx, ny, nz, dx, dy, dz, seed)
    rng = np.random.default_rng(seed + 1000)
    L = (nx * dx, ny * dy, nz * dz)
    x = voxel_centres(nx, dx)[None, None, :]
    y = voxel_centres(ny, dy)[None, :, None]
    z = voxel_centres(nz, dz)[:, None, None]
    env = np.zeros((nz, ny, nx))
    for _ in range(n_clouds):
        c = (rng.uniform(0.15, 0.85) * L[0], rng.uniform(0.15, 0.85) * L[1],
             rng.uniform(0.3, 0.7) * L[2])
        sh = rng.uniform(0.4, 1.0)
        sv = rng.uniform(0.3, 0.6)
        env += np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2 * sh * sh)
                      - (z - c[2]) ** 2 / (2 * sv * sv))
    env = np.minimum(env, 1.0)
    m = noise * env
    return m / m.max()


def smooth(beta3d: np.ndarray, sigma_vox: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(beta3d, sigma=sigma_vox, mode="nearest")


# ----------------------------------------------------------------------------
# the five workloads

def _flat(b3):
    return np.ascontiguousarray(b3, dtype=np.float64).reshape(-1)


def config1(n_photons: int = 100_000, seed: int = 0) -> Scene:
    """16^3 voxels of 0.05 km; beta = 10 exp(-r^2 / (2 0.2^2)) km^-1 about
    the domain centre; albedo 1, g 0.85, sun zenith 30 deg; 4 upward cameras
    of 32x32 px, 60 deg FOV, at x, y in {0.2, 0.6} km on the floor."""
    n, d = 16, 0.05
    b = gaussian_blob(n, n, n, d, d, d, 10.0, 0.2, (0.4, 0.4, 0.4))
    cams = [upward_camera(x, y, 0.0, 32, 32, 60.0) for y in (0.2, 0.6) for x in (0.2, 0.6)]
    return Scene(n, n, n, d, d, d, _flat(b), cams, 1.0, 0.85, math.radians(30.0), 0.0,
                 n_photons, seed, "c1")


def config2(n_photons: int = 100_000_000, seed: int = 0) -> Scene:
    """64^3 voxels of 0.02 km; 4-octave value noise (seed 2) thresholded at
    0.55 and scaled to max 50 km^-1; albedo 0.99, g 0.85, sun zenith 45 deg;
    3x3 upward cameras of 128x128 px, 70 deg FOV."""
    n, d = 64, 0.02
    b = threshold_scale(value_noise(n, n, n, d, d, d, seed=2), 0.55, 50.0)
    cams = camera_lattice(3, n * d, n * d, 128, 128, 70.0)
    return Scene(n, n, n, d, d, d, _flat(b), cams, 0.99, 0.85, math.radians(45.0), 0.0,
                 n_photons, seed, "c2")


def config3_truth(n_photons: int = 100_000_000, seed: int = 0) -> Scene:
    s = config1(n_photons, seed)
    s.albedo = 1.0
    s.name = "c3-truth"
    return s


def config3_initial(n_photons: int = 100_000_000, seed: int = 0) -> Scene:
    """beta0 = 0.7 * gaussian_filter(beta_true, 1 voxel, mode 'nearest')."""
    s = config3_truth(n_photons, seed)
    b0 = 0.7 * smooth(s.beta3d(), 1.0)
    s = s.with_beta(b0)
    s.name = "c3-init"
    return s


def config4(n_photons: int = 1_000_000_000, seed: int = 0) -> Scene:
    """128^3 voxels of 0.02 km; value noise (seed 4) scaled to max 80 km^-1;
    albedo 0.999, g 0.85, sun zenith 20 deg; 5x5 cameras of 256x256, 70 deg."""
    n, d = 128, 0.02
    b = threshold_scale(value_noise(n, n, n, d, d, d, seed=4), 0.55, 80.0)
    cams = camera_lattice(5, n * d, n * d, 256, 256, 70.0)
    return Scene(n, n, n, d, d, d, _flat(b), cams, 0.999, 0.85, math.radians(20.0), 0.0,
                 n_photons, seed, "c4")


def config5(n_photons: int = 2_000_000_000, seed: int = 1000) -> Scene:
    """256x256x128 voxels of 0.02 km; multi-cloud field (seed 5) thresholded
    at 0.55, max 100 km^-1; albedo 0.999, g 0.85, sun zenith 45 deg; 6x6
    cameras of 256x256, 70 deg."""
    nx, ny, nz, d = 256, 256, 128, 0.02
    b = threshold_scale(multi_cloud(nx, ny, nz, d, d, d, seed=5), 0.55, 100.0)
    cams = camera_lattice(6, nx * d, ny * d, 256, 256, 70.0)
    return Scene(nx, ny, nz, d, d, d, _flat(b), cams, 0.999, 0.85, math.radians(45.0), 0.0,
                 n_photons, seed, "c5")


def homogeneous_slab(nx=64, ny=64, nz=4, dx=0.25, dz=0.05, tau=1.0, albedo=1.0, g=0.85,
                     sun_zenith_deg=30.0, cams: Sequence[Camera] | None = None,
                     n_photons=100_000, seed=0) -> Scene:
    """Laterally wide homogeneous slab of vertical optical depth ``tau``."""
    H = nz * dz
    b = np.full(nx * ny * nz, tau / H)
    if cams is None:
        cams = [upward_camera(nx * dx / 2, ny * dx / 2, 0.0, 16, 16, 60.0)]
    return Scene(nx, ny, nz, dx, dx, dz, b, list(cams), albedo, g,
                 math.radians(sun_zenith_deg), 0.0, n_photons, seed, "slab")


def random_scene(rng: np.random.Generator, nx=5, ny=4, nz=3, n_cams=3, sparsity=0.3,
                 bmax=8.0, W=9, H=7, n_photons=2000) -> Scene:
    """Small irregular scene for edge-case tests: non-cubic voxels, zeros in
    beta, odd image sizes, cameras inside, on and outside the domain."""
    dx, dy, dz = rng.uniform(0.05, 0.2, size=3)
    b = rng.uniform(0.0, bmax, size=nx * ny * nz)
    b[rng.random(b.size) < sparsity] = 0.0
    L = (nx * dx, ny * dy, nz * dz)
    cams = []
    for c in range(n_cams):
        x = rng.uniform(-0.2, 1.2) * L[0]
        y = rng.uniform(-0.2, 1.2) * L[1]
        z = rng.choice([0.0, rng.uniform(-0.3, 0.5) * L[2]])
        cams.append(upward_camera(x, y, float(z), W, H, float(rng.uniform(40, 120))))
    return Scene(nx, ny, nz, dx, dy, dz, b, cams, float(rng.uniform(0.5, 1.0)),
                 float(rng.uniform(-0.6, 0.9)), float(rng.uniform(0.0, 1.3)),
                 float(rng.uniform(0, 2 * math.pi)), n_photons, int(rng.integers(0, 2**40)),
                 "random")


CONFIGS = {"c1": config1, "c2": config2, "c3": config3_initial, "c4": config4, "c5": config5}
