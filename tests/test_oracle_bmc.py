"""Pins of the oracle's backward Monte Carlo renderer (Sec. 2.1.4, Eq. ble):
single scattering against the closed form of a homogeneous slab and against
quadrature on a heterogeneous grid with a camera inside, and multiple
scattering against the forward method (an independent estimator of the
same radiance)."""
import math

import numpy as np

from paper_1512_02110_amd import scenes
from tests._scene_helpers import look_camera, single_scatter_image, sun_direction
from tests.test_oracle_render import _slab_single_scatter


def _sigma(img, m2, n):
    return np.sqrt(np.maximum(m2 - img ** 2, 0.0) / n)


def test_bmc_single_scatter_slab_closed_form(oracle):
    tau, g, albedo, zen = 1.0, 0.5, 0.9, 30.0
    cam = look_camera((0.8, 0.8, -0.3), (0, 0, 1), (0, -1, 0), 8, 8, 40.0)
    s = scenes.homogeneous_slab(nx=16, ny=16, nz=4, dx=0.1, dz=0.05, tau=tau, albedo=albedo,
                                g=g, sun_zenith_deg=zen, cams=[cam])
    n = 20000
    img, st, m2 = oracle.bmc_render(s, n, with_m2=True, max_events=1)
    sigma = _sigma(img, m2, n)
    w_sun = sun_direction(s)
    mu0 = math.cos(s.sun_zenith)
    R = np.array(cam.R).reshape(3, 3)
    expect = np.zeros_like(img)
    k = 12
    for row in range(cam.height):
        for col in range(cam.width):
            vals = []
            for b in range(k):
                for a in range(k):
                    q = np.array([(col + (a + 0.5) / k - cam.cx) / cam.fx, (row + (b + 0.5) / k - cam.cy) / cam.fy, 1.0])
                    d = R.T @ q
                    d /= np.linalg.norm(d)
                    vals.append(_slab_single_scatter(d[2], float(w_sun @ -d), g, tau, mu0, albedo))
            expect[row * cam.width + col] = np.mean(vals)
    z = (img - expect) / sigma
    assert np.all(np.abs(z) < 5), z.reshape(8, 8)
    assert abs(img.sum() - expect.sum()) < 4 * math.sqrt((sigma ** 2).sum())
    assert st["events"] > 0 and st["capped"] == st["events"]


def test_bmc_single_scatter_heterogeneous_quadrature(oracle):
    """Single scattering on a 3x3x2 grid with an empty voxel, a camera below
    and a camera inside: quadrature of Eq. (IRTE) with the direct beam."""
    rng = np.random.default_rng(7)
    beta = rng.uniform(0.5, 12.0, size=3 * 3 * 2)
    beta[4] = 0.0
    cams = [look_camera((0.12, 0.17, -0.25), (0.1, 0.05, 1.0), (0, -1, 0), 4, 4, 70.0),
            look_camera((0.45, 0.1, 0.08), (-1.0, 0.3, 0.15), (0, 0, 1), 3, 5, 60.0, cx=1.2, cy=2.6)]
    s = scenes.Scene(3, 3, 2, 0.1, 0.1, 0.1, beta, cams, 0.8, 0.6, math.radians(35.0), 0.7, 1, 4)
    n = 20000
    img, _, m2 = oracle.bmc_render(s, n, with_m2=True, max_events=1)
    sigma = _sigma(img, m2, n)
    ref = np.concatenate([single_scatter_image(s, c, n_sub=24, uniform=True) for c in cams])
    tol = 4 * sigma + 0.005 * ref + 1e-3 * ref.max()
    assert np.all(np.abs(img - ref) <= tol), np.c_[img, ref, sigma]
    assert (ref > 0).sum() >= 15


def test_bmc_agrees_with_forward_method(oracle):
    """Multiple scattering (c1 blob, albedo 1, HG g 0.85, no cap): BMC and FMC
    estimate the same images; per camera and per 8x8 block of pixels they
    agree within 4.5 combined standard deviations."""
    s = scenes.config1(n_photons=400_000)
    n = 256
    bmc, _, bm2 = oracle.bmc_render(s, n, with_m2=True, seed=3)
    fmc, fst, fm2 = oracle.render(s, with_m2=True)
    N = fst["photons"]
    var_b = np.maximum(bm2 - bmc ** 2, 0.0) / n            # per pixel, independent packets
    var_f = np.maximum(fm2 - fmc ** 2 / N, 0.0)            # per pixel (lower bound)
    off = 0
    for cam in s.cameras:
        npix = cam.n_pix
        b = bmc[off:off + npix].reshape(cam.height, cam.width)
        f = fmc[off:off + npix].reshape(cam.height, cam.width)
        vb = var_b[off:off + npix].reshape(cam.height, cam.width)
        vf = var_f[off:off + npix].reshape(cam.height, cam.width)
        assert abs(b.sum() - f.sum()) < 4.5 * math.sqrt(vb.sum() + vf.sum()), (b.sum(), f.sum())
        for r0 in range(0, cam.height, 8):
            for c0 in range(0, cam.width, 8):
                sl = (slice(r0, r0 + 8), slice(c0, c0 + 8))
                d = b[sl].sum() - f[sl].sum()
                assert abs(d) < 4.5 * math.sqrt(vb[sl].sum() + vf[sl].sum()), (r0, c0, b[sl].sum(), f[sl].sum())
        off += npix


def test_bmc_empty_medium_is_dark(oracle):
    s = scenes.config1(n_photons=1).with_beta(np.zeros(16 ** 3))
    img, st = oracle.bmc_render(s, 4)
    assert not img.any() and st["events"] == 0
