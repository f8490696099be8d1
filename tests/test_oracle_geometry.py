"""Pins of the oracle's voxel traversal (optical depth as a sum of
intersection lengths times beta, Eq. (taoKtoc)), of the Beer-Lambert law
Eq. (beer-lambert) as realised by free-path sampling, and of the pixel solid
angles used in the image normalisation."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1512_02110_amd import scenes


def _brute_tau(s, p0, p1, n=200_000):
    """Midpoint Riemann sum of beta along p0->p1 with voxel lookup by floor."""
    p0, p1 = np.asarray(p0, float), np.asarray(p1, float)
    L = np.linalg.norm(p1 - p0)
    t = (np.arange(n) + 0.5) / n
    pts = p0[None, :] + t[:, None] * (p1 - p0)[None, :]
    ix = np.floor(pts[:, 0] / s.dx).astype(int)
    iy = np.floor(pts[:, 1] / s.dy).astype(int)
    iz = np.floor(pts[:, 2] / s.dz).astype(int)
    inside = (ix >= 0) & (ix < s.nx) & (iy >= 0) & (iy < s.ny) & (iz >= 0) & (iz < s.nz)
    b = np.zeros(n)
    b[inside] = s.beta[ix[inside] + s.nx * (iy[inside] + s.ny * iz[inside])]
    return b.sum() * L / n, len({(a, b_, c) for a, b_, c in zip(ix[inside], iy[inside], iz[inside])})


def _rand_scene(seed):
    rng = np.random.default_rng(seed)
    return scenes.random_scene(rng, nx=7, ny=5, nz=6, sparsity=0.2), rng


@pytest.mark.parametrize("seed", range(6))
def test_optical_depth_matches_riemann_sum(oracle, seed):
    s, rng = _rand_scene(seed)
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    for _ in range(25):
        p0 = rng.uniform(-0.3, 1.3, 3) * L
        p1 = rng.uniform(-0.3, 1.3, 3) * L
        tau, nvox = oracle.optical_depth(s, p0, p1)
        ref, ndistinct = _brute_tau(s, p0, p1)
        seg = np.linalg.norm(p1 - p0)
        # Riemann error: a handful of boundary samples of width seg/n
        assert abs(tau - ref) <= 8 * s.beta.max() * seg / 200_000 + 1e-12
        if ndistinct:
            # the traversal visits every voxel the segment crosses (plus
            # possibly voxels touched at a single edge/corner point)
            assert nvox >= ndistinct


def test_optical_depth_axis_aligned_is_exact_sum(oracle):
    s, _ = _rand_scene(11)
    b3 = s.beta3d()
    for iy in range(s.ny):
        for iz in range(s.nz):
            y, z = (iy + 0.3) * s.dy, (iz + 0.6) * s.dz
            tau, nvox = oracle.optical_depth(s, [-1.0, y, z], [s.nx * s.dx + 1.0, y, z])
            assert abs(tau - b3[iz, iy, :].sum() * s.dx) < 1e-12 * (1 + tau)
            assert nvox == s.nx
            tau_r, _ = oracle.optical_depth(s, [s.nx * s.dx + 1.0, y, z], [-1.0, y, z])
            assert abs(tau_r - tau) < 1e-12 * (1 + tau)


def test_optical_depth_partial_voxels_and_reversal(oracle):
    s, rng = _rand_scene(5)
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    for _ in range(50):
        a, b = rng.uniform(0, 1, 3) * L, rng.uniform(0, 1, 3) * L
        m = 0.37 * a + 0.63 * b
        t_ab, _ = oracle.optical_depth(s, a, b)
        t_ba, _ = oracle.optical_depth(s, b, a)
        t_am, _ = oracle.optical_depth(s, a, m)
        t_mb, _ = oracle.optical_depth(s, m, b)
        assert abs(t_ab - t_ba) < 1e-12 * (1 + t_ab)
        assert abs(t_ab - (t_am + t_mb)) < 1e-12 * (1 + t_ab)


def test_uncollided_transmission_follows_beer_lambert(oracle):
    # A photon launched at the top leaves through the bottom without a
    # collision with probability exp(-tau) along its launch ray.  The launch
    # point uses leg 0 of the photon's Philox stream (uniforms 0 and 1).
    s = scenes.config2(n_photons=6000)
    n = 6000
    ev, paths, _ = oracle.trace_paths(s, 0, n, 1, with_pix=False)
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    w = -np.array([math.sin(s.sun_zenith) * math.cos(s.sun_azimuth),
                   math.sin(s.sun_zenith) * math.sin(s.sun_azimuth), math.cos(s.sun_zenith)])
    probs, hits = [], []
    for pid in range(n):
        r = oracle.philox([pid, 0, 0, 0], [s.seed & 0xFFFFFFFF, s.seed >> 32])
        p0 = np.array([oracle.uniform(r[0]) * L[0], oracle.uniform(r[1]) * L[1], L[2]])
        # far end: well beyond the domain along w
        tau, _ = oracle.optical_depth(s, p0, p0 + 10 * L.max() * w)
        probs.append(math.exp(-tau))
        hits.append(paths["n_events"][pid] == 0)
    probs, hits = np.array(probs), np.array(hits, float)
    sigma = math.sqrt((probs * (1 - probs)).sum())
    assert abs(hits.sum() - probs.sum()) < 4 * sigma + 1e-9
    # and uncollided photons left through the bottom or a side face only
    assert set(paths["fate"][paths["n_events"] == 0]) <= {1, 2}


def test_slab_uncollided_fraction(oracle):
    # Homogeneous wide slab, tau = 1, sun zenith 30 deg: photons leaving the
    # bottom uncollided ~ exp(-tau / mu0) (lateral exits removed by a wide box).
    s = scenes.homogeneous_slab(nx=8, ny=8, nz=4, dx=2.0, dz=0.05, tau=1.0, sun_zenith_deg=30.0,
                                n_photons=40000)
    ev, paths, _ = oracle.trace_paths(s, 0, 40000, 1, with_pix=False)
    p = math.exp(-1.0 / math.cos(math.radians(30)))
    unc = ((paths["n_events"] == 0) & (paths["fate"] == 1)).mean()
    side = ((paths["n_events"] == 0) & (paths["fate"] == 2)).mean()
    assert side < 0.01
    assert abs(unc + side - p) < 4 * math.sqrt(p * (1 - p) / 40000)


@pytest.mark.parametrize("cam", [scenes.upward_camera(0, 0, 0, 8, 6, 60.0),
                                 scenes.Camera((0, 0, 0), (1, 0, 0, 0, 1, 0, 0, 0, 1),
                                               30.0, 22.0, 2.3, 7.9, 5, 9)])
def test_pixel_solid_angle_matches_quadrature(oracle, cam):
    total = 0.0
    for row in range(cam.height):
        for col in range(cam.width):
            om = oracle.pixel_solid_angle(cam, row, col)
            x1, x2 = (col - cam.cx) / cam.fx, (col + 1 - cam.cx) / cam.fx
            y1, y2 = (row - cam.cy) / cam.fy, (row + 1 - cam.cy) / cam.fy
            ref, _ = integrate.dblquad(lambda y, x: (1 + x * x + y * y) ** -1.5, x1, x2, y1, y2,
                                       epsabs=1e-13, epsrel=1e-11)
            assert abs(om - ref) < 1e-10 * max(ref, 1e-3)
            total += om
    # the whole sensor: a centred rectangle of half-extents a, b subtends
    # 4 atan(a b / sqrt(1 + a^2 + b^2)) (solid angle of a pyramid)
    if cam.cx == cam.width / 2 and cam.cy == cam.height / 2:
        a, b = cam.width / 2 / cam.fx, cam.height / 2 / cam.fy
        assert abs(total - 4 * math.atan(a * b / math.sqrt(1 + a * a + b * b))) < 1e-12
