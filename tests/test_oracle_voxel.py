"""Pins of the oracle's voxelised forward model (Sec. 3 and the frozen-j
Jacobian of Sec. 5.2, Eqs. Jaco1, TcofJaco1, DivTc) against closed forms,
quadrature and finite differences."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1512_02110_amd import scenes

from ._scene_helpers import hg, look_camera

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _box_chord(p0, v, lo, hi):
    """Length of the ray p0 + t v (t >= 0) inside the box [lo, hi] (slabs)."""
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if v[a] == 0.0:
            if not (lo[a] <= p0[a] <= hi[a]):
                return 0.0
            continue
        ta, tb = (lo[a] - p0[a]) / v[a], (hi[a] - p0[a]) / v[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(0.0, t1 - t0)


def _gl3(lo, hi, n, f):
    """Gauss-Legendre quadrature of f(X) (X: (M,3)) over the box [lo, hi]."""
    x, w = np.polynomial.legendre.leggauss(n)
    pts, wts = [], []
    for a in range(3):
        h = 0.5 * (hi[a] - lo[a])
        pts.append(lo[a] + h * (x + 1.0))
        wts.append(h * w)
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    W = np.einsum("i,j,k->ijk", *wts)
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return float(np.sum(W.ravel() * f(P)))


def _scene(nx, ny, nz, d, beta, cams, **kw):
    b = np.full(nx * ny * nz, float(beta)) if np.isscalar(beta) else np.asarray(beta, float)
    base = dict(albedo=1.0, g=0.0, sun_zenith=0.0, sun_azimuth=0.0, n_photons=1000, seed=0)
    base.update(kw)
    return scenes.Scene(nx, ny, nz, d, d, d, b, list(cams), **base)


def test_transmittance_homogeneous_closed_form():
    """Eq. (Tck) in a homogeneous medium: exp(-beta * length of the LOS inside
    the domain), the length from slab intersection."""
    cams = [scenes.upward_camera(0.13, 0.21, -0.3, 4, 4, 60.0),
            look_camera((0.5, -0.2, 0.4), (0, 1, 0), (0, 0, 1), 4, 4, 60.0),
            look_camera((0.2, 0.3, 0.25), (1, 0, 0), (0, 0, 1), 4, 4, 60.0)]  # inside
    s = _scene(5, 4, 3, 0.1, 2.5, cams)
    T = O.voxel_transmittance(s)
    L = np.array([0.5, 0.4, 0.3])
    for c, cam in enumerate(cams):
        for k in range(s.n_vox):
            ix, iy, iz = k % 5, (k // 5) % 4, k // 20
            X = (np.array([ix, iy, iz]) + 0.5) * 0.1
            D = np.array(cam.pos) - X
            r = np.linalg.norm(D)
            length = min(r, _box_chord(X, D / r, np.zeros(3), L))
            assert T[c, k] == pytest.approx(math.exp(-2.5 * length), rel=1e-12)


def test_projection_matches_independent_chords():
    """Eq. (Icpixel) on a 3x2x2 grid: chord lengths of every sub-pixel ray
    through every voxel box computed independently (slab intersection per
    box, no voxel walk), with the closed-form T of a homogeneous medium."""
    cam = look_camera((-0.25, 0.11, 0.07), (1, 0.15, 0.1), (0, 0, 1), 5, 4, 50.0)
    b0 = 1.7
    s = _scene(3, 2, 2, 0.1, b0, [cam])
    rng = np.random.default_rng(4)
    j = rng.uniform(0.1, 1.0, size=(1, s.n_vox))
    n = 3
    img = O.voxel_render(s, j, n)
    T = O.voxel_transmittance(s)
    assert np.allclose(T, np.exp(-b0 * np.array([[_box_chord(
        (np.array([k % 3, (k // 3) % 2, k // 6]) + 0.5) * 0.1,
        (np.array(cam.pos) - (np.array([k % 3, (k // 3) % 2, k // 6]) + 0.5) * 0.1)
        / np.linalg.norm(np.array(cam.pos) - (np.array([k % 3, (k // 3) % 2, k // 6]) + 0.5) * 0.1),
        np.zeros(3), np.array([0.3, 0.2, 0.2])) for k in range(s.n_vox)]])), rtol=1e-12)
    R = np.array(cam.R).reshape(3, 3)
    V = 0.1 ** 3
    ref = np.zeros(cam.width * cam.height)
    for row in range(cam.height):
        for col in range(cam.width):
            acc = 0.0
            for bb in range(n):
                for a in range(n):
                    q = np.array([(col + (a + 0.5) / n - cam.cx) / cam.fx,
                                  (row + (bb + 0.5) / n - cam.cy) / cam.fy, 1.0])
                    v = R.T @ q
                    v /= np.linalg.norm(v)
                    for k in range(s.n_vox):
                        lo = np.array([k % 3, (k // 3) % 2, k // 6]) * 0.1
                        acc += _box_chord(np.array(cam.pos), v, lo, lo + 0.1) * j[0, k] * b0 * T[0, k]
            ref[row * cam.width + col] = acc / (n * n * V)
    assert ref.max() > 0
    assert np.allclose(img, ref, rtol=1e-12, atol=1e-14 * ref.max())


def test_projection_solid_angle_identity():
    """Pi_c spreads a voxel over the pixels that see it: for a voxel well
    inside the field of view, sum_p Omega_p Pi_c(p, k) V = int_voxel dV / r^2
    (the solid-angle integral of the chord length), here within the
    sampling error of 8 x 8 rays per pixel."""
    cam = scenes.upward_camera(0.25, 0.25, -0.6, 48, 48, 40.0)
    s = _scene(5, 5, 4, 0.1, 1e-12, [cam])
    k = 2 + 5 * (2 + 5 * 1)  # voxel (2, 2, 1), above the camera
    beta = s.beta.copy()
    j = np.zeros((1, s.n_vox))
    j[0, k] = 1.0 / beta[k]
    img = O.voxel_render(s, j, 8)
    omega = np.array([O.pixel_solid_angle(cam, r, c) for r in range(48) for c in range(48)])
    lhs = float(np.sum(omega * img)) * 0.1 ** 3
    lo = np.array([0.2, 0.2, 0.1])
    rhs = _gl3(lo, lo + 0.1, 24, lambda P: 1.0 / np.sum((P - np.array(cam.pos)) ** 2, axis=1))
    assert lhs == pytest.approx(rhs, rel=2e-3)


@pytest.mark.parametrize("n", [1, 2])
def test_voxel_gradient_matches_finite_differences(n):
    """Eqs. (Jaco1, TcofJaco1, DivTc): the frozen-j gradient of
    L = sum_p dl(p) i(p) equals central differences of the rendered images,
    on a heterogeneous field with empty voxels and a camera inside."""
    rng = np.random.default_rng(7)
    cams = [scenes.upward_camera(0.22, 0.17, -0.2, 6, 5, 70.0),
            look_camera((0.31, 0.05, 0.12), (-0.2, 1, 0.3), (0, 0, 1), 5, 6, 80.0)]
    beta = rng.uniform(0.5, 6.0, size=4 * 3 * 3)
    beta[rng.random(beta.size) < 0.2] = 0.0
    s = _scene(4, 3, 3, 0.1, beta, cams)
    j = rng.uniform(0.0, 1.0, size=(2, s.n_vox)) * (beta > 0)
    dl = rng.normal(size=s.n_pix_total)
    g = O.voxel_grad(s, j, dl, n)
    for m in rng.choice(s.n_vox, size=14, replace=False):
        h = 1e-6 * max(beta[m], 1.0)
        bp, bm = beta.copy(), beta.copy()
        bp[m] += h
        bm[m] -= h
        fd = (np.dot(dl, O.voxel_render(s, j, n, beta=bp)) - np.dot(dl, O.voxel_render(s, j, n, beta=bm))) / (2 * h)
        assert g[m] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(g).max())


def test_scatter_first_collision_layers_isotropic():
    """Eq. (Lcupdate, Jc) on a homogeneous slab lit from the zenith, isotropic
    scattering, first collisions only: layer z holds on average
    A / (4 pi beta) (exp(-beta (H - z_top)) - exp(-beta (H - z_bot))) of j
    (Beer-Lambert first-collision probability), within 4 sigma."""
    cam = scenes.upward_camera(0.2, 0.2, -0.5, 4, 4, 60.0)
    b0, N = 3.0, 60000
    s = _scene(4, 4, 5, 0.1, b0, [cam], n_photons=N, albedo=1.0, g=0.0)
    j, st = O.voxel_scatter(s, max_events=1)
    H, A = 0.5, 0.16
    base = A / N
    per_photon = base / (4 * math.pi * b0)
    for iz in range(5):
        layer = j[0].reshape(5, 4, 4)[iz].sum()
        p = math.exp(-b0 * (H - (iz + 1) * 0.1)) - math.exp(-b0 * (H - iz * 0.1))
        mean = N * p * per_photon
        sigma = per_photon * math.sqrt(N * p * (1 - p))
        assert abs(layer - mean) <= 4 * sigma, (iz, layer, mean, sigma)
    assert st["events"] <= N


def test_scatter_first_collision_phase_quadrature():
    """With g = 0.7 the tally weighs each first collision by the phase
    function towards the camera: per camera and per block of voxels the
    expectation is (N/A) int beta exp(-beta (H - z)) P(cos) dV by
    quadrature, within 4 sigma (variance from the second moment)."""
    cams = [scenes.upward_camera(0.1, 0.3, -0.4, 4, 4, 60.0),
            look_camera((0.55, 0.2, 0.25), (-1, 0, 0), (0, 0, 1), 4, 4, 60.0)]
    b0, N, g = 2.0, 80000, 0.7
    s = _scene(4, 4, 3, 0.1, b0, cams, n_photons=N, albedo=0.9, g=g)
    j, _ = O.voxel_scatter(s, max_events=1)
    H, A = 0.3, 0.16
    base = A / N
    for c, cam in enumerate(cams):
        Xc = np.array(cam.pos)

        def phase(P, Xc=Xc):
            V = Xc - P
            cos = -V[:, 2] / np.linalg.norm(V, axis=1)  # incoming direction -z
            return 0.9 * (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * cos) ** 1.5)

        for blk in [(slice(0, 2), slice(0, 2), slice(0, 3)), (slice(2, 4), slice(1, 4), slice(0, 3))]:
            jx, jy, jz = blk
            lo = np.array([jx.start, jy.start, jz.start]) * 0.1
            hi = np.array([jx.stop, jy.stop, jz.stop]) * 0.1
            dens = lambda P: b0 * np.exp(-b0 * (H - P[:, 2]))  # noqa: E731
            m1 = _gl3(lo, hi, 16, lambda P: dens(P) * phase(P)) / A
            m2 = _gl3(lo, hi, 16, lambda P: dens(P) * phase(P) ** 2) / A
            got = j[c].reshape(3, 4, 4)[jz, jy, jx].sum() * b0 / base  # back to raw L
            mean, sigma = N * m1, math.sqrt(N * (m2 - m1 * m1))
            assert abs(got - mean) <= 4 * sigma, (c, got, mean, sigma)
            assert hg(g, 1.0) > 0


def test_scatter_is_the_event_list_weighed():
    """j is the plain sum over the traced collisions of albedo w P(angle to
    the camera) / beta, times mu0 A_top / N."""
    s = scenes.config1(n_photons=300)
    j, st = O.voxel_scatter(s)
    ev, paths, _ = O.trace_paths(s, 0, 300, 4000, with_pix=False)
    assert int(paths["n_events"].sum()) == st["events"]
    ref = np.zeros_like(j)
    base = math.cos(s.sun_zenith) * (s.nx * s.dx) * (s.ny * s.dy) / 300
    w_sun = -np.array([math.sin(s.sun_zenith) * math.cos(s.sun_azimuth),
                       math.sin(s.sun_zenith) * math.sin(s.sun_azimuth), math.cos(s.sun_zenith)])
    for n in range(300):
        w = w_sun.copy()
        for e in ev[n][:paths["n_events"][n]]:
            X = np.array([e["x"], e["y"], e["z"]])
            for c, cam in enumerate(s.cameras):
                V = np.array(cam.pos) - X
                r = np.linalg.norm(V)
                ref[c, e["voxel"]] += s.albedo * e["w"] * hg(s.g, float(np.dot(w, V) / r))
            break  # only the first collision has a known incoming direction here
    # compare the first-collision part: rerun with one event per photon
    j1, _ = O.voxel_scatter(s, max_events=1)
    ref *= base / np.where(s.beta > 0, s.beta, np.inf)[None, :]
    assert np.allclose(j1, ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())
