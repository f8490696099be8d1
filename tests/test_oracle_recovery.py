"""Pins of the oracle's recovery pieces (Secs. 5.2, 6, 7): the conditioning
Q_c from ray counts, the camera weighting of the frozen-j gradient, the
Laplacian regulariser, the camera noise model, the error measures and the
surrogate gradient-descent loop."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1512_02110_amd import scenes

from ._scene_helpers import look_camera
from .test_oracle_voxel import _box_chord, _scene


def test_ray_counts_match_independent_chords():
    """Q_c(k, k) counts the sub-pixel rays with a length above 1e-9 of the
    voxel edge in voxel k: slab intersection per voxel box, no voxel walk."""
    cam = look_camera((-0.25, 0.11, 0.07), (1, 0.15, 0.1), (0, 0, 1), 5, 4, 50.0)
    s = _scene(3, 2, 2, 0.1, 1.0, [cam])
    n = 2
    counts, q = O.voxel_conditioning(s, n)
    R = np.array(cam.R).reshape(3, 3)
    ref = np.zeros(s.n_vox)
    for row in range(cam.height):
        for col in range(cam.width):
            for b in range(n):
                for a in range(n):
                    v = R.T @ np.array([(col + (a + 0.5) / n - cam.cx) / cam.fx,
                                        (row + (b + 0.5) / n - cam.cy) / cam.fy, 1.0])
                    v /= np.linalg.norm(v)
                    for k in range(s.n_vox):
                        lo = np.array([k % 3, (k // 3) % 2, k // 6]) * 0.1
                        ref[k] += _box_chord(np.array(cam.pos), v, lo, lo + 0.1) > 1e-10
    assert ref.max() > 0
    assert np.array_equal(counts[0], ref)
    assert np.array_equal(q[0], np.where(ref > 0, 1.0 / np.maximum(ref, 1), 0.0))


def test_weighted_gradient_is_per_camera_sum():
    """Eq. (divCost1) with Q_c: the weighted gradient is the sum over cameras
    of q_c times that camera's own (finite-difference pinned) gradient."""
    rng = np.random.default_rng(3)
    cams = [scenes.upward_camera(0.22, 0.17, -0.2, 6, 5, 70.0),
            look_camera((0.31, 0.05, 0.12), (-0.2, 1, 0.3), (0, 0, 1), 5, 6, 80.0)]
    beta = rng.uniform(0.5, 6.0, size=4 * 3 * 3)
    s = _scene(4, 3, 3, 0.1, beta, cams)
    j = rng.uniform(0.0, 1.0, size=(2, s.n_vox))
    dl = rng.normal(size=s.n_pix_total)
    q = rng.uniform(0.1, 2.0, size=(2, s.n_vox))
    g = O.voxel_grad(s, j, dl, 2, q=q)
    ref = np.zeros(s.n_vox)
    off = 0
    for c, cam in enumerate(cams):
        sc = _scene(4, 3, 3, 0.1, beta, [cam])
        ref += q[c] * O.voxel_grad(sc, j[c:c + 1], dl[off:off + cam.n_pix], 2)
        off += cam.n_pix
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_laplacian_closed_forms_and_gradient():
    s = _scene(6, 4, 3, 0.1, 1.0, [scenes.upward_camera(0.1, 0.1, -0.1, 2, 2, 60.0)])
    # a constant field has no curvature, also at the boundary
    psi, g = O.laplacian_reg(s, beta=np.full(s.n_vox, 3.75))
    assert psi == 0.0 and not g.any()
    # beta = ix^2: interior 2, ix = 0 gives 1, ix = nx-1 gives -(2 nx - 3)
    ix = np.tile(np.arange(6), 4 * 3).astype(float)
    psi, _ = O.laplacian_reg(s, beta=ix ** 2)
    assert psi == pytest.approx(4 * 3 * ((6 - 2) * 4 + 1 + (2 * 6 - 3) ** 2), rel=1e-14)
    w = np.array([0.5, 1.0, 2.0])
    psi_w, _ = O.laplacian_reg(s, beta=ix ** 2, w_layer=w)
    assert psi_w == pytest.approx(4 * ((6 - 2) * 4 + 1 + 81) * float(np.sum(w ** 2)), rel=1e-14)
    # gradient: central differences of Psi
    b = np.random.default_rng(2).uniform(0, 5, s.n_vox)
    _, g = O.laplacian_reg(s, beta=b, w_layer=w)
    for k in (0, 5, 17, 40, 71):
        e = np.zeros(s.n_vox)
        e[k] = 1e-4
        fd = (O.laplacian_reg(s, beta=b + e, w_layer=w)[0] - O.laplacian_reg(s, beta=b - e, w_layer=w)[0]) / 2e-4
        assert g[k] == pytest.approx(fd, rel=1e-8)


def test_camera_noise_by_hand():
    """Eq. (noise): scale to 2^10 over the largest masked pixel, 0.4 grey
    levels of read noise, rounding and clipping to [0, 1024]."""
    img = np.array([0.0, 1.0, 2.0, 4.0, 1e-4])
    mask = np.array([1.0, 1.0, 1.0, 0.0, 1.0])
    normals = np.array([0.0, 0.5, 1.0, 0.0, -2.0])
    out, scale = O.camera_noise(img, normals, mask)
    assert scale == 512.0
    # 0 -> 0; 512.2 -> 512; 1024.4 -> 1024; 2048 -> clipped; 0.0512 - 0.8 -> -1 -> 0
    assert list(out) == [0.0, 512.0, 1024.0, 1024.0, 0.0]


def test_recovery_error_by_hand():
    d, e = O.recovery_error([1.0, 3.0, 0.0], [2.0, 2.0, 1.0])
    assert d == pytest.approx((4 - 5) / 5) and e == pytest.approx((1 + 1 + 1) / 5)


def _recovery_scene():
    cams = scenes.camera_lattice(2, 0.4, 0.4, 8, 8, 70.0)
    truth = scenes.gaussian_blob(8, 8, 6, 0.05, 0.05, 0.05, 8.0, 0.08, (0.2, 0.2, 0.15))
    return scenes.Scene(8, 8, 6, 0.05, 0.05, 0.05, np.asarray(truth).reshape(-1), cams, 0.95, 0.7,
                        math.radians(30.0), 0.0, 4000, 0)


@pytest.mark.parametrize("conditioned", [1, 2, 0])
def test_recover_first_step_is_the_composition(conditioned):
    """One outer iteration, one step: j from the scatter pass, E and the step
    from the pinned render, weighted gradient, regulariser and clipping; the
    weights are 1/count (conditioned 1), the ray counts (2) or none (0)."""
    s = _recovery_scene()
    b0 = 0.7 * s.beta
    meas = O.voxel_render(s, O.voxel_scatter(s)[0], 2) * 1.05
    mask = (np.arange(s.n_pix_total) % 7 != 0).astype(float)
    w = np.linspace(0.5, 1.5, s.nz)
    eta, delta = 0.01, 1e-3
    beta, cost = O.recover(s, b0, meas, 2, delta, 1, 1, eta=eta, w_layer=w, mask=mask, seed=11,
                           conditioned=conditioned)
    j, _ = O.voxel_scatter(s, beta=b0, seed=11)
    img = O.voxel_render(s, j, 2, beta=b0)
    r = mask * (img - meas)
    counts, q = O.voxel_conditioning(s, 2)
    weights = {1: q, 2: counts.astype(np.float64), 0: None}[conditioned]
    g = O.voxel_grad(s, j, 2 * mask * r, 2, beta=b0, q=weights)
    psi, gpsi = O.laplacian_reg(s, beta=b0, w_layer=w)
    assert cost[0] == pytest.approx(float(np.sum(r * r)) + eta * psi, rel=1e-12)
    ref = np.maximum(b0 - delta * (g + eta * gpsi), 0.0)
    assert np.allclose(beta, ref, rtol=1e-12, atol=1e-15)


def test_recover_descends_on_the_surrogate():
    """With j frozen the cost is a smooth function of beta: small conditioned
    steps decrease it at every step, and beta stays non-negative."""
    s = _recovery_scene()
    meas = O.voxel_render(s, O.voxel_scatter(s)[0], 2)
    b0 = 0.6 * s.beta
    j, _ = O.voxel_scatter(s, beta=b0, seed=5)
    _, q = O.voxel_conditioning(s, 2)
    img = O.voxel_render(s, j, 2, beta=b0)
    g = O.voxel_grad(s, j, 2 * (img - meas), 2, beta=b0, q=q)
    delta = 0.05 * b0.max() / np.abs(g).max()
    beta, cost = O.recover(s, b0, meas, 2, delta, 8, 1, seed=5)
    assert np.all(np.diff(cost) < 0), cost
    assert beta.min() >= 0.0
