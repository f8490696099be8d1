"""The surrogate gradient on a grid too large for an LDS copy of the gradient
(rays binned by tile and deposited tile by tile in LDS) with cameras in every
orientation: tilted, looking sideways, looking down, inside and outside the
domain, and cameras with very wide pixels.  FP64 transport must give the
oracle's gradient per voxel, on the photon replay and on the kept rays of the
render; FP32 transport within the gradient tolerance in L2."""
import numpy as np
import pytest

from paper_1512_02110_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_02110_amd import mcrt
    mcrt.load_library()
    return mcrt


def look_camera(pos, target, width, height, fov_deg, roll=0.0):
    """Pinhole camera at pos looking at target (rows of R: right, down, forward)."""
    f = np.asarray(target, float) - np.asarray(pos, float)
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    c, s = np.cos(roll), np.sin(roll)
    x, y = c * x + s * y, -s * x + c * y
    R = np.stack([x, y, f])
    fx = (width / 2) / np.tan(np.radians(fov_deg) / 2)
    return scenes.Camera(tuple(map(float, pos)), tuple(map(float, R.reshape(-1))), float(fx), float(fx),
                         width / 2, height / 2, width, height)


def mixed_scene(rng, n_photons):
    nx, ny, nz = 26, 22, 16
    dx, dy, dz = 0.05, 0.06, 0.045
    L = np.array([nx * dx, ny * dy, nz * dz])
    b = rng.uniform(0.0, 9.0, size=nx * ny * nz)
    b[rng.random(b.size) < 0.35] = 0.0
    centre = 0.5 * L
    cams = [
        look_camera((0.3 * L[0], 0.4 * L[1], 0.0), centre + [0.1, -0.1, 0.3], 23, 17, 80.0, roll=0.4),  # floor, tilted
        look_camera((-0.4, 0.5 * L[1], 0.5 * L[2]), centre, 19, 21, 60.0),                            # outside, sideways (+x)
        look_camera((0.6 * L[0], 0.3 * L[1], 0.5 * L[2]), centre + [0.0, 0.5, 0.0], 16, 16, 90.0),      # inside, along +y
        look_camera((0.5 * L[0], 0.5 * L[1], L[2] + 0.3), centre - [0.1, 0.0, 0.2], 20, 18, 70.0, 1.1), # above, looking down
        look_camera((L[0] + 0.2, -0.3, 0.2), centre, 17, 13, 50.0),                                    # outside, oblique
    ]
    return scenes.Scene(nx, ny, nz, dx, dy, dz, b, cams, 0.95, float(rng.uniform(0.3, 0.85)),
                        float(rng.uniform(0.1, 1.2)), float(rng.uniform(0, 2 * np.pi)), n_photons,
                        int(rng.integers(0, 2 ** 40)), "orientations")


@pytest.mark.parametrize("seed", [3, 4])
def test_gradient_any_orientation_matches_oracle(M, oracle, seed):
    import torch
    s = mixed_scene(np.random.default_rng(seed), n_photons=2500)
    print(f"case gradient, cameras in every orientation, scene seed {seed}", flush=True)
    dl = np.random.default_rng(seed + 10).normal(size=s.n_pix_total)
    ref, rst = oracle.grad_beta(s, dl)
    b64 = M.beta_tensor(s, "fp64")
    dlt = torch.as_tensor(dl, device="cuda")
    g, st = M.mc_grad_beta(s, b64, dlt, transport="fp64")
    g = g.cpu().numpy()
    assert st["le_jobs"] == rst["le_jobs"] > 0
    assert np.allclose(g, ref, rtol=1e-8, atol=1e-11 * np.abs(ref).max())
    # the kept rays of the render
    _, _, tape = M.mc_render_tape(s, b64, transport="fp64")
    assert tape is not None
    gt, _ = M.mc_grad_beta(s, b64, dlt, transport="fp64", tape=tape)
    tape.free()
    assert np.allclose(gt.cpu().numpy(), ref, rtol=1e-8, atol=1e-11 * np.abs(ref).max())
    # FP32 transport within the gradient tolerance in L2
    g32, _ = M.mc_grad_beta(s, M.beta_tensor(s, "fp32"), dlt)
    assert np.linalg.norm(g32.cpu().numpy() - ref) <= 1e-3 * np.linalg.norm(ref)


def test_gradient_wide_pixels_matches_oracle(M, oracle):
    """Two cameras of 2 x 3 pixels with 150-degree fields of view on a 40^3
    grid (a ray's pixel says little about where it runs): the gradient is the
    oracle's."""
    import torch
    rng = np.random.default_rng(21)
    n = 40
    b = rng.uniform(0.0, 6.0, size=n ** 3)
    b[rng.random(b.size) < 0.5] = 0.0
    cams = [look_camera((0.5, 0.5, 0.0), (0.5, 0.5, 1.0), 2, 3, 150.0),
            look_camera((1.0, 0.2, 0.4), (0.4, 0.6, 0.5), 3, 2, 150.0)]
    s = scenes.Scene(n, n, n, 0.025, 0.025, 0.025, b, cams, 0.9, 0.7, 0.5, 0.3, 2000, 5, "wide")
    print("case gradient, wide pixels", flush=True)
    dl = rng.normal(size=s.n_pix_total)
    ref, _ = oracle.grad_beta(s, dl)
    g, _ = M.mc_grad_beta(s, M.beta_tensor(s, "fp64"), torch.as_tensor(dl, device="cuda"), transport="fp64")
    assert np.allclose(g.cpu().numpy(), ref, rtol=1e-8, atol=1e-11 * np.abs(ref).max())
