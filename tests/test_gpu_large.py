"""The large workloads on the GPU: the 128^3 cloud with 25 cameras of 256^2
(forward + gradient) and the 256x256x128 multi-cloud field with 36 cameras
of 256^2 (forward, gradient, one projected descent step, and the oracle on a
32^3 crop).

Grids, cameras and launch configuration are the workloads' own; the photon
counts are cut so that each test takes seconds (measured at the full counts:
the 128^3 forward at 1e9 photons takes 52 s and its gradient 85 s).  What
is checked at these sizes: photon bookkeeping, finite and non-negative
images, the last photon-id block of a run against the oracle, and the
gradient of a photon range as the sum of its two halves' gradients."""
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


def _sigma(ref, m2, n):
    return np.sqrt(np.maximum(m2 - 2 * ref ** 2 / max(n, 1), 0.0))


def _tail_matches_oracle(M, oracle, s, beta, n_total, n=2000):
    tail, gm2, _ = M.mc_render_moments(s, beta, n_photons=n, photon_offset=n_total - n)
    ref, rst, m2 = oracle.render(s, with_m2=True, n_photons=n, photon_offset=n_total - n)
    tail = tail.cpu().numpy()
    tol = np.maximum(1e-4 * np.abs(ref), 3 * _sigma(ref, m2 + gm2.cpu().numpy(), n))
    bad = np.abs(tail - ref) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:10], tail[bad][:10], ref[bad][:10])
    assert rst["events"] > 0


def _bookkeeping(st, n):
    assert st["photons"] == n
    assert st["esc_top"] + st["esc_bottom"] + st["esc_side"] + st["rr_killed"] + st["capped"] == n


def _gradient_halves(M, s, beta, dl, n):
    """g over photon ids [0, n) against g([0, n/2)) + g([n/2, n)), all with
    the normalisation of n photons (FP64 sums of the same terms)."""
    import torch
    g, st = M.mc_grad_beta(s, beta, dl, n_photons=n)
    h = n // 2
    g1, _ = M.mc_grad_beta(s, beta, dl, n_photons=h, n_photons_norm=n)
    g2, _ = M.mc_grad_beta(s, beta, dl, n_photons=n - h, photon_offset=h, n_photons_norm=n)
    assert bool(torch.isfinite(g).all())
    assert float(g.abs().max()) > 0
    assert torch.allclose(g, g1 + g2, rtol=1e-9, atol=1e-12 * float(g.abs().max()))
    return g, st


def test_large_grid_128_forward_and_gradient(M, oracle):
    import torch
    n = 20_000_000
    s = scenes.config4(n_photons=n)
    print(f"case 128^3, 25 cameras 256^2, {n} photons", flush=True)
    beta = M.beta_tensor(s, "fp32")
    img, st = M.mc_render(s, beta)
    _bookkeeping(st, n)
    img_np = img.cpu().numpy()
    assert np.isfinite(img_np).all() and (img_np >= 0).all() and img_np.max() > 0
    _tail_matches_oracle(M, oracle, s, beta, n)
    dl = torch.as_tensor(np.random.default_rng(2).normal(size=img.numel()), device="cuda")
    _gradient_halves(M, s, beta, dl, 4_000_000)


def _crop(s, x0, y0, z0, m):
    """m^3 sub-grid of s starting at voxel (x0, y0, z0), cameras moved with it."""
    b = s.beta3d()[z0:z0 + m, y0:y0 + m, x0:x0 + m]
    o = np.array([x0 * s.dx, y0 * s.dy, z0 * s.dz])
    cams = [scenes.Camera(tuple(np.array(c.pos) - o), c.R, c.fx, c.fy, c.cx, c.cy, c.width, c.height)
            for c in s.cameras]
    return scenes.Scene(m, m, m, s.dx, s.dy, s.dz, np.ascontiguousarray(b).reshape(-1), cams, s.albedo, s.g,
                        s.sun_zenith, s.sun_azimuth, s.n_photons, s.seed, s.name + "-crop")


def test_multi_cloud_256_forward_gradient_and_step(M, oracle):
    import torch
    n = 50_000_000
    s = scenes.config5(n_photons=n)
    print(f"case 256x256x128, 36 cameras 256^2, {n} photons", flush=True)
    beta = M.beta_tensor(s, "fp32")
    img, st = M.mc_render(s, beta)
    _bookkeeping(st, n)
    img_np = img.cpu().numpy()
    assert np.isfinite(img_np).all() and (img_np >= 0).all() and img_np.max() > 0
    _tail_matches_oracle(M, oracle, s, beta, n)
    # one projected gradient step of the descent loop on an L2 image loss
    dl = 2.0 * (img - 1.1 * img)
    g, _ = _gradient_halves(M, s, beta, dl, 2_000_000)
    b64 = torch.as_tensor(s.beta, dtype=torch.float64, device="cuda")
    delta = 0.05 * float(b64.max()) / float(g.abs().max())
    M.mc_gd_step(b64, g, delta)
    ref = np.maximum(s.beta - delta * g.cpu().numpy(), 0.0)
    assert bool((b64 >= 0).all())
    np.testing.assert_allclose(b64.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * ref.max())


def test_multi_cloud_crop_fp64_matches_oracle(M, oracle):
    """The multi-cloud field's 32^3 crop about its densest column, the
    workload's 36 cameras: FP64 images per pixel and the gradient per voxel
    against the oracle on the same photons."""
    import torch
    s5 = scenes.config5(n_photons=1)
    col = (s5.beta3d() * s5.dz).sum(axis=0)
    iy, ix = np.unravel_index(np.argmax(col), col.shape)
    x0 = int(min(max(ix - 16, 0), s5.nx - 32))
    y0 = int(min(max(iy - 16, 0), s5.ny - 32))
    z0 = int(np.argmax(s5.beta3d()[:, iy, ix].reshape(-1)))
    z0 = int(min(max(z0 - 16, 0), s5.nz - 32))
    s = _crop(s5, x0, y0, z0, 32)
    s.n_photons = 3000
    print(f"case multi-cloud crop at ({x0},{y0},{z0})", flush=True)
    img, st = M.mc_render(s, M.beta_tensor(s, "fp64"), transport="fp64")
    ref, rst = oracle.render(s)
    for k in ("photons", "events", "le_jobs", "vox_free", "rr_killed", "capped"):
        assert st[k] == rst[k], (k, st[k], rst[k])
    img = img.cpu().numpy()
    assert np.abs(ref).max() > 0
    assert np.allclose(img, ref, rtol=1e-9, atol=1e-13 * np.abs(ref).max())
    dl = np.random.default_rng(5).normal(size=img.size)
    g, _ = M.mc_grad_beta(s, M.beta_tensor(s, "fp64"), torch.as_tensor(dl, device="cuda"), transport="fp64")
    gref, _ = oracle.grad_beta(s, dl)
    g = g.cpu().numpy()
    assert np.allclose(g, gref, rtol=1e-9, atol=1e-12 * np.abs(gref).max())


@pytest.mark.parametrize("transport", ["fp32", "fp64"])
def test_c4_kept_and_replayed_gradients_agree(M, transport):
    """On the 128^3 grid (128 tiles of 16x16x64) the gradient from a render's
    kept rays equals the replayed one up to summation order: both routes bin
    the same rays (C_e recorded, the pixel weight applied by the binning
    pass), also when a small tape forces many binning passes of a few
    wavefront slices each (split over many binning blocks), many replay
    chunks and small deposit items."""
    import torch
    s = scenes.config4(n_photons=200_000)
    print(f"case c4 kept vs replay {transport}", flush=True)
    beta = M.beta_tensor(s, transport)
    img, _, tape = M.mc_render_tape(s, beta, transport=transport)
    assert tape is not None
    dl = torch.as_tensor(np.random.default_rng(5).normal(size=img.numel()), device="cuda")
    g_rep, _ = M.mc_grad_beta(s, beta, dl, transport=transport)
    g_tape, _ = M.mc_grad_beta(s, beta, dl, transport=transport, tape=tape)
    g_tape_small, _ = M.mc_grad_beta(s, beta, dl, transport=transport, tape=tape, tape_limit=5_000_000)
    g_rep_small, _ = M.mc_grad_beta(s, beta, dl, transport=transport, tape_limit=5_000_000)
    tape.free()
    assert bool(torch.isfinite(g_rep).all())
    scale = float(g_rep.abs().max())
    assert scale > 0
    for g in (g_tape, g_tape_small, g_rep_small):
        assert torch.allclose(g, g_rep, rtol=1e-10, atol=1e-12 * scale)

