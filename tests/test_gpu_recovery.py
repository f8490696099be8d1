"""GPU parity of the recovery pieces (Secs. 5.2, 6, 7) and of the whole
surrogate gradient-descent loop against the oracle, through the C ABI.
Deterministic FP64 parts agree to the order of FP64 sums (1e-10); the loop
with FP64 transport follows the oracle's photons (1e-8 after several
steps); with FP32 transport, to 1e-3 in relative L2."""
import numpy as np
import pytest

from paper_1512_02110_amd import scenes

from ._scene_helpers import look_camera
from .test_oracle_recovery import _recovery_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_02110_amd import mcrt
    mcrt.load_library()
    return mcrt


def _cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def test_conditioning_and_weighted_gradient(M, oracle):
    s = _recovery_scene()
    s.cameras.append(look_camera((0.21, 0.37, 0.12), (0.1, -1, 0.2), (0, 0, 1), 7, 5, 80.0))  # inside
    print("case recovery conditioning", flush=True)
    counts, q = M.mc_voxel_conditioning(s, 3)
    rc, rq = oracle.voxel_conditioning(s, 3)
    assert np.array_equal(counts.cpu().numpy(), rc.reshape(-1))
    assert np.allclose(q.cpu().numpy(), rq.reshape(-1), rtol=1e-15, atol=0)
    rng = np.random.default_rng(2)
    j = rng.uniform(0, 1, size=(s.n_cams, s.n_vox))
    dl = rng.normal(size=s.n_pix_total)
    w = rng.uniform(0.2, 2.0, size=(s.n_cams, s.n_vox))
    g = M.mc_voxel_grad(s, _cuda(s.beta), _cuda(j), _cuda(dl), 3, cam_weights=_cuda(w)).cpu().numpy()
    ref = oracle.voxel_grad(s, j, dl, 3, q=w)
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())


def test_regularizer_residual_step_noise_error(M, oracle):
    s = _recovery_scene()
    print("case recovery pieces", flush=True)
    rng = np.random.default_rng(4)
    b = rng.uniform(0, 5, s.n_vox)
    wl = rng.uniform(0.5, 1.5, s.nz)
    val, g = M.mc_regularizer(s, _cuda(b), _cuda(wl), eta=0.3)
    psi, gref = oracle.laplacian_reg(s, beta=b, w_layer=wl)
    assert float(val.item()) == pytest.approx(psi, rel=1e-12)
    assert np.allclose(g.cpu().numpy(), 0.3 * gref, rtol=1e-12, atol=1e-14 * np.abs(gref).max())
    img, meas = rng.uniform(0, 2, 300), rng.uniform(0, 2, 300)
    mask = (rng.random(300) > 0.2).astype(float)
    dl, loss = M.mc_image_residual(_cuda(img), _cuda(meas), _cuda(mask))
    r = mask * (img - meas)
    assert np.allclose(dl.cpu().numpy(), 2 * mask * r, rtol=1e-15, atol=0)
    assert float(loss.item()) == pytest.approx(float(np.sum(r * r)), rel=1e-12)
    beta = _cuda(b)
    gg = rng.normal(size=s.n_vox)
    M.mc_gd_step(beta, _cuda(gg), 0.7)
    # (the kernel may fuse the multiply-add: one rounding fewer)
    assert np.allclose(beta.cpu().numpy(), np.maximum(b - 0.7 * gg, 0.0), rtol=1e-15, atol=1e-15 * b.max())
    normals = rng.normal(size=300)
    out, scale = M.mc_camera_noise(_cuda(img), _cuda(normals), _cuda(mask))
    rout, rscale = oracle.camera_noise(img, normals, mask)
    assert float(scale.item()) == rscale and np.array_equal(out.cpu().numpy(), rout)
    assert M.mc_recovery_error(_cuda(b), _cuda(s.beta)) == pytest.approx(oracle.recovery_error(b, s.beta),
                                                                         rel=1e-12)


@pytest.mark.parametrize("transport", ["fp64", "fp32"])
def test_recover_loop_matches_oracle(M, oracle, transport):
    """Two surrogate iterations of three conditioned, regularised, masked
    steps from 0.7 x truth, against images of the truth."""
    s = _recovery_scene()
    print(f"case recover loop {transport}", flush=True)
    meas = oracle.voxel_render(s, oracle.voxel_scatter(s, seed=99)[0], 2)
    mask = (np.arange(s.n_pix_total) % 5 != 0).astype(float)
    wl = np.linspace(0.5, 1.5, s.nz)
    b0 = 0.7 * s.beta
    kw = dict(eta=0.01, w_layer=wl, mask=mask, seed=21)
    ref, rcost = oracle.recover(s, b0, meas, 2, 1.0, 3, 2, **kw)
    b, cost = M.mc_recover(s, _cuda(b0), _cuda(meas), 1.0, 3, 2, transport=transport,
                           eta=0.01, w_layer=_cuda(wl), mask=_cuda(mask), seed=21)
    b = b.cpu().numpy()
    assert np.abs(ref - b0).max() > 1e-3 * b0.max()  # the loop moved beta
    if transport == "fp64":
        assert np.allclose(b, ref, rtol=1e-8, atol=1e-12 * ref.max())
        assert np.allclose(cost, rcost, rtol=1e-9)
    else:
        assert np.linalg.norm(b - ref) <= 1e-3 * np.linalg.norm(ref)
        assert np.allclose(cost, rcost, rtol=1e-3)
    assert b.min() >= 0.0


@pytest.mark.parametrize("conditioned,delta", [(0, 0.2), (2, 1e-3)])
def test_recover_loop_other_conditionings(M, oracle, conditioned, delta):
    """The loop without conditioning, and with Q_c = the ray counts (the
    passage's wording taken literally), against the oracle (FP64)."""
    s = _recovery_scene()
    print(f"case recover loop, conditioning {conditioned}", flush=True)
    meas = oracle.voxel_render(s, oracle.voxel_scatter(s, seed=99)[0], 2)
    b0 = 0.7 * s.beta
    ref, rcost = oracle.recover(s, b0, meas, 2, delta, 3, 2, eta=0.01, seed=21, conditioned=conditioned)
    b, cost = M.mc_recover(s, _cuda(b0), _cuda(meas), delta, 3, 2, transport="fp64", eta=0.01, seed=21,
                           conditioned=conditioned)
    b = b.cpu().numpy()
    assert np.abs(ref - b0).max() > 1e-4 * b0.max()
    assert np.allclose(b, ref, rtol=1e-8, atol=1e-12 * ref.max())
    assert np.allclose(cost, rcost, rtol=1e-9)


def test_recover_edge_cases(M):
    import torch
    s = _recovery_scene()
    print("case recover edge cases", flush=True)
    b0 = _cuda(0.5 * s.beta)
    meas = torch.zeros(s.n_pix_total, dtype=torch.float64, device="cuda")
    b, cost = M.mc_recover(s, b0, meas, 1e-3, 2, 0)
    assert torch.equal(b, b0) and cost.size == 0
    with pytest.raises(M.McError):
        M.mc_recover(s, b0, meas, 1e-3, 0, 1)
    with pytest.raises(M.McError):
        M.mc_recover(s, b0, meas, 1e-3, 1, 1, rays_per_side=0)
    with pytest.raises(M.McError):
        M.mc_recover(s, b0, meas, 1e-3, 1, 1, conditioned=3)
