"""GPU parity of the voxelised forward model (Sec. 3) and its frozen-j
gradient (Sec. 5.2) against the oracle, through the C ABI.

Tolerances: the deterministic parts (transmittance, projection, gradient)
are FP64 on both sides and differ only in the order of FP64 sums: 1e-10
relative.  The scatter pass (Monte Carlo) with FP64 transport follows the
oracle's photons exactly: 1e-9 per value, equal counters; with FP32
transport a rounding can move a collision to a neighbouring voxel: 1e-3 in
relative L2 against the oracle and 1e-4 against the FP64 GPU pass."""
import numpy as np
import pytest

from paper_1512_02110_amd import scenes

from ._scene_helpers import look_camera

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_02110_amd import mcrt
    mcrt.load_library()
    return mcrt


def _random_scene(seed):
    rng = np.random.default_rng(seed)
    cams = [scenes.upward_camera(0.21, 0.13, -0.15, 9, 7, 70.0),
            look_camera((0.33, 0.07, 0.11), (-0.3, 1.0, 0.2), (0, 0, 1), 8, 9, 80.0),  # inside
            look_camera((-0.4, 0.2, 0.15), (1, 0, 0), (0, 0, 1), 6, 6, 40.0)]
    beta = rng.uniform(0.5, 12.0, size=7 * 5 * 4)
    beta[rng.random(beta.size) < 0.3] = 0.0
    return scenes.Scene(7, 5, 4, 0.06, 0.06, 0.06, beta, cams, 0.95, 0.6, 0.5, 0.7, 4000, seed)


@pytest.mark.parametrize("case", ["c1", "random"])
def test_voxel_scatter_fp64_matches_oracle(M, oracle, case):
    s = scenes.config1(n_photons=3000) if case == "c1" else _random_scene(3)
    print(f"case voxel scatter fp64 {case}", flush=True)
    j, st = M.mc_voxel_scatter(s, M.beta_tensor(s, "fp64"), transport="fp64")
    ref, rst = oracle.voxel_scatter(s)
    j = j.cpu().numpy().reshape(ref.shape)
    assert st == rst
    assert np.allclose(j, ref, rtol=1e-9, atol=1e-13 * np.abs(ref).max())


def test_voxel_scatter_fp32(M, oracle):
    s = scenes.config2(n_photons=3000)
    print("case voxel scatter fp32 c2", flush=True)
    j32, st32 = M.mc_voxel_scatter(s, M.beta_tensor(s, "fp32"))
    j64, _ = M.mc_voxel_scatter(s, M.beta_tensor(s, "fp64"), transport="fp64")
    ref, rst = oracle.voxel_scatter(s)
    j32 = j32.cpu().numpy().reshape(ref.shape)
    j64 = j64.cpu().numpy().reshape(ref.shape)
    assert np.allclose(j64, ref, rtol=1e-9, atol=1e-13 * np.abs(ref).max())
    assert np.linalg.norm(j32 - ref) <= 1e-3 * np.linalg.norm(ref)
    assert abs(st32["events"] - rst["events"]) <= max(2, 1e-3 * rst["events"])


@pytest.mark.parametrize("n_side", [1, 3])
def test_voxel_render_and_grad_match_oracle(M, oracle, n_side):
    import torch
    s = _random_scene(5)
    print(f"case voxel render/grad random n_side {n_side}", flush=True)
    rng = np.random.default_rng(6)
    j = rng.uniform(0.0, 1.0, size=(s.n_cams, s.n_vox)) * (s.beta > 0)
    dl = rng.normal(size=s.n_pix_total)
    beta = M.beta_tensor(s, "fp64")
    jt = torch.as_tensor(j, device="cuda")
    img = M.mc_voxel_render(s, beta, jt, n_side).cpu().numpy()
    g = M.mc_voxel_grad(s, beta, jt, torch.as_tensor(dl, device="cuda"), n_side).cpu().numpy()
    ref = oracle.voxel_render(s, j, n_side)
    gref = oracle.voxel_grad(s, j, dl, n_side)
    assert np.abs(ref).max() > 0 and np.abs(gref).max() > 0
    assert np.allclose(img, ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())
    assert np.allclose(g, gref, rtol=1e-10, atol=1e-13 * np.abs(gref).max())


def test_voxel_pipeline_config2(M, oracle):
    """The c2 workload end to end: j from the GPU scatter pass (1e6 photons),
    then images and gradient on the GPU against the oracle's for that j."""
    import torch
    s = scenes.config2(n_photons=1_000_000)
    print("case voxel pipeline c2", flush=True)
    j, st = M.mc_voxel_scatter(s, M.beta_tensor(s, "fp32"))
    assert st["photons"] == 1_000_000 and torch.isfinite(j).all() and (j >= 0).all()
    beta = M.beta_tensor(s, "fp64")
    img = M.mc_voxel_render(s, beta, j, 2)
    dl = torch.as_tensor(np.random.default_rng(1).normal(size=s.n_pix_total), device="cuda")
    g = M.mc_voxel_grad(s, beta, j, dl, 2)
    jn = j.cpu().numpy().reshape(s.n_cams, s.n_vox)
    ref = oracle.voxel_render(s, jn, 2)
    gref = oracle.voxel_grad(s, jn, dl.cpu().numpy(), 2)
    img, g = img.cpu().numpy(), g.cpu().numpy()
    assert np.allclose(img, ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())
    assert np.allclose(g, gref, rtol=1e-10, atol=1e-13 * np.abs(gref).max())


def test_voxel_edge_cases(M):
    import torch
    s = scenes.config1(n_photons=0)
    print("case voxel edge cases", flush=True)
    j, st = M.mc_voxel_scatter(s, M.beta_tensor(s, "fp32"))
    assert st["events"] == 0 and float(j.abs().max()) == 0.0
    beta = M.beta_tensor(s, "fp64")
    img = M.mc_voxel_render(s, beta, j, 1)
    assert float(img.abs().max()) == 0.0
    for n_side in (0, 65):
        with pytest.raises(M.McError) as e:
            M.mc_voxel_render(s, beta, j, n_side)
        assert e.value.code == M.MC_ERR_INVALID_ARG
    with pytest.raises(M.McError):
        M.mc_voxel_scatter(s.replace(n_photons=10), M.beta_tensor(s, "fp32"), tally="kahan32")
    g = M.mc_voxel_grad(s, beta, j, torch.zeros(s.n_pix_total, dtype=torch.float64, device="cuda"), 2)
    assert float(g.abs().max()) == 0.0
