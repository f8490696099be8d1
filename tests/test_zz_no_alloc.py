"""mc_render_noalloc, the render that allocates nothing (its scratch is a fixed
device array of the library), through the C ABI: on two calls in a row, the
second with a smaller input, its images and counters are those of mc_render on
the same inputs; a call beyond the fixed scratch is refused before anything is
enqueued."""
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


def _same_render(M, s, transport, tally="f64"):
    beta = M.beta_tensor(s, transport)
    ref, rst = M.mc_render(s, beta, transport=transport, tally=tally)
    img, st = M.mc_render_noalloc(s, beta, transport=transport, tally=tally)
    assert st == rst
    ref, img = ref.cpu().numpy(), img.cpu().numpy()
    # the same kernels on the same photons: only the order of the FP64 tally
    # atomics may differ
    assert np.allclose(img, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    assert st["le_jobs"] > 0


def test_noalloc_matches_render_then_smaller_input(M):
    s2 = scenes.config2(n_photons=200_000)
    print("case noalloc c2 fp32 2e5 photons, then c1 fp64 2e4", flush=True)
    _same_render(M, s2, "fp32")
    s1 = scenes.config1(n_photons=20_000)
    _same_render(M, s1, "fp64")
    # and the compensated FP32 tally on the small grid
    _same_render(M, s1, "fp32", tally="kahan32")


def test_noalloc_refuses_inputs_beyond_its_scratch(M):
    import torch
    s5 = scenes.config5(n_photons=1000)
    print("case noalloc scratch limit (256x256x128 fp64)", flush=True)
    beta = M.beta_tensor(s5, "fp64")  # 64 MiB of extinction alone
    out = torch.full((M.n_pixels(s5),), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(M.McError) as e:
        M.mc_render_noalloc(s5, beta, transport="fp64", out=out)
    assert e.value.code == M.MC_ERR_SCRATCH_LIMIT
    torch.cuda.synchronize()
    assert bool((out == -7.0).all())
    # the same grid in FP32 transport fits
    img, st = M.mc_render_noalloc(s5, M.beta_tensor(s5, "fp32"), out=out)
    assert st["photons"] == 1000 and bool(torch.isfinite(img).all())
