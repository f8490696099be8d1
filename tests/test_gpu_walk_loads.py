"""The connection walks' two ways of reading the extinction, through the C ABI.

By default the render's and the tape's walks fetch through a buffer over
the voxels, so that a lane whose ray has ended or which is in an empty run
reads zero without a memory access.  Grids whose voxels exceed a buffer's
range take plain loads of the zero word instead; MC_PLAIN_WALK_LOADS=1
forces that path on the small grids here.  Both read the same values in the
same order per ray, so the counters are equal and the images and gradients
agree up to the order of the FP64 atomic sums."""
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


def _both(monkeypatch, fn):
    """fn() with the buffer, then with plain loads."""
    a = fn()
    monkeypatch.setenv("MC_PLAIN_WALK_LOADS", "1")
    try:
        b = fn()
    finally:
        monkeypatch.delenv("MC_PLAIN_WALK_LOADS")
    return a, b


def _close(a, b, rtol):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(np.abs(a) > 0, np.abs(b) > 0)
    scale = np.abs(a).max(initial=0.0)
    assert scale > 0
    assert np.allclose(a, b, rtol=rtol, atol=1e-13 * scale), np.abs(a - b).max() / scale


@pytest.mark.parametrize("transport,tally", [("fp32", "f64"), ("fp64", "f64"), ("mixed", "f64"),
                                             ("fp32", "kahan32")])
def test_render_plain_loads_match_buffer(M, monkeypatch, transport, tally):
    s = scenes.config2(n_photons=200_000)
    print(f"case plain vs buffer walk loads: c2 2e5 photons {transport} {tally}", flush=True)
    b = M.beta_tensor(s, transport)
    (i1, s1), (i2, s2) = _both(monkeypatch, lambda: M.mc_render(s, b, transport=transport, tally=tally, seed=7))
    assert s1 == s2
    # the compensated FP32 tally rounds in the order its atomics land
    _close(i1, i2, 1e-12 if tally == "f64" else 1e-5)


@pytest.mark.parametrize("transport", ["fp32", "fp64"])
def test_kept_and_replayed_gradients_plain_loads_match_buffer(M, monkeypatch, transport):
    import torch
    s = scenes.config2(n_photons=200_000)
    print(f"case plain vs buffer walk loads: c2 kept-ray render + gradient, replay gradient, {transport}",
          flush=True)
    b = M.beta_tensor(s, transport)
    dl = torch.as_tensor(np.random.default_rng(5).normal(size=M.n_pixels(s)), device="cuda")

    def run():
        img, st, tape = M.mc_render_tape(s, b, transport=transport, seed=3)
        assert tape is not None
        g_kept, _ = M.mc_grad_beta(s, b, dl, transport=transport, seed=3, tape=tape)
        tape.free()
        g_rep, st_rep = M.mc_grad_beta(s, b, dl, transport=transport, seed=3, tape_limit=5_000_000)
        return img, st, g_kept, g_rep, st_rep

    (i1, s1, k1, r1, t1), (i2, s2, k2, r2, t2) = _both(monkeypatch, run)
    assert s1 == s2 and t1 == t2
    _close(i1, i2, 1e-12)
    _close(k1, k2, 1e-10)
    _close(r1, r2, 1e-10)
    _close(k1, r1, 1e-10)


def test_capture_refuses_plain_load_walks(M, monkeypatch):
    """The gather capture runs the buffer walk only: with plain loads forced
    it returns MC_ERR_INVALID_ARG, as an argument error, before enqueueing
    anything."""
    s = scenes.config2(n_photons=10_000)
    print("case gather capture with plain walk loads forced: rejected", flush=True)
    b = M.beta_tensor(s, "fp32")
    monkeypatch.setenv("MC_PLAIN_WALK_LOADS", "1")
    with pytest.raises(M.McError) as e:
        M.mc_capture_gathers(s, b, 0, 8, 64)
    assert e.value.code == M.MC_ERR_INVALID_ARG
    monkeypatch.delenv("MC_PLAIN_WALK_LOADS")
    idx, steps, nw, st = M.mc_capture_gathers(s, b, 0, 8, 64)
    assert st["photons"] == s.n_photons and nw > 0
