"""The gather capture (a diagnostic of the FP32 render): the render it runs
is the plain render (same counters, same images up to the order of the FP64
tally atomics), and every captured index is either n_vox (a lane with no
ray or in an empty run, which the walk's buffer answers with zero and no
memory access) or a voxel whose extinction is not zero; the wavefronts'
steps account for every connection-ray voxel visit."""
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


def test_capture_is_the_render(M):
    s = scenes.config2(n_photons=400_000)
    print("case gather capture c2 4e5 photons", flush=True)
    beta = M.beta_tensor(s, "fp32")
    idx, steps, nw, st = M.mc_capture_gathers(s, beta, 100, 32, 4096)
    ref, rst = M.mc_render(s, beta)
    assert st == rst
    assert 0 < nw <= 4096
    steps = steps[:nw].cpu().numpy().astype(np.int64)
    # each lane-step of a busy lane is one voxel visit
    assert 64 * steps.sum() >= rst["vox_conn"]
    full = steps >= 132
    assert full.any()
    got = idx[:nw].cpu().numpy().view(np.uint32)[full]
    # the walk skips the loads of empty runs of 2^msh voxels (the FP32
    # render's bitmask holds at most 131072 runs)
    msh = 0
    while -(-s.n_vox // (1 << msh)) > 131072:
        msh += 1
    run = 1 << msh
    pad = np.zeros(-(-s.n_vox // run) * run, bool)
    pad[:s.n_vox] = s.beta > 0
    run_occ = pad.reshape(-1, run).any(axis=1)
    occupied = np.append(run_occ[np.arange(s.n_vox) >> msh], True)  # the last entry: the zero word
    assert got.max() <= s.n_vox
    assert occupied[got].all()
    # waves that stopped before the window left it untouched
    assert (idx[:nw].cpu().numpy()[steps < 100] == -1).all()
