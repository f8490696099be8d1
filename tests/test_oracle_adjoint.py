"""Pins of the oracle's surrogate gradient (Sec. 5.2, Eqs. (Jaco1),
(TcofJaco1), (DivTc)): with the in-scatter field frozen at the events of the
current render, each local estimate C_e varies with beta as
C_e * beta(k_e)/beta0(k_e) * exp(-sum_m l_e(m) (beta(m) - beta0(m))).
The frozen-event render evaluates exactly this image; its central finite
differences must match the adjoint."""
import math

import numpy as np
import pytest

from paper_1512_02110_amd import scenes


def _scene(seed=0, n=400):
    s = scenes.config3_initial(n_photons=n, seed=seed)
    return s


def test_frozen_render_at_same_beta_equals_render(oracle):
    s = _scene(n=2000)
    a, sta = oracle.render(s)
    b, stb = oracle.render_frozen(s, s.beta, s.beta)
    assert np.array_equal(a, b)
    assert sta == stb


def test_frozen_render_keeps_events(oracle):
    # transport depends only on beta_sample: event statistics do not change
    s = _scene(n=2000)
    _, st0 = oracle.render_frozen(s, s.beta, s.beta)
    _, st1 = oracle.render_frozen(s, s.beta, 1.3 * s.beta + 0.1)
    for k in ("events", "le_jobs", "vox_free", "esc_top", "esc_bottom", "esc_side"):
        assert st0[k] == st1[k]


@pytest.mark.parametrize("loss", ["linear", "l2"])
def test_gradient_matches_central_differences(oracle, loss):
    s = _scene(n=600)
    beta0 = s.beta.copy()
    img0, _ = oracle.render(s)
    rng = np.random.default_rng(3)
    if loss == "linear":
        gvec = rng.normal(size=img0.size)
        meas = None
    else:
        meas = img0 * (1 + 0.3 * rng.normal(size=img0.size))
        gvec = 2 * (img0 - meas)

    def L(beta):
        i, _ = oracle.render_frozen(s, beta0, beta)
        return float(gvec @ i) if loss == "linear" else float(((i - meas) ** 2).sum())

    grad, _ = oracle.grad_beta(s, gvec)
    # 64 voxels drawn at random plus the largest-gradient ones
    idx = np.unique(np.concatenate([rng.choice(s.n_vox, 64, replace=False),
                                    np.argsort(-np.abs(grad))[:16]]))
    for m in idx:
        h = 1e-3 * beta0[m] if beta0[m] > 0 else 1e-4
        bp, bm = beta0.copy(), beta0.copy()
        bp[m] += h
        bm[m] -= h
        if bm[m] < 0:  # one-sided at beta = 0 (no collisions there)
            bm[m] = beta0[m]
            fd = (L(bp) - L(bm)) / h
            tol = 1e-3 * abs(fd) + 1e-9 * np.abs(grad).max()
        else:
            fd = (L(bp) - L(bm)) / (2 * h)
            tol = 1e-5 * abs(fd) + 1e-9 * np.abs(grad).max()
        assert abs(grad[m] - fd) <= tol, (m, grad[m], fd)


def test_single_event_gradient_closed_form(oracle):
    """One photon, one collision, one camera: dC/dbeta(m) = C (delta/beta(k)
    - l(m)); summed over m with weights beta(m), the total is
    C (1 - tau_c) where tau_c is the optical depth of the connection."""
    s = _scene(n=1)
    s.cameras = s.cameras[:1]
    for pid in range(200):
        ev, paths, pix = oracle.trace_paths(s, pid, 1, 4, max_events=1)
        if paths["n_events"][0] == 1 and pix[0, 0, 0] >= 0:
            break
    else:
        pytest.skip("no visible single collision found")
    g = np.zeros(s.cameras[0].n_pix)
    g[pix[0, 0, 0]] = 1.0
    grad, _ = oracle.grad_beta(s, g, photon_offset=pid, n_photons=1, max_events=1)
    img, _ = oracle.render(s, photon_offset=pid, n_photons=1, max_events=1)
    C = img[pix[0, 0, 0]]
    e = ev[0, 0]
    cam = s.cameras[0]
    tau_c, _ = oracle.optical_depth(s, [e["x"], e["y"], e["z"]], cam.pos)
    assert abs(grad @ s.beta - C * (1 - tau_c)) < 1e-12 * abs(C) * (1 + tau_c)
    k = e["voxel"]
    # the collision voxel holds the +C/beta(k) term minus its own segment
    others = grad.copy()
    others[k] = 0
    assert np.all(others <= 0)
