"""Pins of the oracle's air + aerosol mixture (the particle choice of step
iv, the Rayleigh phase function Eq. (Pray) and its sampling Eq. (thetaREY),
the per-channel extinction of Eq. (channelBeta)) and of its two gradients:
the surrogate with the in-scatter field frozen and the full derivative of
the expected images (path probabilities included)."""
import math

import numpy as np
import pytest

from paper_1512_02110_amd import scenes
from tests._scene_helpers import (hg, look_camera, pixel_grid, rayleigh, single_scatter_image,
                                  sun_direction)


def test_rayleigh_phase_normalised_and_symmetric(oracle):
    x, w = np.polynomial.legendre.leggauss(8)  # exact for the degree-2 polynomial
    assert abs(2 * math.pi * sum(wi * oracle.rayleigh_phase(xi) for xi, wi in zip(x, w)) - 1) < 1e-14
    for c in (0.0, 0.3, 0.77, 1.0):
        assert oracle.rayleigh_phase(c) == oracle.rayleigh_phase(-c)
        assert abs(oracle.rayleigh_phase(c) - rayleigh(c)) < 1e-16
    assert abs(oracle.rayleigh_phase(1.0) / oracle.rayleigh_phase(0.0) - 2.0) < 1e-15


def test_rayleigh_sampling_inverts_its_cdf(oracle):
    # the CDF of mu by quadrature of 2 pi P_Ray over [-1, mu] (Gauss-Legendre,
    # exact for the polynomial), not from the cubic the sampler solves
    x, w = np.polynomial.legendre.leggauss(6)

    def cdf(mu):
        a, b = -1.0, mu
        t = 0.5 * (a + b) + 0.5 * (b - a) * x
        return 2 * math.pi * 0.5 * (b - a) * float(np.dot(w, [rayleigh(ti) for ti in t]))

    us = np.linspace(0.0, 1.0, 401)
    mus = np.array([oracle.rayleigh_sample(u) for u in us])
    assert mus[0] == pytest.approx(-1.0, abs=1e-12) and mus[-1] == pytest.approx(1.0, abs=1e-12)
    assert abs(oracle.rayleigh_sample(0.5)) < 1e-15
    assert np.all(np.diff(mus) > 0)
    assert max(abs(cdf(m) - u) for m, u in zip(mus, us)) < 1e-12
    # moments of the stratified sample: E[mu] = 0, E[mu^2] = 2/5
    um = (np.arange(4000) + 0.5) / 4000
    m = np.array([oracle.rayleigh_sample(u) for u in um])
    assert abs(m.mean()) < 1e-12 and abs((m * m).mean() - 0.4) < 1e-6


def _tiny_scene(rng, n_photons):
    cams = [look_camera((0.12, 0.17, -0.25), (0.1, 0.05, 1.0), (0, -1, 0), 4, 4, 70.0),
            look_camera((0.45, 0.1, 0.08), (-1.0, 0.3, 0.15), (0, 0, 1), 3, 5, 60.0, cx=1.2, cy=2.6)]
    beta = rng.uniform(0.5, 12.0, size=3 * 3 * 2)
    beta[4] = 0.0
    return scenes.Scene(3, 3, 2, 0.1, 0.1, 0.1, beta, cams, 0.8, 0.6, math.radians(35.0), 0.7, n_photons, 4)


def test_without_air_the_mixture_is_the_single_constituent_model(oracle):
    rng = np.random.default_rng(11)
    s = _tiny_scene(rng, 4000)
    zero = np.zeros_like(s.beta)
    img, st = oracle.render(s)
    img_m, st_m = oracle.render_mix(s, zero, s.beta, sigma=1.0)
    assert st_m == st
    assert np.array_equal(img_m, img)
    # the channel ratio scales the aerosol field (Eq. channelBeta)
    img2, st2 = oracle.render(s, beta=2.5 * s.beta)
    img2_m, st2_m = oracle.render_mix(s, zero, s.beta, sigma=2.5)
    assert st2_m == st2
    np.testing.assert_allclose(img2_m, img2, rtol=1e-11, atol=1e-14 * abs(img2).max())
    dl = rng.normal(size=img.size)
    g, _ = oracle.grad_beta(s, dl)
    g_m, _ = oracle.grad_mix(s, dl, zero, s.beta, sigma=1.0)
    assert np.array_equal(g_m, g)
    # accumulation into the caller's array
    g_acc, _ = oracle.grad_mix(s, dl, zero, s.beta, sigma=1.0, grad=g_m.copy())
    np.testing.assert_allclose(g_acc, 2 * g, rtol=1e-12, atol=1e-15 * abs(g).max())


def _slab_mix(mu, cs, g, tau_air, tau_aer, mu0, albedo):
    """Single-scatter radiance below a homogeneous mixed slab (per unit
    irradiance at cosine mu0): the one-constituent slab form with albedo P
    replaced by the extinction-weighted source (tau_air P_Ray + albedo tau_aer
    P_HG) / tau."""
    tau = tau_air + tau_aer
    src = (tau_air * rayleigh(cs) + albedo * tau_aer * hg(g, cs)) / tau
    if abs(mu - mu0) < 1e-9:
        return src * tau * math.exp(-tau / mu0) / mu0
    return src * mu0 * (math.exp(-tau / mu) - math.exp(-tau / mu0)) / (mu - mu0)


def _slab_scene(tau_air, tau_aer, n_photons, seed=0):
    cam = look_camera((0.8, 0.8, -0.3), (0, 0, 1), (0, -1, 0), 6, 6, 40.0)
    s = scenes.homogeneous_slab(nx=16, ny=16, nz=4, dx=0.1, dz=0.05, tau=1.0, albedo=0.7, g=0.5,
                                sun_zenith_deg=30.0, cams=[cam], n_photons=n_photons, seed=seed)
    H = s.nz * s.dz
    return s, np.full(s.beta.size, tau_air / H), np.full(s.beta.size, tau_aer / H)


def _slab_expect(s, tau_air, tau_aer):
    cam = s.cameras[0]
    w_sun = sun_direction(s)
    mu0 = math.cos(s.sun_zenith)
    out = np.zeros(cam.width * cam.height)
    for row in range(cam.height):
        for col in range(cam.width):
            d, wts = pixel_grid(cam, row, col, 12)
            v = [_slab_mix(di[2], float(w_sun @ -di), s.g, tau_air, tau_aer, mu0, s.albedo) for di in d]
            out[row * cam.width + col] = np.dot(v, wts) / wts.sum()
    return out


@pytest.mark.parametrize("tau_air,tau_aer", [(0.8, 0.0), (0.5, 0.7)])
def test_single_scatter_slab_closed_form(oracle, tau_air, tau_aer):
    # pure air (the scene's albedo 0.7 must not apply) and a mixture
    s, b_air, b_aer = _slab_scene(tau_air, tau_aer, 1_500_000)
    img, st, m2 = oracle.render_mix(s, b_air, b_aer, with_m2=True, max_events=1)
    N = st["photons"]
    sigma = np.sqrt(np.maximum(m2 - img ** 2 / N, 0))
    expect = _slab_expect(s, tau_air, tau_aer)
    z = (img - expect) / sigma
    assert np.all(np.abs(z) < 5), z
    assert abs(img.sum() / expect.sum() - 1) < 0.015


def test_heterogeneous_mixture_single_scatter_quadrature(oracle):
    rng = np.random.default_rng(5)
    s = _tiny_scene(rng, 2_000_000)
    b_air = rng.uniform(0.0, 6.0, size=s.beta.size)
    b_air[[2, 9]] = 0.0
    b_aer = s.beta.copy()
    s_tot = s.with_beta(b_air + b_aer)
    img, st, m2 = oracle.render_mix(s, b_air, b_aer, with_m2=True, max_events=1)
    N = st["photons"]
    sigma = np.sqrt(np.maximum(m2 - img ** 2 / N, 0))
    ref = np.concatenate([single_scatter_image(s_tot, c, n_sub=24, mix=(b_air, b_aer))
                          for c in s.cameras])
    tol = 4 * sigma + 0.005 * ref + 1e-3 * ref.max()
    assert np.all(np.abs(img - ref) <= tol), np.c_[img, ref, sigma]
    assert (ref > 0).sum() >= 15


def test_full_gradient_is_the_derivative_of_the_single_scatter_image(oracle):
    """Single scattering (one collision per photon) below a mixed slab: the
    derivative of the closed-form image along the aerosol field equals
    sum_m beta_aer(m) dI/dbeta_aer(m) of the full gradient (Monte Carlo error
    from 8 independent batches); the surrogate, which misses the score of
    the free flight to the collision, does not."""
    tau_air, tau_aer = 0.4, 0.8
    n_b, per = 8, 250_000
    s, b_air, b_aer = _slab_scene(tau_air, tau_aer, per)
    wpix = np.linspace(0.5, 1.5, s.cameras[0].width * s.cameras[0].height)  # dL/d image
    eps = 1e-5
    d_cf = (np.dot(wpix, _slab_expect(s, tau_air, tau_aer * (1 + eps)))
            - np.dot(wpix, _slab_expect(s, tau_air, tau_aer * (1 - eps)))) / (2 * eps)
    full, surr = [], []
    for b in range(n_b):
        kw = dict(max_events=1, photon_offset=b * per, n_photons_norm=per)
        g_f, _ = oracle.grad_mix(s, wpix, b_air, b_aer, full=True, **kw)
        g_s, _ = oracle.grad_mix(s, wpix, b_air, b_aer, full=False, **kw)
        full.append(float(np.dot(b_aer, g_f)))
        surr.append(float(np.dot(b_aer, g_s)))
    full, surr = np.array(full), np.array(surr)
    se = full.std(ddof=1) / math.sqrt(n_b)
    assert abs(full.mean() - d_cf) < 4 * se + 0.01 * abs(d_cf), (full.mean(), d_cf, se)
    se_s = surr.std(ddof=1) / math.sqrt(n_b)
    assert abs(surr.mean() - d_cf) > 8 * max(se, se_s), (surr.mean(), d_cf)


def _box_lengths(s, p, q):
    """Length of the segment p -> q inside every voxel box (slab clipping per
    box, no walk)."""
    d = np.array([s.dx, s.dy, s.dz])
    v = q - p
    out = np.zeros(s.nx * s.ny * s.nz)
    for iz in range(s.nz):
        for iy in range(s.ny):
            for ix in range(s.nx):
                lo = np.array([ix, iy, iz]) * d
                hi = lo + d
                t0, t1 = 0.0, 1.0
                for a in range(3):
                    if abs(v[a]) < 1e-300:
                        if not (lo[a] <= p[a] <= hi[a]):
                            t1 = -1.0
                        continue
                    ta, tb = sorted(((lo[a] - p[a]) / v[a], (hi[a] - p[a]) / v[a]))
                    t0, t1 = max(t0, ta), min(t1, tb)
                if t1 > t0:
                    out[ix + s.nx * (iy + s.ny * iz)] = (t1 - t0) * np.linalg.norm(v)
    return out


def test_full_gradient_brute_force_in_prefix_form(oracle):
    """Multiple scattering, aerosol only: the oracle accumulates the score
    terms with suffix sums A_s over later estimates; here the same gradient is
    summed the other way round, per estimate over its path prefix, from the
    traced events, per-box segment lengths and the LE of Eq. (fle) rebuilt
    from the oracle's pinned parts."""
    rng = np.random.default_rng(21)
    n = 300
    s = _tiny_scene(rng, n)
    zero = np.zeros_like(s.beta)
    max_rec = 200
    ev, paths, pix = oracle.trace_paths(s, 0, n, max_rec)
    assert paths["n_events"].max() <= max_rec
    assert paths["n_events"].max() >= 3
    n_pix = sum(c.width * c.height for c in s.cameras)
    dl = rng.normal(size=n_pix)
    norm = oracle.normalisation(s, n_photons=n)
    off = np.cumsum([0] + [c.width * c.height for c in s.cameras])
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    expect = np.zeros(s.beta.size)
    for pid in range(n):
        r = oracle.philox([pid & 0xFFFFFFFF, pid >> 32, 0, 0], [s.seed & 0xFFFFFFFF, s.seed >> 32])
        X_prev = np.array([oracle.uniform(r[0]) * L[0], oracle.uniform(r[1]) * L[1], L[2]])
        prefix = np.zeros(s.beta.size)
        for e in range(paths["n_events"][pid]):
            E = ev[pid, e]
            X = np.array([E["x"], E["y"], E["z"]])
            w_in = (X - X_prev) / np.linalg.norm(X - X_prev)
            prefix -= _box_lengths(s, X_prev, X)
            prefix[E["voxel"]] += 1.0 / s.beta[E["voxel"]]
            a_e = 0.0
            for c, cam in enumerate(s.cameras):
                pp = pix[pid, e, c]
                if pp < 0:
                    continue
                Xc = np.array(cam.pos)
                V = Xc - X
                r2 = float(V @ V)
                tau, _ = oracle.optical_depth(s, X, Xc)
                C = s.albedo * E["w"] * hg(s.g, float(w_in @ V) / math.sqrt(r2)) * math.exp(-tau) / r2
                a = dl[off[c] + pp] * norm[off[c] + pp] * C
                a_e += a
                expect -= a * _box_lengths(s, X, Xc)
            expect += a_e * prefix
            X_prev = X
    got, _ = oracle.grad_mix(s, dl, zero, s.beta, full=True)
    scale = np.abs(expect).max()
    assert scale > 0
    np.testing.assert_allclose(got, expect, rtol=1e-8, atol=1e-10 * scale)
