"""Helpers for tests: general camera poses and closed forms from the paper."""
import math

import numpy as np

from paper_1512_02110_amd import scenes


def look_camera(pos, forward, up_hint, width, height, fov_deg, cx=None, cy=None):
    """Pinhole camera at pos looking along forward.  R rows: right, down, forward."""
    f = np.asarray(forward, float)
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up_hint, float))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    foc = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return scenes.Camera(tuple(map(float, pos)), tuple(map(float, R.reshape(-1))), foc, foc,
                         width / 2.0 if cx is None else cx, height / 2.0 if cy is None else cy,
                         width, height)


def sun_direction(s):
    """Propagation direction of sunlight (photons travel towards -s)."""
    return -np.array([math.sin(s.sun_zenith) * math.cos(s.sun_azimuth),
                      math.sin(s.sun_zenith) * math.sin(s.sun_azimuth), math.cos(s.sun_zenith)])


def hg(g, c):
    """Eq. (Phg)."""
    return (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * c) ** 1.5)


def pixel_grid(cam, row, col, n):
    """n x n sub-pixel directions (world frame) and solid-angle weights."""
    R = np.array(cam.R).reshape(3, 3)
    xs = (col + (np.arange(n) + 0.5) / n - cam.cx) / cam.fx
    ys = (row + (np.arange(n) + 0.5) / n - cam.cy) / cam.fy
    X, Y = np.meshgrid(xs, ys)
    q = np.stack([X.ravel(), Y.ravel(), np.ones(X.size)], axis=1)
    nrm = np.linalg.norm(q, axis=1)
    d = (q / nrm[:, None]) @ R  # camera -> world
    w = (1.0 / cam.fx / n) * (1.0 / cam.fy / n) / nrm ** 3
    return d, w


def _exact_tau_along(s, P, v):
    """Optical depth from points P (M,3), inside the box, along unit v to the
    box exit, by sorting all face-plane crossings (no voxel walk).  Returns
    (tau, exit_point)."""
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    d = np.array([s.dx, s.dy, s.dz])
    n = np.array([s.nx, s.ny, s.nz])
    M = P.shape[0]
    texit = np.full(M, np.inf)
    for a in range(3):
        if v[a] > 0:
            texit = np.minimum(texit, (L[a] - P[:, a]) / v[a])
        elif v[a] < 0:
            texit = np.minimum(texit, -P[:, a] / v[a])
    ts = [np.zeros(M), texit]
    for a in range(3):
        if v[a] == 0:
            continue
        planes = np.arange(n[a] + 1) * d[a]
        t = (planes[None, :] - P[:, a:a + 1]) / v[a]
        t = np.where((t > 0) & (t < texit[:, None]), t, texit[:, None])
        ts.append(t)
    T = np.sort(np.column_stack(ts), axis=1)
    mid = 0.5 * (T[:, 1:] + T[:, :-1])
    seg = T[:, 1:] - T[:, :-1]
    Q = P[:, None, :] + mid[:, :, None] * v[None, None, :]
    b = beta_lookup(s, Q)
    return (b * seg).sum(axis=1), P + texit[:, None] * v[None, :]


def beta_lookup(s, Q):
    ix = np.floor(Q[..., 0] / s.dx).astype(int)
    iy = np.floor(Q[..., 1] / s.dy).astype(int)
    iz = np.floor(Q[..., 2] / s.dz).astype(int)
    ok = (ix >= 0) & (ix < s.nx) & (iy >= 0) & (iy < s.ny) & (iz >= 0) & (iz < s.nz)
    out = np.zeros(Q.shape[:-1])
    out[ok] = s.beta3d()[iz[ok], iy[ok], ix[ok]]
    return out


def _break_planes(s, to_sun):
    """Planes (normal, offset) across which the single-scatter integrand
    along a line of sight is not smooth: voxel faces (beta and tau_cam), and
    the planes swept along the sun direction by every voxel edge (tau_sun and
    the top-face shadow boundary)."""
    d = [s.dx, s.dy, s.dz]
    n = [s.nx, s.ny, s.nz]
    planes = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1
        for i in range(n[a] + 1):
            planes.append((e, i * d[a]))
    for a in range(3):  # edges parallel to axis a
        e = np.zeros(3)
        e[a] = 1
        nrm = np.cross(e, to_sun)
        if np.linalg.norm(nrm) < 1e-12:
            continue
        b_, c_ = [x for x in range(3) if x != a]
        for i in range(n[b_] + 1):
            for j in range(n[c_] + 1):
                p = np.zeros(3)
                p[b_], p[c_] = i * d[b_], j * d[c_]
                planes.append((nrm, float(nrm @ p)))
    return planes


def rayleigh(c):
    """Eq. (Pray)."""
    return 3.0 / (16.0 * math.pi) * (1.0 + c * c)


def single_scatter_image(s, cam, n_sub=16, n_gl=4, uniform=False, mix=None):
    """Pixel-averaged single-scatter radiance per unit solar irradiance,
    Eq. (IRTE) with J = albedo P exp(-tau_sun) (Eq. (JEq) for the direct
    beam), by quadrature: sub-pixel directions, then along each line of sight
    Gauss-Legendre on pieces where the integrand is smooth.  Points whose sun
    path leaves through a side face are unlit (light enters at the top).
    mix = (beta_air, beta_aer), flat fields summing to s.beta: the source per
    unit length is then beta_air P_Ray + albedo beta_aer P_HG (air scatters
    with albedo 1)."""
    L = np.array([s.nx * s.dx, s.ny * s.dy, s.nz * s.dz])
    w_sun = sun_direction(s)
    to_sun = -w_sun
    planes = _break_planes(s, to_sun)
    gx, gw = np.polynomial.legendre.leggauss(n_gl)
    pos = np.array(cam.pos, float)
    out = np.zeros(cam.height * cam.width)
    for row in range(cam.height):
        for col in range(cam.width):
            dirs, wts = pixel_grid(cam, row, col, n_sub)
            if uniform:  # average over the image plane instead of the solid angle
                wts = np.ones_like(wts)
            acc = 0.0
            for dvec, wt in zip(dirs, wts):
                t0, t1 = 0.0, np.inf
                for a in range(3):
                    if dvec[a] != 0:
                        ta, tb = sorted(((0 - pos[a]) / dvec[a], (L[a] - pos[a]) / dvec[a]))
                        t0, t1 = max(t0, ta), min(t1, tb)
                    elif not (0 <= pos[a] <= L[a]):
                        t1 = -1.0
                if not t1 > t0:
                    continue
                br = [t0, t1]
                for nrm, off in planes:
                    den = nrm @ dvec
                    if abs(den) > 1e-15:
                        t = (off - nrm @ pos) / den
                        if t0 < t < t1:
                            br.append(t)
                br = np.unique(np.array(br))
                a_, b_ = br[:-1], br[1:]
                keep = b_ - a_ > 1e-14
                a_, b_ = a_[keep], b_[keep]
                # nodes
                tn = 0.5 * (a_ + b_)[:, None] + 0.5 * (b_ - a_)[:, None] * gx[None, :]
                wn = 0.5 * (b_ - a_)[:, None] * gw[None, :]
                X = pos[None, None, :] + tn[:, :, None] * dvec[None, None, :]
                bseg = beta_lookup(s, (pos + 0.5 * (a_ + b_)[:, None] * dvec)[:, None, :])[:, 0]
                # tau from the camera: beta constant on each piece
                tau_start = np.concatenate([[0.0], np.cumsum(bseg * (b_ - a_))[:-1]])
                tau_cam = tau_start[:, None] + bseg[:, None] * (tn - a_[:, None])
                flat = X.reshape(-1, 3)
                tau_sun, ex = _exact_tau_along(s, flat, to_sun)
                lit = np.abs(ex[:, 2] - L[2]) < 1e-9
                cs = float(w_sun @ -dvec)
                if mix is None:
                    src = bseg * s.albedo * hg(s.g, cs)
                else:
                    mid = (pos + 0.5 * (a_ + b_)[:, None] * dvec)[:, None, :]
                    b_air = beta_lookup(s.with_beta(mix[0]), mid)[:, 0]
                    b_aer = beta_lookup(s.with_beta(mix[1]), mid)[:, 0]
                    src = b_air * rayleigh(cs) + s.albedo * b_aer * hg(s.g, cs)
                f = (src[:, None] * np.exp(-tau_cam)
                     * (np.exp(-tau_sun) * lit).reshape(tn.shape))
                acc += wt * (f * wn).sum()
            out[row * cam.width + col] = acc / wts.sum()
    return out
