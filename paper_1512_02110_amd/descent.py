"""Recovery of the extinction field by projected gradient descent with the
Monte Carlo surrogate gradient (Sec. 5.2, Eqs. Cost and GD; the error
measures delta_mass and eps of Sec. 7).

Iteration q renders the images of the current beta with photon seed
seed0 + q (mc_render), forms the image gradient of the L2 data term
dL/di = 2 (i - i_measured) (mc_image_residual), takes the surrogate gradient
on the same photons (mc_grad_beta: the in-scatter field frozen at the
render's events) and steps beta <- max(beta - delta grad, 0) (mc_gd_step).
The step size is fixed at the first iteration so that its step moves the
largest |grad| voxel by step_frac of max beta0, unless given.  Every step of
the loop runs in the library's kernels; this module only sequences the
calls.

The voxelised route (Secs. 3 and 6, mc_voxel_descent) runs the same
problem the way the paper recovers: per outer iteration one photon pass for
the in-scatter field j of the voxelised model, then n_gd steps on the images
of that model with j frozen and the per-camera conditioning Q_c; its step
size starts at 5% of max beta0 over the largest first conditioned gradient
and is halved whenever an outer iteration's steps do not all lower its cost
(that iteration is then taken again).

    python -m paper_1512_02110_amd.descent [--config c5] [--iters 50] [--photons 250000000]
                                           [--model le|voxel] [--conditioned 1] [--n-gd 5]
                                           [--start smoothed|uniform] [--grow 1.25]

prints one JSON line per iteration (loss, relative image residual,
delta_mass and eps against the true field) and a summary line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def mc_descent(s, beta0, measured, n_iter, delta=None, step_frac=0.05, seed0=1000, transport="fp32", truth=None,
               log=None, tape_limit=0):
    """Runs n_iter iterations from beta0 (float64 CUDA tensor, not modified).
    Returns (beta, records, delta); a record holds the iteration's loss
    sum (i - i_measured)^2 and relative residual |i - i_measured| / |i_measured|
    before its step, and (with truth) delta_mass and eps of the beta the step
    starts from; the last record also has the errors after the last step."""
    import torch
    from paper_1512_02110_amd import mcrt as M
    b = beta0.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1).clone()
    meas = measured.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
    meas_norm = float(torch.linalg.vector_norm(meas))
    b_max0 = float(b.max())
    recs = []
    for it in range(n_iter):
        t0 = time.perf_counter()
        bt = b.float() if transport == "fp32" else b
        img, st = M.mc_render(s, bt, transport=transport, seed=seed0 + it)
        dl, loss = M.mc_image_residual(img, meas)
        g, _ = M.mc_grad_beta(s, bt, dl, transport=transport, seed=seed0 + it, stats=False, tape_limit=tape_limit)
        ga = g.abs()
        gmax, kmax = ga.max(dim=0)
        gmax, kmax = float(gmax), int(kmax)
        if delta is None:
            delta = step_frac * b_max0 / gmax
        loss = float(loss.item())
        rec = {"iter": it, "seed": seed0 + it, "loss": loss,
               "residual": math.sqrt(loss) / meas_norm if meas_norm > 0 else 0.0, "events": st["events"],
               # where the gradient peaks (voxel indices) and how that compares with its bulk
               "grad_max": gmax, "grad_max_voxel": [kmax % s.nx, (kmax // s.nx) % s.ny, kmax // (s.nx * s.ny)],
               "grad_p999": float(torch.quantile(ga[ga > 0][:16_000_000].float(), 0.999)) if bool((ga > 0).any())
               else 0.0,
               "step_max": delta * gmax}
        if truth is not None:
            rec["delta_mass"], rec["eps"] = M.mc_recovery_error(b, truth)
        M.mc_gd_step(b, g, delta)
        torch.cuda.synchronize()
        rec["seconds"] = time.perf_counter() - t0
        if truth is not None and it == n_iter - 1:
            rec["delta_mass_after"], rec["eps_after"] = M.mc_recovery_error(b, truth)
        recs.append(rec)
        if log is not None:
            log(rec)
    return b, recs, delta


def mc_voxel_descent(s, beta0, measured, n_outer, n_gd=5, delta=None, conditioned=1, rays_per_side=2, eta=0.0,
                     seed0=1000, transport="fp32", truth=None, log=None, max_halvings=12, backtrack=True,
                     grow=1.0):
    """The voxelised-model recovery loop from beta0 (float64 CUDA tensor, not
    modified): n_outer calls of mc_recover with one outer iteration each
    (photon seed seed0 + q).  With j frozen the cost of an outer iteration is
    a smooth function of beta, so its steps must lower it: with backtrack,
    an outer iteration whose costs do not fall at every step is taken again
    from the same beta and photons with half the step (at most max_halvings
    times); an iteration that needed no halving multiplies the step by grow
    for the next one.  The first step size is 5% of max beta0 over the
    largest first (conditioned) gradient unless given.  Returns (beta, records, delta); a
    record holds the outer iteration's costs before each of its steps, the
    step size used and the halvings it took, and, with truth, delta_mass
    and eps after its last step."""

    import torch
    from paper_1512_02110_amd import mcrt as M
    b = beta0.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1).clone()
    meas = measured.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
    meas_norm = float(torch.linalg.vector_norm(meas))
    kw = dict(rays_per_side=rays_per_side, eta=eta, conditioned=conditioned, transport=transport)
    if delta is None:
        j0, _ = M.mc_voxel_scatter(s, b.float() if transport == "fp32" else b, transport=transport, seed=seed0,
                                   stats=False)
        img0 = M.mc_voxel_render(s, b, j0, rays_per_side)
        dl0, _ = M.mc_image_residual(img0, meas)
        counts, q = M.mc_voxel_conditioning(s, rays_per_side)
        g0 = M.mc_voxel_grad(s, b, j0, dl0, rays_per_side, cam_weights={0: None, 1: q, 2: counts}[conditioned])
        delta = 0.05 * float(b.max()) / float(g0.abs().max())
        del j0, img0, dl0, counts, q, g0
    recs = []
    for it in range(n_outer):
        t0 = time.perf_counter()
        halvings = 0
        while True:
            b_new, c = M.mc_recover(s, b, meas, delta, n_gd, 1, seed=seed0 + it, **kw)
            if not backtrack or np.all(np.diff(c) < 0) or halvings == max_halvings:
                break
            delta *= 0.5
            halvings += 1
        b = b_new
        torch.cuda.synchronize()
        rec = {"iter": it, "seed": seed0 + it, "cost": [float(x) for x in c],
               "residual_first_step": math.sqrt(max(float(c[0]), 0.0)) / meas_norm if meas_norm > 0 else 0.0,
               "seconds": time.perf_counter() - t0, "delta": delta, "halvings": halvings}
        if halvings == 0:
            delta *= grow
        if truth is not None:
            rec["delta_mass"], rec["eps"] = M.mc_recovery_error(b, truth)
        recs.append(rec)
        if log is not None:
            log(rec)
    return b, recs, delta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c5")
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--photons", type=int, default=250_000_000)
    ap.add_argument("--transport", default="fp32")
    ap.add_argument("--step-frac", type=float, default=0.05)
    ap.add_argument("--model", choices=("le", "voxel"), default="le",
                    help="le: local-estimation render and surrogate gradient; voxel: the voxelised model")
    ap.add_argument("--conditioned", type=int, default=1, help="voxel model: 0 none, 1 Q_c = 1/count, 2 count")
    ap.add_argument("--n-gd", type=int, default=5)
    ap.add_argument("--start", choices=("smoothed", "uniform"), default="smoothed",
                    help="smoothed: 0.7 x the true field smoothed over one voxel; uniform: the true field's mean")
    ap.add_argument("--grow", type=float, default=1.0, help="voxel model: step growth after an accepted iteration")
    args = ap.parse_args(argv)
    import torch
    from paper_1512_02110_amd import mcrt as M
    from paper_1512_02110_amd import scenes
    M.load_library()
    truth = scenes.CONFIGS[args.config](n_photons=args.photons)
    t64 = torch.as_tensor(truth.beta, dtype=torch.float64, device="cuda")
    if args.start == "uniform":
        b0 = torch.full((truth.n_vox,), float(truth.beta.mean()), dtype=torch.float64, device="cuda")
        start = "start: uniform at the true field's mean extinction"
    else:
        b0 = torch.as_tensor(0.7 * scenes.smooth(truth.beta3d(), 1.0).reshape(-1), dtype=torch.float64,
                             device="cuda")
        start = "start: 0.7 x the true field smoothed over one voxel"
    e0 = M.mc_recovery_error(b0, t64)
    t0 = time.perf_counter()
    if args.model == "voxel":
        # measured images: the voxelised model of the true field (photon seed 99, 2x2 rays per pixel) as
        # 10-bit grey levels with seeded read noise (Eq. noise), back in radiance units
        jt, _ = M.mc_voxel_scatter(truth, M.beta_tensor(truth, "fp32"), seed=99, stats=False)
        clean = M.mc_voxel_render(truth, t64, jt, 2)
        del jt
        normals = torch.as_tensor(np.random.default_rng(5).normal(size=clean.numel()), device="cuda")
        grey, scale = M.mc_camera_noise(clean, normals)
        meas = grey / scale
        del clean, normals, grey
        print(json.dumps({"workload": f"{args.config}: {truth.nx}x{truth.ny}x{truth.nz} voxels, {truth.n_cams} "
                                      f"cameras, voxelised model, {args.photons:.2e} photons per outer iteration, "
                                      f"{args.n_gd} steps per outer iteration, conditioning {args.conditioned}; "
                                      f"measured images: the voxelised model of the true field (seed 99) with "
                                      f"camera noise; {start}", "iters": args.iters,
                          "delta_mass_start": e0[0], "eps_start": e0[1]}), flush=True)
        _, recs, delta = mc_voxel_descent(truth, b0, meas, args.iters, n_gd=args.n_gd,
                                          conditioned=args.conditioned, truth=t64, grow=args.grow,
                                          log=lambda r: print(json.dumps(r), flush=True))
        print(json.dumps({"summary": True, "delta": delta, "seconds": time.perf_counter() - t0,
                          "cost_first": recs[0]["cost"][0], "cost_last": recs[-1]["cost"][-1],
                          "eps_start": e0[1], "eps_last": recs[-1]["eps"], "eps_min": min(r["eps"] for r in recs),
                          "delta_mass_start": e0[0], "delta_mass_last": recs[-1]["delta_mass"]}), flush=True)
        return
    # measurements: the true field rendered with photon seed 1
    meas, _ = M.mc_render(truth, M.beta_tensor(truth, args.transport), transport=args.transport, seed=1,
                          stats=False)
    print(json.dumps({"workload": f"{args.config}: {truth.nx}x{truth.ny}x{truth.nz} voxels, {truth.n_cams} cameras, "
                                  f"{args.photons:.2e} photons per render and per gradient, {args.transport} "
                                  f"transport; measured images: the true field, photon seed 1; {start}",
                      "iters": args.iters}), flush=True)
    _, recs, delta = mc_descent(truth, b0, meas, args.iters, step_frac=args.step_frac, transport=args.transport,
                                truth=t64, log=lambda r: print(json.dumps(r), flush=True))
    print(json.dumps({"summary": True, "delta": delta, "seconds": time.perf_counter() - t0,
                      "loss_first": recs[0]["loss"], "loss_last": recs[-1]["loss"],
                      "residual_first": recs[0]["residual"], "residual_last": recs[-1]["residual"],
                      "eps_first": recs[0]["eps"], "eps_last": recs[-1]["eps_after"],
                      "delta_mass_first": recs[0]["delta_mass"], "delta_mass_last": recs[-1]["delta_mass_after"]}),
          flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
