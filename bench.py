#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (default): 64^3 voxels of 0.02 km with a thresholded fractal cloud
field (max beta 50 km^-1), 9 in-situ cameras of 128x128 px (70 deg FOV) on a
3x3 ground lattice, albedo 0.99, g 0.85, sun zenith 45 deg, 1e8 photons per
render; FP32 transport with FP64 tallies.

One step = the whole hot path on one photon batch: the forward render
(launch, free flights, local estimates to all cameras, albedo/roulette,
scattering, normalisation), then one reverse-mode step for an L2 image loss:
the render that keeps its connection rays (mc_render_tape) and dL/dbeta from
those rays (mc_grad_beta with the tape).  Each step uses its own seed.  The
value is the scattering-event rate of the plain forward render; the adjoint
ratio is (render with tape + gradient) / plain render.  The gradient by
photon replay (no tape) is timed once after the steps, for comparison.

Printed: one JSON line with the forward scattering-event rate (value), the
adjoint cost ratios, the FP32-vs-FP64 transport comparison, the roofline of
the transport kernel and the CPU oracle baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32, dense
PEAK_HBM_GBPS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1512_02110_amd", "csrc", "mcrt_kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_render_c2_hbm_traffic.md")


def _source_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per forward launch from the committed rocprofv3 counter
    summary, or None when the kernels changed since it was taken."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = re.search(r"kernel source sha256\[:16\]: ([0-9a-f]{16})", text)
    b = re.search(r"hbm_bytes_per_launch: ([0-9.eE+]+)", text)
    if not h or not b or h.group(1) != _source_hash():
        return None
    return float(b.group(1))


# one CPU worker: the oracle over a photon range; prints "events seconds"
_CPU_WORKER = """
import sys, time
sys.path.insert(0, {root!r})
from oracle import oracle as O
from paper_1512_02110_amd import scenes
s = scenes.CONFIGS[{cfg!r}](n_photons={n})
t0 = time.perf_counter()
_, st = O.render(s, n_photons={n}, photon_offset={off})
print(st["events"], time.perf_counter() - t0)
"""


def _cpu_model():
    """The host CPU as lscpu (or /proc/cpuinfo) describes it."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Vendor ID", "CPU family", "Model", "CPU(s)", "Thread(s) per core",
                             "Core(s) per socket", "Socket(s)", "CPU max MHz", "Hypervisor vendor"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "Model name" not in info:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return info


def cpu_baseline(cfg, per_proc, procs):
    """The oracle as it stands, P independent single-threaded processes over
    disjoint photon ranges (plain child processes, all ended before the GPU
    work starts)."""
    import subprocess
    from oracle import oracle as O
    O.lib()  # build if needed, before the workers start
    t0 = time.perf_counter()
    kids = [subprocess.Popen([sys.executable, "-c", _CPU_WORKER.format(root=ROOT, cfg=cfg, n=per_proc,
                                                                      off=i * per_proc)],
                             stdout=subprocess.PIPE, text=True, env=dict(os.environ, OMP_NUM_THREADS="1"))
            for i in range(procs)]
    res = []
    for k in kids:
        o, _ = k.communicate()
        if k.returncode != 0:
            raise RuntimeError(f"CPU oracle worker failed ({k.returncode})")
        ev, sec = o.split()
        res.append((int(ev), float(sec)))
    wall = time.perf_counter() - t0
    events = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    return {"value": events / wall, "unit": "scattering events/s", "cores": procs, "kind": "oracle",
            "sample": f"{cfg} workload, photon ids 0..{procs * per_proc - 1} split over {procs} "
                      f"single-threaded processes ({per_proc} photons each), FP64",
            "events": events, "wall_s": round(wall, 3), "cpu_s": round(cpu_s, 3),
            "cpu_s_per_process_min": round(min(r[1] for r in res), 3),
            "per_core": events / cpu_s, "cpu": _cpu_model(), "host_threads": os.cpu_count()}


def _pixel_errors(np, img, ref, sig=None):
    """Per-pixel relative errors of img against ref (pixels where ref > 0)."""
    diff = np.abs(img - ref)
    nz = np.abs(ref) > 0
    rel = diff[nz] / np.abs(ref)[nz]
    out = {"frac_pixels_within_1e-4_rel": float((rel <= 1e-4).mean()) if rel.size else 1.0,
           "pixels_over_1e-4_rel": int((rel > 1e-4).sum()),
           "pixel_rel_err_median": float(np.median(rel)) if rel.size else 0.0,
           "pixel_rel_err_max": float(rel.max()) if rel.size else 0.0,
           "image_rel_l1": float(diff.sum() / max(np.abs(ref).sum(), 1e-300)),
           "nonzero_where_ref_zero": int((np.abs(img) > 0)[~nz].sum())}
    if sig is not None:
        out["frac_pixels_within_max_1e-4_rel_3sigma"] = float((diff <= np.maximum(1e-4 * np.abs(ref), 3 * sig)).mean())
    return out


def precisions(M, torch, np, s, classes=True, seed=1000):
    """FP32, mixed and FP64 transport on the same photons (seed 1000): kernel
    times (HIP events on the launch stream, one warm-up each) and per-pixel
    errors against FP64; sigma of a pixel from both renders' second moments.
    With `classes`, the FP32 differences are split by photon: photons whose
    path differs from FP64 (collisions, fate or exit point; traced for all N),
    photons with the same path but a local estimate in another pixel (the
    first 64 collisions of each traced; photons with more are counted as
    unchecked), and the rest: both images without the first two kinds (and the
    unchecked) are compared again."""
    b32, b64 = M.beta_tensor(s, "fp32"), M.beta_tensor(s, "fp64")
    N = s.n_photons
    res = {}
    for t, b in (("fp32", b32), ("mixed", b64), ("fp64", b64)):
        M.mc_render(s, b, transport=t, seed=7, n_photons=min(N, 10_000_000), stats=False)
        img, st = M.mc_render(s, b, transport=t, seed=seed)
        res[t] = (img, st, st.timing["transport_ms"])
    _, m2_32, _ = M.mc_render_moments(s, b32, transport="fp32", seed=seed, stats=False)
    _, m2_64, _ = M.mc_render_moments(s, b64, transport="fp64", seed=seed, stats=False)
    i64 = res["fp64"][0].cpu().numpy()
    i32 = res["fp32"][0].cpu().numpy()
    sig = np.sqrt(np.maximum(m2_32.cpu().numpy() + m2_64.cpu().numpy() - 2 * i64 ** 2 / N, 0.0))
    del m2_32, m2_64
    t64 = res["fp64"][2]
    out = {"workload": f"same launch as the forward ({N:.0e} photons, seed {seed}), kernel times",
           "fp64": {"kernel_ms": round(t64, 3), "events_per_s": res["fp64"][1]["events"] / (t64 * 1e-3)}}
    counters = ("events", "le_jobs", "vox_free", "esc_top", "esc_bottom", "esc_side", "rr_killed", "capped")
    for t in ("fp32", "mixed"):
        img, st, ms = res[t]
        r = {"kernel_ms": round(ms, 3), "events_per_s": st["events"] / (ms * 1e-3),
             "speedup_over_fp64": round(t64 / ms, 4),
             "counters_equal_fp64": all(st[k] == res["fp64"][1][k] for k in counters),
             "events_minus_fp64": int(st["events"] - res["fp64"][1]["events"])}
        r.update(_pixel_errors(np, img.cpu().numpy(), i64, sig))
        out[t] = r
    out["mixed"]["precision"] = ("photons FP64, connection rays walked in FP32 (transmittance exp in FP32), optical "
                                 "depths and tallies FP64")
    out["fp32"]["precision"] = "photons and connection rays FP32, projection, optical depths and tallies FP64"
    if classes:
        out["fp32"]["classes"] = fp32_classes(M, torch, np, s, b32, b64, i32, i64, sig, seed)
    return out


def fp32_classes(M, torch, np, s, b32, b64, i32, i64, sig, seed, chunk=2_000_000, max_rec=64):
    N = s.n_photons
    tol = 1e-3 * min(s.dx, s.dy, s.dz)
    diverged, flipped, unchecked = [], [], []
    n_est = n_flip_est = 0
    for first in range(0, N, chunk):
        n = min(chunk, N - first)
        _, a, pa = M.mc_trace_paths(s, b32, first, n, max_rec, transport="fp32", seed=seed, device=True)
        _, c, pc = M.mc_trace_paths(s, b64, first, n, max_rec, transport="fp64", seed=seed, device=True)
        d = (a["n_events"] != c["n_events"]) | (a["fate"] != c["fate"]) | \
            ((a["exit_pos"] - c["exit_pos"]).abs().amax(dim=1) > tol)
        rec = (pa > -2) & (pc > -2)
        fl = ((pa != pc) & rec)
        f = fl.flatten(1).any(dim=1) & ~d
        u = (c["n_events"] > max_rec) & ~d & ~f
        n_est += int(((pc >= 0) & rec)[~d].sum())
        n_flip_est += int(fl[~d].sum())
        for lst, m in ((diverged, d), (flipped, f), (unchecked, u)):
            lst += (torch.nonzero(m).flatten() + first).tolist()
        del a, c, pa, pc, d, rec, fl, f, u
    part = {}
    for name, ids in (("diverged", diverged), ("flipped", flipped), ("unchecked", unchecked)):
        acc = {t: torch.zeros(i64.size, dtype=torch.float64, device="cuda") for t in ("fp32", "fp64")}
        for pid in ids:
            for t, b in (("fp32", b32), ("fp64", b64)):
                img, _ = M.mc_render(s, b, transport=t, seed=seed, n_photons=1, photon_offset=pid, n_photons_norm=N,
                                     stats=False)
                acc[t] += img
        part[name] = {t: v.cpu().numpy() for t, v in acc.items()}
    total = np.abs(i32 - i64).sum()
    share = lambda k: float(np.abs(part[k]["fp32"] - part[k]["fp64"]).sum() / max(total, 1e-300))
    r32 = i32 - part["diverged"]["fp32"]
    r64 = i64 - part["diverged"]["fp64"]
    out = {"photons": N, "diverged_photons": len(diverged), "flipped_photons": len(flipped),
           "unchecked_photons": len(unchecked), "estimates_checked": n_est, "flipped_estimates": n_flip_est,
           "flips_per_estimate": n_flip_est / max(n_est, 1),
           "share_of_abs_diff": {k: share(k) for k in part},
           "without_diverged": _pixel_errors(np, r32, r64, sig)}
    for k in ("flipped", "unchecked"):
        r32 = r32 - part[k]["fp32"]
        r64 = r64 - part[k]["fp64"]
    out["without_diverged_flipped_unchecked"] = _pixel_errors(np, r32, r64, sig)
    return out


def forward_c1(M, np):
    """The 16^3 Gaussian blob (4 cameras of 32^2, 1e5 photons): the forward's
    events/s in each transport precision (FP64 is the workload's own); kernel
    times, the fastest of three after a warm-up."""
    from paper_1512_02110_amd import scenes
    s = scenes.config1()
    out = {"workload": f"c1: 16^3 blob, 4 cameras 32x32, {s.n_photons:.0e} photons"}
    for t in ("fp64", "mixed", "fp32"):
        b = M.beta_tensor(s, t)
        M.mc_render(s, b, transport=t, stats=False)
        best = None
        for _ in range(3):
            _, st = M.mc_render(s, b, transport=t)
            ms = st.timing["transport_ms"]
            best = ms if best is None or ms < best else best
        out[t] = {"kernel_ms": round(best, 4), "events_per_s": st["events"] / (best * 1e-3), "events": st["events"]}
    return out


def adjoint_c3(M, torch, np, stream, n_photons):
    """Forward + adjoint on the 16^3 Gaussian-blob workload: beta0 = 0.7 x
    smoothed truth, L2 loss against images of the truth (another seed);
    FP32 transport, FP64 and compensated-FP32 gradient tallies."""
    from paper_1512_02110_amd import scenes
    truth = scenes.config3_truth(n_photons=n_photons, seed=1)
    s = scenes.config3_initial(n_photons=n_photons, seed=0)
    meas, _ = M.mc_render(truth, M.beta_tensor(truth, "fp32"), stats=False)
    beta = M.beta_tensor(s, "fp32")

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    timed(lambda: M.mc_render(s, beta, stats=False))  # warm-up
    (img, _), t_fwd = timed(lambda: M.mc_render(s, beta, stats=False))
    dl = 2.0 * (img - meas)
    timed(lambda: M.mc_grad_beta(s, beta, dl, stats=False))  # warm-up
    (g64, _), t_adj = timed(lambda: M.mc_grad_beta(s, beta, dl, stats=False))
    (g32, _), t_adj32 = timed(lambda: M.mc_grad_beta(s, beta, dl, tally="kahan32", stats=False))
    # the adjoint on the events of an independent photon stream (seed 7)
    (gi, _), t_adji = timed(lambda: M.mc_grad_beta(s, beta, dl, seed=7, stats=False))
    a, b, c = g64.cpu().numpy(), g32.cpu().numpy(), gi.cpu().numpy()
    return {"workload": f"c3: 16^3 blob, 4 cameras 32x32, {n_photons:.0e} photons, FP32 transport",
            "fwd_ms": round(t_fwd, 3), "adj_ms_f64": round(t_adj, 3), "adj_ms_kahan32": round(t_adj32, 3),
            "fwd_plus_adj_over_fwd": round((t_fwd + t_adj) / t_fwd, 4),
            "kahan32_vs_f64_rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(a)),
            "kahan32_vs_f64_max_rel": float(np.max(np.abs(a - b)) / np.max(np.abs(a))),
            "adj_ms_independent_seed": round(t_adji, 3),
            "independent_seed_vs_same_seed_rel_l2": float(np.linalg.norm(c - a) / np.linalg.norm(a)),
            "independent_seed_cosine": float(np.dot(a, c) / (np.linalg.norm(a) * np.linalg.norm(c)))}


def full_size_replay(M, torch, np, stream, name, make, n_photons, what):
    """One large workload at its full photon count: the forward, and the
    gradient by photon replay (a render's rays at these counts, ~1e10-1e11
    records, do not fit in memory), one timed call each."""
    s = make(n_photons=n_photons)
    beta = M.beta_tensor(s, "fp32")

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)
    # warm-up (also gives the replay its rays-per-photon hint for this workload)
    img0, _ = M.mc_render(s, beta, n_photons=2_000_000, stats=False)
    dl0 = torch.as_tensor(np.random.default_rng(2).normal(size=img0.numel()), device=img0.device)
    M.mc_grad_beta(s, beta, dl0, n_photons=2_000_000, stats=False)
    print(f"[bench] {name} full: forward", flush=True)
    (img, st), t_fwd = timed(lambda: M.mc_render(s, beta))
    print(f"[bench] {name} full: forward {t_fwd:.0f} ms; gradient by replay", flush=True)
    (g, gst), t_adj = timed(lambda: M.mc_grad_beta(s, beta, dl0))
    print(f"[bench] {name} full: gradient {t_adj:.0f} ms", flush=True)
    del beta, img, g
    M.mc_release_memory()
    return {"workload": f"{what}, {n_photons:.1e} photons, FP32 transport + FP64 tallies; gradient by photon "
                        f"replay (no kept rays)",
            "fwd_ms": round(t_fwd, 1), "fwd_kernel_ms": round(st.timing["transport_ms"], 1),
            "events_per_s": st["events"] / (t_fwd * 1e-3), "events": st["events"], "le_jobs": st["le_jobs"],
            "adj_ms": round(t_adj, 1), "adj_replay_kernel_ms": round(gst.timing["transport_ms"], 1),
            "adj_bin_deposit_ms": round(gst.timing["tape_ms"], 1),
            "parts": "device time of the replay launches and of the binning and deposits, summed per part; "
                     "the two overlap (chunks on two streams), adj_ms is the wall time",
            "fwd_plus_adj_over_fwd": round((t_fwd + t_adj) / t_fwd, 4)}


def descent_c5(M, torch, np, n_photons=25_000_000, n_iter=3, n_outer_voxel=4):
    """A few iterations of both recovery loops on the 256x256x128 multi-cloud
    field with 36 cameras (paper_1512_02110_amd.descent): projected gradient
    descent with the local-estimation surrogate gradient (measured images: the
    truth rendered at photon seed 1), with where its largest gradient sits, and
    the voxelised model with conditioning Q_c = 1/count, 5 steps per photon
    pass (measured images: the voxelised model of the truth with camera noise).
    The 50-iteration runs at 2.5e8 photons per pass are
    `python -m paper_1512_02110_amd.descent [--model voxel]`."""
    from paper_1512_02110_amd import scenes
    from paper_1512_02110_amd.descent import mc_descent, mc_voxel_descent
    truth = scenes.config5(n_photons=n_photons)
    t64 = torch.as_tensor(truth.beta, dtype=torch.float64, device="cuda")
    meas, _ = M.mc_render(truth, M.beta_tensor(truth, "fp32"), seed=1, stats=False)
    b0 = torch.as_tensor(0.7 * scenes.smooth(truth.beta3d(), 1.0).reshape(-1), dtype=torch.float64, device="cuda")
    _, recs, delta = mc_descent(truth, b0, meas, n_iter, truth=t64)
    out = {"workload": f"c5 recovery loops: 256x256x128, 36 cameras 256x256, {n_photons:.1e} photons per render "
                       f"and per gradient (per photon pass), FP32 transport",
           "local_estimation": {
               "delta": delta, "iterations": [{k: r[k] for k in ("iter", "loss", "residual", "eps", "delta_mass",
                                                                "grad_max", "grad_max_voxel", "grad_p999",
                                                                "seconds")} for r in recs],
               "eps_after": recs[-1]["eps_after"], "delta_mass_after": recs[-1]["delta_mass_after"]}}
    del meas
    jt, _ = M.mc_voxel_scatter(truth, M.beta_tensor(truth, "fp32"), seed=99, stats=False)
    clean = M.mc_voxel_render(truth, t64, jt, 2)
    del jt
    normals = torch.as_tensor(np.random.default_rng(5).normal(size=clean.numel()), device="cuda")
    grey, scale = M.mc_camera_noise(clean, normals)
    _, vrecs, vdelta = mc_voxel_descent(truth, b0, grey / scale, n_outer_voxel, truth=t64)
    out["voxel_model_q_1_over_count"] = {
        "delta_last": vdelta, "eps_start": M.mc_recovery_error(b0, t64)[1],
        "iterations": [{k: r[k] for k in ("iter", "cost", "eps", "delta_mass", "delta", "halvings", "seconds")}
                       for r in vrecs]}
    return out


def gradient_statistics(M, torch, np, n_photons=100_000_000, parts=16, seeds=8):
    """Monte Carlo statistics of the surrogate gradient on the 16^3 adjoint
    workload (beta0 = 0.7 x smoothed truth; L2 loss against images of the
    truth at photon seed 1; FP32 transport): the gradient on the render's own
    photons (seed 0, the frozen-event derivative of the render) as the sum of
    `parts` disjoint photon ranges, whose spread gives per-voxel standard
    errors; gradients with the same image residual on `seeds` independent
    photon streams; the same-stream gradient with the residual of an
    independent render (seed 2) instead; and the voxelised model's gradient
    (Sec. 3) with the same residual."""
    from paper_1512_02110_amd import scenes
    truth = scenes.config3_truth(n_photons=n_photons, seed=1)
    s = scenes.config3_initial(n_photons=n_photons, seed=0)
    b32 = M.beta_tensor(s, "fp32")
    meas, _ = M.mc_render(truth, M.beta_tensor(truth, "fp32"), stats=False)
    i0, _ = M.mc_render(s, b32, stats=False)
    i1, _ = M.mc_render(s, b32, seed=2, stats=False)
    dl0, dl1 = 2.0 * (i0 - meas), 2.0 * (i1 - meas)
    n = n_photons // parts
    gp = [M.mc_grad_beta(s, b32, dl0, n_photons=n, photon_offset=k * n, n_photons_norm=n_photons, stats=False)[0]
          .cpu().numpy() for k in range(parts)]
    gp = np.array(gp)
    g_same = gp.sum(axis=0)
    se_same = np.sqrt(parts * gp.var(axis=0, ddof=1))
    gi = np.array([M.mc_grad_beta(s, b32, dl0, seed=100 + j, stats=False)[0].cpu().numpy() for j in range(seeds)])
    g_ind = gi.mean(axis=0)
    se_ind = gi.std(axis=0, ddof=1) / np.sqrt(seeds)
    g_x = M.mc_grad_beta(s, b32, dl1, stats=False)[0].cpu().numpy()  # seed-0 events, independent residual
    j, _ = M.mc_voxel_scatter(s, b32, seed=3, stats=False)
    g_vox = M.mc_voxel_grad(s, M.beta_tensor(s, "fp64"), j, dl0, 2).cpu().numpy()

    def cos(a, b):
        return float(np.dot(a, b) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))
    pair = [cos(gi[a], gi[b]) for a in range(seeds) for b in range(a + 1, seeds)]
    sig = np.abs(g_ind) > 3 * se_ind
    bias = g_same - g_ind
    iz = np.arange(s.n_vox) // (s.nx * s.ny)
    return {"workload": f"c3: 16^3 blob, 4 cameras 32x32 on the floor, {n_photons:.0e} photons, FP32 transport",
            "same_stream_vs_independent_mean_cosine": cos(g_same, g_ind),
            "independent_streams_pairwise_cosine_mean": float(np.mean(pair)),
            "independent_streams_pairwise_cosine_min": float(np.min(pair)),
            "same_stream_events_independent_residual_vs_independent_mean_cosine": cos(g_x, g_ind),
            "voxel_model_vs_independent_mean_cosine": cos(g_vox, g_ind),
            "median_snr_same_stream": float(np.median(np.abs(g_same) / np.maximum(se_same, 1e-300))),
            "median_snr_one_independent_stream": float(np.median(np.abs(g_ind) / np.maximum(se_ind * np.sqrt(seeds),
                                                                                          1e-300))),
            "frac_voxels_significant_independent_mean": float(sig.mean()),
            "frac_significant_voxels_sign_disagrees_same_stream": float((np.sign(g_same) != np.sign(g_ind))[sig].mean())
            if sig.any() else 0.0,
            "same_minus_independent_rel_l2": float(np.linalg.norm(bias) / max(np.linalg.norm(g_ind), 1e-300)),
            "same_minus_independent_in_sigmas_median": float(np.median(np.abs(bias) / np.maximum(
                np.sqrt(se_same ** 2 + se_ind ** 2), 1e-300))),
            "share_of_same_minus_independent_in_bottom_two_layers": float(
                np.abs(bias)[iz < 2].sum() / max(np.abs(bias).sum(), 1e-300)),
            "share_of_independent_gradient_in_bottom_two_layers": float(
                np.abs(g_ind)[iz < 2].sum() / max(np.abs(g_ind).sum(), 1e-300))}


def large_grids(M, torch, np, stream, n_photons):
    """The 128^3 cloud (25 cameras of 256^2) and the 256x256x128 multi-cloud
    field (36 cameras of 256^2), whose extinction copies (8 and 34 MB) sit in
    the MALL rather than in L2: the forward's events/s and voxel steps/s, and
    the render that keeps its rays plus the gradient from them against the
    plain render, at n_photons (their own photon counts, 1e9 and 2e9, take a
    minute and more per render); warm-up, then one timed call of each."""
    from paper_1512_02110_amd import scenes

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    out = {}
    for name, make, what in (("c4", scenes.config4, "128^3 cloud, 25 cameras 256x256"),
                             ("c5", scenes.config5, "256x256x128 multi-cloud field, 36 cameras 256x256")):
        s = make(n_photons=n_photons)
        beta = M.beta_tensor(s, "fp32")
        M.mc_render(s, beta, n_photons=min(n_photons, 1_000_000), stats=False)  # warm-up
        (img, st), t_fwd = timed(lambda: M.mc_render(s, beta))
        dl = torch.as_tensor(np.random.default_rng(2).normal(size=img.numel()), device=img.device)
        steps = st["vox_free"] + st["vox_conn"]
        r = {"workload": f"{name}: {what}, {n_photons:.0e} photons, FP32 transport + FP64 tallies",
             "fwd_ms": round(t_fwd, 3), "events_per_s": st["events"] / (t_fwd * 1e-3),
             "events": st["events"], "le_jobs": st["le_jobs"], "voxel_steps_per_s": steps / (t_fwd * 1e-3),
             "gather_GBps": 4.0 * steps / (t_fwd * 1e-3) / 1e9}
        # warm-up of the kept render: the first one of a workload allocates its ray buffer
        _, _, tape = M.mc_render_tape(s, beta, n_photons=min(n_photons, 1_000_000), stats=False)
        if tape is not None:
            tape.free()
        (_, _, tape), t_tape = timed(lambda: M.mc_render_tape(s, beta, stats=False))
        if tape is None:
            # a kept tape that overflowed (sized from an earlier kept render
            # of this workload with fewer rays per photon): the next kept
            # render is sized from this one's count
            (_, _, tape), t_tape = timed(lambda: M.mc_render_tape(s, beta, stats=False))
        if tape is not None:
            # the render's rays kept: render with rays + gradient from them
            _, t_adj = timed(lambda: M.mc_grad_beta(s, beta, dl, tape=tape, stats=False))
            tape.free()
            r.update({"adj_route": "kept rays", "fwd_tape_ms": round(t_tape, 3), "adj_ms": round(t_adj, 3),
                      "fwd_plus_adj_over_fwd": round((t_tape + t_adj) / t_fwd, 4)})
        else:
            # more rays than the tape holds: the gradient replays the photons
            _, t_adj = timed(lambda: M.mc_grad_beta(s, beta, dl, stats=False))
            r.update({"adj_route": "replay", "adj_ms": round(t_adj, 3),
                      "fwd_plus_adj_over_fwd": round((t_fwd + t_adj) / t_fwd, 4)})
        out[name] = r
        del tape, img, beta
        M.mc_release_memory()
    return out


def voxel_model(M, torch, np, stream, s, n_side=2):
    """The paper's voxelised forward model (Sec. 3) on the same workload: the
    scatter pass (photons without local estimates, j_c(k) per camera and
    voxel), the images from j (n x n rays per pixel) and the frozen-j
    gradient; warm-up, then one timed call of each."""
    b32, b64 = M.beta_tensor(s, "fp32"), M.beta_tensor(s, "fp64")

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    M.mc_voxel_scatter(s, b32, seed=7, stats=False)
    (j, st), t_sc = timed(lambda: M.mc_voxel_scatter(s, b32, seed=7, stats=True))
    M.mc_voxel_render(s, b64, j, n_side)
    img, t_r = timed(lambda: M.mc_voxel_render(s, b64, j, n_side))
    dl = torch.ones_like(img)
    M.mc_voxel_grad(s, b64, j, dl, n_side)
    _, t_g = timed(lambda: M.mc_voxel_grad(s, b64, j, dl, n_side))
    k_s = st.timing["transport_ms"] / 1e3
    return {"workload": f"same scene, {s.n_photons:.0e} photons, FP32 transport, {n_side}x{n_side} rays per pixel",
            "scatter_ms": round(t_sc, 3), "scatter_events_per_s": st["events"] / (t_sc / 1e3),
            "scatter_kernel_ms": round(st.timing["transport_ms"], 3),
            "voxel_camera_tallies": st["le_jobs"],
            "tally_atomics_per_s": st["le_jobs"] / k_s,
            "render_ms": round(t_r, 3), "grad_ms": round(t_g, 3)}


def bmc(M, torch, np, stream, s, n_per_pixel=64):
    """Backward Monte Carlo (Sec. 2.1.4) on the same scene: n_per_pixel
    packets per pixel, FP32 transport; warm-up, then one timed call."""
    b32 = M.beta_tensor(s, "fp32")
    M.mc_bmc_render(s, b32, 4, seed=3, stats=False)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    img, st = M.mc_bmc_render(s, b32, n_per_pixel, seed=3, stats=True)
    b.record(stream)
    torch.cuda.synchronize()
    t = a.elapsed_time(b)
    return {"workload": f"same scene, {n_per_pixel} packets per pixel ({st['photons']:.3e} packets), FP32 transport",
            "ms": round(t, 3), "kernel_ms": round(st.timing["transport_ms"], 3),
            "events_per_s": st["events"] / (t / 1e3), "events": st["events"],
            "vox_free_per_s": st["vox_free"] / (t / 1e3)}


# Air + aerosol channels (synthetic): Rayleigh extinction at the floor
# ~ lambda^-4 (650, 550, 450 nm; km^-1), an air scale height of 8 km, and
# aerosol cross-sections relative to green with an Angstrom exponent of 1.3.
RGB_AIR_KM = (0.0059, 0.0116, 0.0259)
RGB_SIGMA = (0.80, 1.0, 1.30)


def mixture(M, torch, np, stream, s, n_grad=10_000_000):
    """Air + aerosol mixture (step iv; Eqs. Pray, thetaREY, channelBeta) on the
    same grid and cameras: the cloud is the green aerosol field, air falls off
    with height; one RGB render (FP32 transport, the workload's photons per
    channel) and the full and surrogate gradients of one channel at n_grad
    photons; warm-up, then one timed call of each."""
    z = (np.arange(s.nz) + 0.5) * s.dz
    airs = [torch.as_tensor(np.ascontiguousarray(np.broadcast_to(
        (b * np.exp(-z / 8.0))[:, None, None], (s.nz, s.ny, s.nx)).reshape(-1)), dtype=torch.float64,
        device="cuda") for b in RGB_AIR_KM]
    aer = torch.as_tensor(s.beta, dtype=torch.float64, device="cuda")

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    M.mc_render_mixture(s, airs[1], aer, 1.0, n_photons=min(s.n_photons, 1_000_000), stats=False)
    rgb, t_rgb = timed(lambda: M.mc_render_rgb(s, airs, aer, RGB_SIGMA))
    events = sum(st["events"] for _, st in rgb)
    dl = torch.ones(M.n_pixels(s), dtype=torch.float64, device="cuda")
    out = {"workload": f"same grid and cameras, RGB: air {RGB_AIR_KM} km^-1 at the floor, aerosol ratios "
                       f"{RGB_SIGMA}; {s.n_photons:.0e} photons per channel, FP32 transport",
           "rgb_render_ms": round(t_rgb, 3), "events_per_s": events / (t_rgb / 1e3),
           "events": events}
    for full in (True, False):
        M.mc_grad_mixture(s, airs[1], aer, dl, 1.0, full=full, n_photons=n_grad // 10, stats=False)
        (g, st), t_g = timed(lambda: M.mc_grad_mixture(s, airs[1], aer, dl, 1.0, full=full, n_photons=n_grad))
        key = "grad_full" if full else "grad_surrogate"
        out[key + "_ms"] = round(t_g, 3)
        out[key + "_photons"] = n_grad
        out[key + "_events_per_s"] = st["events"] / (t_g / 1e3)
    return out


def recovery(M, torch, np, stream, s, n_photons=10_000_000, n_outer=40, n_gd=5, n_side=2):
    """The surrogate recovery loop (Secs. 5.2, 6, 7) on the same grid and
    cameras, with each reading of the conditioning Q_c of Sec. 6: 1/count
    (this build's reading), the count itself (the passage's wording taken
    literally) and none.  Measured images of the truth from the voxelised
    model (seed 99, Eq. (noise) grey levels with seeded read noise, back to
    radiance); start: a uniform field at the truth's mean extinction; no
    regulariser.  paper_1512_02110_amd.descent.mc_voxel_descent: step size
    from 5% of max beta over the largest first gradient, halved whenever an
    outer iteration's steps do not all lower its cost and grown by 1.25
    after one that needed no halving.  eps and delta_mass after every outer
    iteration (a photon pass for j, then n_gd steps), and the time per
    photon pass."""
    from paper_1512_02110_amd.descent import mc_voxel_descent
    truth = s.with_beta(s.beta)
    t32 = M.beta_tensor(truth, "fp32")
    t64 = M.beta_tensor(truth, "fp64")
    jt, _ = M.mc_voxel_scatter(truth.replace(n_photons=n_photons), t32, seed=99, stats=False)
    clean = M.mc_voxel_render(truth, t64, jt, n_side)
    normals = torch.as_tensor(np.random.default_rng(5).normal(size=clean.numel()), device="cuda")
    grey, scale = M.mc_camera_noise(clean, normals)
    meas = grey / scale
    s0 = truth.replace(n_photons=n_photons)
    b0t = torch.full((s.n_vox,), float(truth.beta.mean()), dtype=torch.float64, device="cuda")
    e0 = M.mc_recovery_error(b0t, t64)
    out = {"workload": f"same grid and cameras; {n_photons:.0e} photons per surrogate iteration, {n_outer} "
                       f"iterations x {n_gd} steps, {n_side}x{n_side} rays per pixel; start: uniform at the "
                       f"truth's mean extinction",
           "delta_mass_start": e0[0], "eps_start": e0[1], "readings": {}}
    for name, cond in (("q_1_over_count", 1), ("q_count", 2), ("none", 0)):
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _, recs, delta = mc_voxel_descent(s0, b0t, meas, n_outer, n_gd=n_gd, conditioned=cond, rays_per_side=n_side,
                                          truth=t64, grow=1.25)
        e.record(stream)
        torch.cuda.synchronize()
        eps = [e0[1]] + [r["eps"] for r in recs]
        out["readings"][name] = {"delta_last": delta, "halvings": [r["halvings"] for r in recs],
                                 "loop_ms": round(a.elapsed_time(e), 3), "eps": eps,
                                 "delta_mass": [e0[0]] + [r["delta_mass"] for r in recs],
                                 "cost_first": recs[0]["cost"][0], "cost_last": recs[-1]["cost"][-1],
                                 "eps_end_below_start": eps[-1] < eps[0]}
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    M.mc_voxel_scatter(s0, b0t.float(), seed=1000, stats=False)
    e.record(stream)
    torch.cuda.synchronize()
    out["photon_pass_ms"] = round(a.elapsed_time(e), 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--photons", type=int, default=None)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP32 / mixed / FP64 comparison")
    ap.add_argument("--no-precision-classes", action="store_true",
                    help="skip the per-photon classification of the FP32 differences")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-photons", type=int, default=1_100_000,
                    help="photons per CPU process (about 10 s of one core on the 64^3 workload)")
    ap.add_argument("--cpu-procs", type=int, default=None)
    ap.add_argument("--c3-photons", type=int, default=100_000_000)
    ap.add_argument("--no-voxel", action="store_true", help="skip the voxelised-model section")
    ap.add_argument("--no-large", action="store_true", help="skip the 128^3 and 256x256x128 section")
    ap.add_argument("--large-photons", type=int, default=20_000_000)
    ap.add_argument("--no-full-size", "--no-c4-full", dest="no_full_size", action="store_true",
                    help="skip the gradients by replay at full photon counts: the 256x256x128 workload at "
                         "its one-GPU share of 2.5e8 photons and the 128^3 workload at its own 1e9 (about three "
                         "minutes)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(photon ranges would shard with one FP64 all-reduce of the images; not built).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1512_02110_amd import scenes
    make = scenes.CONFIGS[args.config]
    s = make() if args.photons is None else make(n_photons=args.photons)

    cpu = None
    if not args.no_cpu_baseline:
        procs = args.cpu_procs or max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(args.config, args.cpu_photons, procs)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} events/s on {procs} processes", flush=True)

    import numpy as np
    import torch
    from paper_1512_02110_amd import mcrt as M

    assert torch.cuda.is_available(), "bench needs a GPU"
    M.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    beta32 = M.beta_tensor(s, "fp32")
    # a 'measured' image for the L2 loss: a different seed on a perturbed field
    meas, _ = M.mc_render(s, M.beta_tensor(s, "fp32", beta=s.beta * 0.9), seed=99,
                          n_photons=min(s.n_photons, 10_000_000))

    def step(seed):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        img, st = M.mc_render(s, beta32, seed=seed, stats=True)
        e1.record(stream)
        ast = None
        if not args.no_adjoint:
            img_t, _, tape = M.mc_render_tape(s, beta32, seed=seed, stats=False)
            e2.record(stream)
            dl = 2.0 * (img_t - meas)
            _, ast = M.mc_grad_beta(s, beta32, dl, seed=seed, stats=True, tape=tape)
            e3.record(stream)
            if tape is not None:
                tape.free()
            ast["kept_tape"] = tape is not None
        return img, st, ast, (e0, e1, e2, e3)

    for w in range(args.warmup):
        step(500 + w)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    recs = [step(1000 + k) for k in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    fwd_ms = [r[3][0].elapsed_time(r[3][1]) for r in recs]
    if not args.no_adjoint:
        fwd_tape_ms = [r[3][1].elapsed_time(r[3][2]) for r in recs]
        adj_ms = [r[3][2].elapsed_time(r[3][3]) for r in recs]
    events = sum(r[1]["events"] for r in recs)
    st = {k: sum(r[1][k] for r in recs) for k in recs[0][1]}
    fwd_s = sum(fwd_ms) / 1e3
    value = events / fwd_s

    # roofline of the transport kernel k_render (one launch per render),
    # timed by the library with HIP events on the launch stream; algorithmic
    # work from the launch's own counters: per voxel step (free flight or
    # connection ray) one 4-byte extinction read and 10 flops, per local
    # estimate a 16-byte FP64 tally and 60 flops, per event 150 flops.  The
    # kernel is bound by its memory side (the gathers: the vector-memory
    # address/data units are the busiest units, the VALU is not the limit),
    # so the memory roof is the one it is measured against; the grid itself
    # stays in L2, hence traffic (HBM bytes) well below the algorithmic bytes
    k_ms = [r[1].timing["transport_ms"] for r in recs]
    k_s = sum(k_ms) / 1e3
    steps = st["vox_free"] + st["vox_conn"]
    flops = 10.0 * steps + 60.0 * st["le_jobs"] + 150.0 * st["events"]
    gbytes = 4.0 * steps + 16.0 * st["le_jobs"]
    achieved_gbps = gbytes / k_s / 1e9
    traffic = measured_traffic()
    # the ceiling of the walk's gathers on its own address stream (a capture
    # of the render's loads replayed without the walk, micro.gather_ceiling)
    from paper_1512_02110_amd import micro
    ceil = micro.gather_ceiling(s, min(s.n_photons, 20_000_000))
    roofline = {"bound": "hbm", "achieved": round(achieved_gbps, 1), "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": round(achieved_gbps / PEAK_HBM_GBPS, 4),
                "achieved_is": "algorithmic bytes of the launch (4 B per voxel step read from the extinction grid, "
                               "16 B per FP64 image tally) per second of kernel time; the 1 MiB grid is served by "
                               "L1/L2, so this is not HBM traffic (that is `traffic`)",
                "traffic": traffic,
                "kernel": "k_render<float, MODE_RENDER, TALLY_F64>",
                "kernel_ms_avg": round(sum(k_ms) / len(k_ms), 3),
                "algorithmic_bytes_per_launch": gbytes / len(recs),
                "binding_unit": "VALU issue (95% of one wave64 instruction per CU cycle, with the gather "
                                "pipeline's address and data units 88% / 98% busy; on the 128^3 and "
                                "256x256x128 grids the gathers bind: profiles/k_render_fwd_c2_counters.md, "
                                "profiles/k_render_fwd_c4_c5_counters.md)",
                "gather_ceiling": {
                    "what": "loads/s of the render's own connection-walk loads (captured per wavefront and lane) "
                            "replayed through the same buffer with no walk arithmetic, same wavefronts per CU",
                    "ceiling_gloads_per_s": round(ceil["replay_gloads_per_s"], 1),
                    "render_issued_gloads_per_s": round(ceil["render_issued_gloads_per_s"], 1),
                    "frac_issued": round(ceil["frac_issued_of_replay"], 4),
                    "render_algorithmic_gloads_per_s": round(ceil["render_algorithmic_gloads_per_s"], 1),
                    "frac_algorithmic": round(ceil["frac_algorithmic_of_replay"], 4),
                    "target_frac": 0.5, "met": ceil["frac_algorithmic_of_replay"] >= 0.5,
                    "photons": ceil["photons"], "working_set_bytes": ceil["working_set_bytes"]},
                "alu_tflops": round(flops / k_s / 1e12, 3),
                "alu_frac_of_fp32_peak": round(flops / k_s / 1e12 / PEAK_FP32_TFLOPS, 4),
                "voxel_steps_per_s": steps / k_s}

    out = {
        "metric": "scattering events/s fwd; fwd+adjoint time vs fwd, FP32 vs FP64 at <=1e-4 error",
        "value": value,
        "unit": "scattering events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {s.nx}x{s.ny}x{s.nz} voxels of {s.dx} km, "
                               f"{s.n_cams} cameras {s.cameras[0].width}x{s.cameras[0].height}, "
                               f"{s.n_photons:.0e} photons/render, FP32 transport + FP64 tallies",
                   "photons": s.n_photons, "n_cams": s.n_cams,
                   "max_column_tau": round(float((s.beta3d() * s.dz).sum(axis=0).max()), 2)},
        "fwd_ms": round(sum(fwd_ms) / len(fwd_ms), 3),
        "events_per_render": events // args.steps,
        "stats_per_render": {k: v // args.steps for k, v in st.items()},
        "roofline": roofline,
    }
    if not args.no_adjoint:
        # reverse mode with the kept tape (the optimisation step)
        out["fwd_tape_ms"] = round(sum(fwd_tape_ms) / len(fwd_tape_ms), 3)
        out["adj_ms"] = round(sum(adj_ms) / len(adj_ms), 3)
        out["adj_bin_deposit_ms"] = round(sum(r[2].timing["tape_ms"] for r in recs) / len(recs), 3)
        out["adj_used_kept_tape"] = all(r[2]["kept_tape"] for r in recs)
        out["fwd_plus_adj_over_fwd"] = round((sum(fwd_tape_ms) + sum(adj_ms)) / sum(fwd_ms), 4)
        # the gradient by photon replay (no tape), once, after the steps
        dl = 2.0 * (recs[0][0] - meas)
        M.mc_grad_beta(s, beta32, dl, seed=1000, stats=False)  # warm-up
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        _, rst = M.mc_grad_beta(s, beta32, dl, seed=1000, stats=True)
        r1.record(stream)
        torch.cuda.synchronize()
        t_rep = r0.elapsed_time(r1)
        out["adj_by_replay"] = {"adj_ms": round(t_rep, 3),
                                "replay_ms": round(rst.timing["transport_ms"], 3),
                                "bin_deposit_ms": round(rst.timing["tape_ms"], 3),
                                "parts_overlap": True,
                                "fwd_plus_adj_over_fwd": round((fwd_ms[0] + t_rep) / fwd_ms[0], 4)}

    if not args.no_fp64:
        out["precision"] = precisions(M, torch, np, s, classes=not args.no_precision_classes)
        print(f"[bench] precisions: {json.dumps(out['precision'])}", flush=True)
        # the metric's "FP32 vs FP64 at <= 1e-4 error": each reduced-precision
        # render of the same photons against the FP64 one, pixel by pixel
        pr = out["precision"]
        out["vs_fp64_at_1e-4"] = {
            name: {"kernel_ms": pr[name]["kernel_ms"], "events_per_s": pr[name]["events_per_s"],
                   "speedup_over_fp64": pr[name]["speedup_over_fp64"],
                   "frac_pixels_within_1e-4_rel": pr[name]["frac_pixels_within_1e-4_rel"],
                   "frac_pixels_within_max_1e-4_rel_3sigma": pr[name]["frac_pixels_within_max_1e-4_rel_3sigma"],
                   "counters_equal_fp64": pr[name]["counters_equal_fp64"]}
            for name in ("fp32", "mixed")}
    if args.config == "c2":
        out["forward_c1"] = forward_c1(M, np)
    if not args.no_adjoint and args.config == "c2":
        out["fwd_adjoint_c3"] = adjoint_c3(M, torch, np, stream, args.c3_photons)
        out["gradient_statistics_c3"] = gradient_statistics(M, torch, np, args.c3_photons)
        print(f"[bench] gradient statistics: {json.dumps(out['gradient_statistics_c3'])}", flush=True)
    if not args.no_large and not args.no_adjoint and args.config == "c2":
        out["large_grids"] = large_grids(M, torch, np, stream, args.large_photons)
        from paper_1512_02110_amd import micro
        out["large_grids"]["gather_ceiling"] = {
            name: micro.gather_ceiling(make(), n)
            for name, make, n in (("c4", scenes.config4, 4_000_000), ("c5", scenes.config5, 10_000_000))}
        out["recovery_c5"] = descent_c5(M, torch, np)
        print(f"[bench] c5 descent: {json.dumps(out['recovery_c5'])}", flush=True)
        if not args.no_full_size:
            out["large_grids"]["c5_share"] = full_size_replay(
                M, torch, np, stream, "c5", scenes.config5, 250_000_000,
                "c5: 256x256x128 multi-cloud field, 36 cameras 256x256, its one-GPU share of 2e9 photons")
            out["large_grids"]["c4_full"] = full_size_replay(
                M, torch, np, stream, "c4", scenes.config4, 1_000_000_000, "c4: 128^3 cloud, 25 cameras 256x256")
    if not args.no_voxel:
        out["voxel_model"] = voxel_model(M, torch, np, stream, s)
        out["recovery"] = recovery(M, torch, np, stream, s)
        out["bmc"] = bmc(M, torch, np, stream, s)
        out["mixture"] = mixture(M, torch, np, stream, s)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
