"""Renders one of the benchmark workloads a few times and prints the
kernel time of each render: a fixed, small command for profilers (counter
runs want a program whose transport dispatches are exactly the renders).
With --grad each render keeps its rays and is followed by the surrogate
gradient from them (binning and deposits only, no replay), for a seeded
normal dL/di.

    python -m paper_1512_02110_amd.render_once --config c4 --photons 4000000 [--transport fp32] [--repeat 1] [--grad]
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--photons", type=int, default=None)
    ap.add_argument("--transport", default="fp32", choices=("fp32", "fp64", "mixed"))
    ap.add_argument("--repeat", type=int, default=1)
    ap.add_argument("--grad", action="store_true")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("render_once needs a GPU")
    from paper_1512_02110_amd import mcrt as M
    from paper_1512_02110_amd import scenes
    M.load_library()
    make = scenes.CONFIGS[args.config]
    s = make() if args.photons is None else make(n_photons=args.photons)
    beta = M.beta_tensor(s, args.transport)
    for i in range(args.repeat):
        if not args.grad:
            _, st = M.mc_render(s, beta, transport=args.transport, seed=1000 + i)
            print(json.dumps({"config": args.config, "photons": s.n_photons, "transport": args.transport,
                              "kernel_ms": st.timing["transport_ms"], "events": st["events"],
                              "voxel_steps": st["vox_free"] + st["vox_conn"], "le_jobs": st["le_jobs"]}),
                  flush=True)
            continue
        img, _, tape = M.mc_render_tape(s, beta, transport=args.transport, seed=1000 + i, stats=False)
        gen = torch.Generator(device="cpu").manual_seed(2 + i)
        dl = torch.randn(img.shape, generator=gen, dtype=torch.float64).to(img.device)
        _, st = M.mc_grad_beta(s, beta, dl, transport=args.transport, seed=1000 + i, tape=tape)
        torch.cuda.synchronize()
        if tape is not None:
            tape.free()
        print(json.dumps({"config": args.config, "photons": s.n_photons, "transport": args.transport,
                          "kept_rays": tape is not None, "grad_ms": st.timing["tape_ms"]}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
