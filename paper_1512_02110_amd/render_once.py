"""Renders one of the benchmark workloads a few times and prints the
kernel time of each render: a fixed, small command for profilers (counter
runs want a program whose transport dispatches are exactly the renders).

    python -m paper_1512_02110_amd.render_once --config c4 --photons 4000000 [--transport fp32] [--repeat 1]
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
        _, st = M.mc_render(s, beta, transport=args.transport, seed=1000 + i)
        print(json.dumps({"config": args.config, "photons": s.n_photons, "transport": args.transport,
                          "kernel_ms": st.timing["transport_ms"], "events": st["events"],
                          "voxel_steps": st["vox_free"] + st["vox_conn"], "le_jobs": st["le_jobs"]}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
