"""Writes tests/golden/oracle_regression.json by calling only the oracle.

The paper prints no worked numeric example for forward Monte Carlo with local
estimation (Sec. 2.1.2-2.1.3), so the stored values here are the oracle's own
outputs on small seeded inputs.  They freeze the oracle: any later change of
its arithmetic changes them, and the commit that regenerates this file must
name the passage of the paper (or the reading of it) that justifies it.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1512_02110_amd import scenes  # noqa: E402

CASES = {
    "c1_2000": dict(scene=("config1", 2000, 0), kw={}),
    "c2_300": dict(scene=("config2", 300, 0), kw={}),
    "c1_single_order_seed5": dict(scene=("config1", 1500, 5), kw={"max_events": 1}),
}


def make_scene(name, n, seed):
    return getattr(scenes, name)(n_photons=n, seed=seed)


def run_case(case):
    name, n, seed = case["scene"]
    s = make_scene(name, n, seed)
    img, st = O.render(s, **case["kw"])
    rng = np.random.default_rng(17)
    g = rng.normal(size=img.size)
    grad, _ = O.grad_beta(s, g, **case["kw"])
    top = np.argsort(-img)[:12]
    gtop = np.argsort(-np.abs(grad))[:12]
    return {
        "stats": st,
        "image_sum": float(img.sum()),
        "image_top": [[int(i), float(img[i])] for i in top],
        "grad_dot_beta": float(grad @ s.beta),
        "grad_top": [[int(i), float(grad[i])] for i in gtop],
    }


def main():
    out = {"note": "oracle outputs on seeded synthetic inputs; see make_golden.py",
           "cases": {k: {"input": v, "output": run_case(v)} for k, v in CASES.items()}}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
