"""Writes tests/golden/c1_oracle_trajectory.json from the FP64 oracle only.

The file locks the oracle's trajectory on the 2-D three-blob workload
(n=2000, k=3, b=256, Gaussian sigma=1, last 4 batches, kernel k-means++
seeding, 20 iterations, seed 0) so that an unintended change to the oracle's
arithmetic shows up as a test failure.  Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2410_05902_amd import workloads as W  # noqa: E402


def trajectory():
    wl = W.c1_blobs(seed=0)
    init = O.kmeanspp(wl.X, wl.kernel, wl.kernel_param, wl.k, wl.kmeanspp_uniforms())
    orc = O.Oracle(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param, wl.lr)
    orc.init_centers(init)
    steps = []
    for i in range(1, wl.iterations + 1):
        out = orc.step(wl.batch(i), want_D=False)
        steps.append(dict(i=i, counts=out["counts"].tolist(), fbefore=out["fbefore"],
                          labels_head=out["labels"][:32].tolist(),
                          min_margin=float(out["margin"].min())))
    import numpy as np
    fX = orc.objective(np.arange(wl.n, dtype=np.int32))
    return dict(workload=wl.name, init=init.tolist(), steps=steps, final_objective_all=fX)


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_oracle_trajectory.json"), "w") as f:
        json.dump(trajectory(), f, indent=1)
