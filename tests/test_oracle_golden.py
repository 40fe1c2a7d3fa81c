"""Stored values: the paper's gamma table, and the oracle's own locked C1
trajectory (written by tests/golden/make_golden.py, which calls only oracle/)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2410_05902_amd import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_paper_gamma_table_gaussian_rows():
    """Appendix C table: gamma = max ||phi(x)|| = 1 for the Gaussian kernel on
    every dataset.  Checked on synthetic rows of each dataset's shape."""
    shapes = {"pendigits": 16, "har": 561, "mnist_784": 784, "letter": 16}
    rows = [l.split() for l in open(os.path.join(GOLD, "paper_gamma_table.txt"))
            if l.strip() and not l.startswith("#")]
    gauss = {r[0]: float(r[2]) for r in rows if r[1] == "gaussian"}
    assert set(gauss) == set(shapes)
    rng = np.random.default_rng(0)
    for name, d in shapes.items():
        X = rng.uniform(0, 1, size=(20, d))
        gamma = max(np.sqrt(O.kernel(O.GAUSS, 3.0, x, x)) for x in X)
        assert gamma == pytest.approx(gauss[name], abs=5e-4)


def test_c1_trajectory_locked():
    ref = json.load(open(os.path.join(GOLD, "c1_oracle_trajectory.json")))
    wl = W.c1_blobs(seed=0)
    assert ref["workload"] == wl.name
    init = O.kmeanspp(wl.X, wl.kernel, wl.kernel_param, wl.k, wl.kmeanspp_uniforms())
    assert init.tolist() == ref["init"]
    orc = O.Oracle(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param, wl.lr)
    orc.init_centers(init)
    for s in ref["steps"]:
        out = orc.step(wl.batch(s["i"]), want_D=False)
        assert out["counts"].tolist() == s["counts"]
        assert out["labels"][:32].tolist() == s["labels_head"]
        assert out["fbefore"] == pytest.approx(s["fbefore"], rel=1e-12)
    assert orc.objective(np.arange(wl.n, dtype=np.int32)) == pytest.approx(
        ref["final_objective_all"], rel=1e-12)
