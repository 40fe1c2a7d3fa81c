"""The quality comparison of Section 6 (learning rates, truncation) through
the harness, against the same comparison run on the FP64 oracle: the
trajectories take identical labels, so the adjusted Rand index and the NMI of
the final assignment against the generating components must match the
oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from oracle import scores
from paper_2410_05902_amd import workloads as W
from tests._parity import agreement

pytestmark = pytest.mark.gpu

LR = {"beta": W.LR_BETA, "sklearn": W.LR_SKLEARN}


def _oracle_run(wl, lr, window, iterations):
    init = O.kmeanspp(wl.X, wl.kernel, wl.kernel_param, wl.k, wl.kmeanspp_uniforms())
    orc = O.Oracle(wl.X, wl.k, window, wl.kernel, wl.kernel_param, LR[lr])
    orc.init_centers(init)
    for i in range(1, iterations + 1):
        orc.step(wl.batch(i), threads=4, want_D=False)
    ref = orc.distances(np.arange(wl.n, dtype=np.int32), threads=4, want_D=False)
    return ref


@pytest.mark.parametrize("lr", ["beta", "sklearn"])
@pytest.mark.parametrize("window", [4, 0])
def test_quality_harness_matches_oracle(lr, window):
    from paper_2410_05902_amd.quality import run_config
    wl = W.c1_blobs(seed=0)
    X = torch.from_numpy(wl.X).cuda()
    got = run_config(wl, X, lr, window, "fp32", 20)
    ref = _oracle_run(wl, lr, window, 20)
    c = int(wl.comp.max()) + 1
    n = scores.contingency(ref["labels"], wl.comp, wl.k, c)
    assert got["iterations"] == 20 and got["window"] == window
    assert got["ari"] == pytest.approx(scores.ari(n), abs=2e-3)
    assert got["nmi"] == pytest.approx(scores.nmi(n), abs=2e-3)
    assert got["objective_all"] == pytest.approx(ref["mind"].mean(), rel=1e-4)
    assert 0.0 < got["ari"] <= 1.0 and 0.0 < got["nmi"] <= 1.0


def test_compare_lists_every_configuration():
    from paper_2410_05902_amd.quality import compare
    wl = W.c1_blobs(seed=1)
    rows = compare(wl, 5, lrs=("beta", "sklearn"), windows=(2, 0), precisions=("fp32", "bf16x3"))
    keys = {(r["lr"], r["window"], r["precision"]) for r in rows}
    # every rate, window and form: the table form (window 0) has FP32 and BF16X3 too
    assert keys == {(lr, w, p) for lr in ("beta", "sklearn") for w in (2, 0) for p in ("fp32", "bf16x3")}
