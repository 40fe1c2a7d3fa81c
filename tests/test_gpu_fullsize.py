"""The benchmark workloads at full size, in the configuration bench.py times
(kernel k-means++ seeding on the GPU, the workload's window and batch, the
benchmark's precision forms), against the FP64 oracle on sampled rows.

After W + 1 steps (the steady-state support of W full batches), the GPU's
state is exported (mbkk_get_state) and loaded into the oracle as explicit
centers; one more GPU step then runs in the benchmark's launch configuration
(b rows), and its labels and minimum distances on every row of that batch are
compared with the oracle's assignment of the same rows on the same state:
labels identical on every row whose margin exceeds the form's threshold, at
least 99.9 % agreement over all rows, and the distance error within the
form's tolerance (the floored plain relative error is reported beside it).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import workloads as W
from tests._parity import agreement, dist_rel_err, dist_rel_err_floor, oracle_from_gpu_state

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-2}
MARGIN = {"fp32": 1e-4, "bf16x3": 1e-4}
KNAME = {W.GAUSS: "gauss", W.LAPLACE: "laplace"}


@pytest.mark.parametrize("name,precision", [("c3", "bf16x3"), ("c3", "fp32"), ("c5", "fp32"),
                                            ("c2", "bf16x3"), ("c2", "fp32")])
def test_full_size_step_against_oracle(name, precision):
    from paper_2410_05902_amd import Model
    wl = W.make(name)
    X = torch.from_numpy(wl.X).cuda()
    model = Model(X, k=wl.k, b_max=wl.b, window=wl.window, kernel=KNAME[wl.kernel],
                  kernel_param=wl.kernel_param, precision=precision, validate=False)
    model.init_kmeanspp(wl.kmeanspp_uniforms())
    for i in range(1, wl.window + 2):
        model.step_noout(torch.from_numpy(wl.batch(i)).cuda())
    st = model.get_state()
    orc = O.Oracle(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param)
    m_sup = oracle_from_gpu_state(orc, st, wl.k, wl.window)
    # the live terms of the steady state: at most W full batches and the initial
    # points (terms whose coefficient the learning rate has taken to 0 drop out)
    assert wl.b <= m_sup <= wl.window * wl.b + wl.k
    B = wl.batch(wl.window + 2)
    out = model.step(torch.from_numpy(B).cuda())
    ref = orc.distances(B, threads=16, want_D=False)
    lab = out["labels"].cpu().numpy()
    mind = out["mind"].cpu().numpy().astype(np.float64)
    ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
    assert ag["on_margin"], f"labels differ on rows with margin: {ag['mismatches'][:8]}"
    assert ag["all"] >= 0.999, f"agreement {ag['all']:.5f} over all {wl.b} rows"
    same = lab == ref["labels"]
    scale = 1.0 + ref["N"][ref["labels"]]  # K(x, x) = 1 for the Gaussian and Laplacian kernels
    err = dist_rel_err(mind[same], ref["mind"][same], scale[same])
    errf = dist_rel_err_floor(mind[same], ref["mind"][same], scale[same])
    print(f"[full size {wl.name} {precision}] {wl.b} rows: agreement {ag['all']:.6f}, "
          f"distance error {err.max():.3e} (floored {errf.max():.3e}), "
          f"{ag['n_margin']} rows with margin >= {MARGIN[precision]}", flush=True)
    assert err.max() <= TOL[precision], f"min-distance error {err.max():.3e}"
