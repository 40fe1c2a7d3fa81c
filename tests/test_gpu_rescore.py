"""FP64 re-scoring of near ties in the BF16 forms, against the FP64 oracle.

The assignment step of Algorithm 2 takes the argmin of the distances; Section 5
leaves ties to an arbitrary choice, and both sides here take the lowest center
index.  In the BF16 forms a row whose two best approximate distances are
closer than the form's error bound gets the cross term of every candidate
center recomputed in FP64, so its distances then carry only the error of the
self norms N_j (FP32 kernel values summed in FP64), whose bound the library
reports.  The tests require:
  - every row re-scored (tie_delta above any distance spread): the FP64
    distances of every (row, center) within eN of the oracle's, and the
    oracle's label on every row whose exact margin exceeds 2 eN;
  - near ties made from duplicated and near-duplicated initial points, at the
    library's own bound: a positive count of re-scored rows, the lowest index
    on exact ties, and the oracle's label wherever the margin exceeds 2 eN;
  - lock-step iterations of the 128-D mixture: the oracle's label on every row
    whose margin exceeds 2 eN (the rows between 2 eN and the BF16 bound are
    decided only by the re-scoring).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import workloads as W
from tests._parity import dist_rel_err, dist_rel_err_floor, oracle_state_to_gpu

pytestmark = pytest.mark.gpu


def _mixture(seed=3, n=16384, d=128, c=16, std=0.3):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((c, d))
    comp = rng.integers(0, c, n)
    X = (means[comp] + std * rng.standard_normal((n, d))).astype(np.float32)
    sigma = W.median_pairwise_distance(X, seed)
    return X, comp, 2.0 * sigma * sigma


def _model(X, k, b_max, window, kappa, precision="bf16x3", tie=0.0):
    from paper_2410_05902_amd import Model
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    return Model(Xd, k=k, b_max=b_max, window=window, kernel="gauss", kernel_param=kappa,
                 precision=precision, tie_delta=tie)


def _init(comp, k, seed=4):
    rng = np.random.default_rng(seed)
    return np.array([rng.choice(np.flatnonzero(comp == j)) for j in range(k)], np.int32)


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x1"])
def test_every_row_rescored(precision):
    """tie_delta = 10 exceeds every distance spread (0 <= D <= 4), so every
    row is re-scored against every center: all distances are FP64 up to the
    self norms' error, in both BF16 forms."""
    X, comp, kappa = _mixture()
    k, b, win = 16, 1024, 3
    init = _init(comp, k)
    orc = O.Oracle(X, k, win, O.GAUSS, kappa)
    orc.init_centers(init)
    model = _model(X, k, b, win, kappa, precision, tie=10.0)
    model.init_centers(init)
    eN = model.selfnorm_error_bound()
    assert 0.0 < eN < 1e-4
    model.rescore_count(reset=True)
    for i in range(1, 7):
        B = W.batch_indices(11, i, X.shape[0], b)
        model.set_state(oracle_state_to_gpu(orc.state(), init, k, win, b))
        a = model.assign(B, want_D=True)
        assert model.rescore_count(reset=True) == b, f"step {i}: not every row was re-scored"
        ref = orc.step(B, threads=8)
        D = a["D"].cpu().numpy()
        # every entry is a re-scored FP64 distance: only N_j's error is left
        err = np.abs(D - ref["D"]).max()
        assert err <= eN + 1e-12, f"step {i}: re-scored distance error {err:.3e} > eN {eN:.3e}"
        lab = a["labels"].cpu().numpy()
        sel = ref["margin"] > 2.0 * eN
        bad = np.flatnonzero((lab != ref["labels"]) & sel)
        assert bad.size == 0, f"step {i}: labels differ on rows with margin > 2 eN: {bad[:8]}"
        mind = a["mind"].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(mind, ref["mind"], rtol=2.0 ** -23, atol=eN + 1e-12)
        print(f"[rescore all {precision}] step {i}: max |dD| {err:.2e} (eN {eN:.2e}), "
              f"{int((~sel).sum())} rows within 2 eN", flush=True)


def _near_tie_data():
    """The 128-D mixture with three extra rows: an exact copy of a point p of
    component 0 and two copies moved by eps along random unit directions."""
    X, comp, kappa = _mixture(seed=5)
    rng = np.random.default_rng(6)
    p = int(np.flatnonzero(comp == 0)[0])
    extra = [X[p].astype(np.float64)]
    for eps in (0.02, 0.05):
        u = rng.standard_normal(X.shape[1])
        extra.append(X[p] + eps * u / np.linalg.norm(u))
    X2 = np.ascontiguousarray(np.vstack([X, np.asarray(extra, np.float32)]))
    n = X.shape[0]
    # centers 0..3: p, its exact copy, the two near copies; 4..15: one point
    # of each other component
    init = np.concatenate([[p, n, n + 1, n + 2], _init(comp, 16, seed=7)[4:]]).astype(np.int32)
    return X2, np.concatenate([comp, [0, 0, 0]]), kappa, init


def test_near_ties_from_duplicate_centers():
    X, comp, kappa, init = _near_tie_data()
    k, b, win = 16, 2048, 3
    orc = O.Oracle(X, k, win, O.GAUSS, kappa)
    orc.init_centers(init)
    model = _model(X, k, b, win, kappa)
    model.init_centers(init)
    eN = model.selfnorm_error_bound()
    # rows of component 0 (their best centers are the four copies of p)
    rows = np.flatnonzero(comp == 0)[:b].astype(np.int32)
    model.rescore_count(reset=True)
    a = model.assign(rows, want_D=True)
    nres = model.rescore_count(reset=True)
    ref = orc.distances(rows, threads=8)
    lab = a["labels"].cpu().numpy()
    assert nres > 0, "no row was re-scored"
    # the exact copies tie exactly: the lowest index on every such row
    tie_rows = np.isin(ref["labels"], [0, 1])
    assert tie_rows.any()
    assert (ref["margin"][tie_rows] == 0.0).all()
    np.testing.assert_array_equal(lab[tie_rows], ref["labels"][tie_rows])
    # everywhere else the oracle's label wherever the margin exceeds 2 eN
    sel = ref["margin"] > 2.0 * eN
    bad = np.flatnonzero((lab != ref["labels"]) & sel)
    assert bad.size == 0, f"labels differ on rows with margin > 2 eN: {bad[:8]}"
    # the near copies decide rows whose margins lie between 2 eN and the BF16
    # bound: these are the rows that only the re-scoring gets right
    between = (ref["margin"] > 2.0 * eN) & (ref["margin"] < 1e-4)
    assert between.sum() > 0
    print(f"[near ties] {nres} rows re-scored of {rows.size}; {int(tie_rows.sum())} exact ties, "
          f"{int(between.sum())} rows with 2 eN < margin < 1e-4", flush=True)
    # the iteration scores the same way: a step on these rows gives the same labels
    model.rescore_count(reset=True)
    g = model.step(rows)
    assert model.rescore_count() == nres
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), lab)


@pytest.mark.parametrize("precision", ["bf16x3"])
def test_lockstep_labels_beyond_the_selfnorm_bound(precision):
    """The 128-D mixture in lock-step at its own bound: every row with an
    exact margin above 2 eN carries the oracle's label, far below the BF16
    product's own error (about 1e-4 here)."""
    wl = W.c3_gaussian_mixture(n=60000, c=40)
    k, b, win = 40, 2048, 4
    init = wl.random_init()[:k]
    orc = O.Oracle(wl.X, k, win, wl.kernel, wl.kernel_param)
    orc.init_centers(init)
    model = _model(wl.X, k, b, win, wl.kernel_param, precision)
    model.init_centers(init)
    eN = model.selfnorm_error_bound()
    total = 0
    for i in range(1, 8):
        B = wl.batch(i, b)
        model.set_state(oracle_state_to_gpu(orc.state(), init, k, win, b))
        model.rescore_count(reset=True)
        a = model.assign(B, want_D=True)
        nres = model.rescore_count()
        total += nres
        ref = orc.step(B, threads=8)
        lab = a["labels"].cpu().numpy()
        sel = ref["margin"] > 2.0 * eN
        bad = np.flatnonzero((lab != ref["labels"]) & sel)
        assert bad.size == 0, f"step {i}: labels differ on rows with margin > 2 eN: {bad[:8]}"
        scale = 1.0 + ref["N"][None, :]
        D = a["D"].cpu().numpy()
        e = dist_rel_err(D, ref["D"], scale).max()
        ef = dist_rel_err_floor(D, ref["D"], scale).max()  # reported
        assert e <= 1e-2
        print(f"[lockstep {precision}] step {i}: {nres} rows re-scored, error {e:.2e} "
              f"(floored {ef:.2e}), agreement {(lab == ref['labels']).mean():.6f}", flush=True)
