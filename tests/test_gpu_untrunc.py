"""Untruncated mini-batch kernel k-means (Algorithm 1, window 0) on the table
of cross terms of Appendix A, against the FP64 oracle run with no window.

The oracle keeps every center as an explicit combination of all the points
it has absorbed and evaluates distances from that combination; the GPU keeps
only <phi(x), C_j> for every x and <C_j, C_j>, updated by the recursion of
Section 4.  Free-running: the same initial centers and batches on both sides,
no state import (the table form has no state image).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import workloads as W
from tests._parity import agreement, dist_rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-5, "bf16x3": 1e-2}
MARGIN = {"fp64": 1e-9, "fp32": 1e-4, "bf16x3": 1e-4}
KNAME = {O.GAUSS: "gauss", O.LAPLACE: "laplace", O.LINEAR: "linear", O.POLY2: "poly2"}
LRNAME = {W.LR_BETA: "beta", W.LR_FULL: "full", W.LR_SKLEARN: "sklearn"}


def _model(X, k, b_max, kind, param, precision, lr=W.LR_BETA, impl="auto"):
    from paper_2410_05902_amd import Model
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    return Model(Xd, k=k, b_max=b_max, window=0, kernel=KNAME[kind], kernel_param=param,
                 precision=precision, lr=LRNAME[lr], cross_impl=impl)


def _kxx(X, kind, param):
    if kind in (O.GAUSS, O.LAPLACE):
        return np.ones(X.shape[0])
    sq = (X.astype(np.float64) ** 2).sum(1)
    return sq if kind == O.LINEAR else (sq + param) ** 2


def run_untrunc(X, k, kind, param, init, batches, precision, lr=W.LR_BETA, check_all=True, threads=4,
                impl="auto"):
    """Steps both sides; per step the labels agree on rows with margin and the
    minimum distances agree; while every label agrees, the distances of every
    point of X to every center and the self norms agree.  Returns the number
    of steps with identical labels."""
    orc = O.Oracle(X, k, 0, kind, param, lr)
    orc.init_centers(init)
    model = _model(X, k, max(len(B) for B in batches), kind, param, precision, lr, impl)
    model.init_centers(init)
    tol = TOL[precision]
    kxx = _kxx(X, kind, param)
    same = 0
    for B in batches:
        ref = orc.step(B, threads=threads)
        g = model.step(B, want_objective=True)
        lab = g["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
        assert ag["on_margin"], f"step {same + 1}: {ag['mismatches'][:8]}"
        if not (lab == ref["labels"]).all():
            return same
        scale = kxx[B] + ref["N"][ref["labels"]]
        e = dist_rel_err(g["mind"].cpu().numpy().astype(np.float64), ref["mind"], scale)
        assert e.max() <= max(tol, 2e-7), f"step {same + 1}: min-distance error {e.max():.3e}"
        # the mean of the minimum distances, each within tol of its scale
        assert abs(g["fbefore"] - ref["fbefore"]) <= max(tol, 2e-7) * scale.mean()
        same += 1
    N = orc.norms()
    np.testing.assert_allclose(model.center_norms(), N, rtol=max(tol, 1e-12), atol=1e-12 + tol * 1e-3)
    if check_all:
        allidx = np.arange(X.shape[0], dtype=np.int32)
        ref = orc.distances(allidx, threads=threads)
        a = model.assign(allidx, want_D=True)
        D = a["D"].cpu().numpy()
        err = dist_rel_err(D, ref["D"], kxx[:, None] + N[None, :])
        assert err.max() <= tol, f"table distances: error {err.max():.3e}"
        ag = agreement(a["labels"].cpu().numpy(), ref["labels"], ref["margin"], MARGIN[precision])
        assert ag["on_margin"]
        sc = (kxx + N[ref["labels"]]).mean()
        assert abs(model.objective(allidx) - ref["mind"].mean()) <= max(tol, 2e-7) * sc
    return same


def _gmm(n, d, c, std, seed):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((c, d))
    comp = rng.integers(0, c, n)
    X = (means[comp] + std * rng.standard_normal((n, d))).astype(np.float32)
    init = np.array([np.flatnonzero(comp == j)[0] for j in range(c)], np.int32)
    return X, comp, init


def test_laplace_d32_two_rows_per_lane():
    """FP32 Laplacian, d = 32 (two rows per lane), n not a multiple of the row tile."""
    wl = W.c5_laplace_mixture(seed=4, n=9001, d=32, c=24)
    init = np.array([np.flatnonzero(wl.comp == j)[0] for j in range(24)], np.int32)
    rng = np.random.default_rng(40)
    batches = [rng.integers(0, wl.n, 600).astype(np.int32) for _ in range(6)]
    assert run_untrunc(wl.X, 24, wl.kernel, 20.0, init, batches, "fp32") == 6


@pytest.mark.parametrize("d,impl", [(8, "auto"), (8, "mfma"), (20, "auto"), (64, "auto"), (72, "auto"), (100, "auto"),
                                    (64, "direct"), (128, "auto")])
def test_gauss_fp32_widths(d, impl):
    """d >= 16 with cross_impl auto, or cross_impl mfma: the table update on
    MFMA (product form); d < 16 with auto, or direct: the VALU kernel with
    coordinate differences."""
    X, comp, init = _gmm(5000, d, 10, 0.3, seed=41 + d)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(42)
    batches = [rng.integers(0, 5000, 400).astype(np.int32) for _ in range(6)]
    assert run_untrunc(X, 10, O.GAUSS, 2 * sigma * sigma, init, batches, "fp32", impl=impl) == 6


@pytest.mark.parametrize("kind,param", [(O.GAUSS, 4.0), (O.LAPLACE, 3.0), (O.LINEAR, 0.0), (O.POLY2, 0.7)])
def test_fp64_every_kernel(kind, param):
    X, comp, init = _gmm(2000, 6, 5, 0.4, seed=43)
    rng = np.random.default_rng(44)
    batches = [rng.integers(0, 2000, 150).astype(np.int32) for _ in range(6)]
    assert run_untrunc(X, 5, kind, param, init, batches, "fp64") == 6


@pytest.mark.parametrize("lr", [W.LR_SKLEARN, W.LR_FULL])
def test_learning_rates(lr):
    X, comp, init = _gmm(3000, 16, 8, 0.3, seed=45)
    rng = np.random.default_rng(46)
    batches = [rng.integers(0, 3000, 256).astype(np.int32) for _ in range(6)]
    assert run_untrunc(X, 8, O.GAUSS, 6.0, init, batches, "fp32", lr=lr) == 6


def test_many_centers_ragged_batches_duplicates_and_empty_clusters():
    """k = 40 (more centers than scoring waves), batch sizes 1 .. b_max with
    repeated points, a center that attracts nothing."""
    X, comp, init = _gmm(4000, 12, 40, 0.25, seed=47)
    far = X[init[0]].copy()
    X[init[39]] = far + 1e3  # an initial center far from every other point
    rng = np.random.default_rng(48)
    sizes = [1, 513, 7, 1024, 64, 300]
    batches = [rng.integers(0, 4000, s).astype(np.int32) for s in sizes]
    batches[2] = np.array([5, 5, 5, 9, 9, 5, 5], np.int32)
    assert run_untrunc(X, 40, O.GAUSS, 6.0, init, batches, "fp32") == len(sizes)


def test_single_center():
    X, comp, init = _gmm(1500, 4, 3, 0.5, seed=49)
    rng = np.random.default_rng(50)
    batches = [rng.integers(0, 1500, 100).astype(np.int32) for _ in range(4)]
    assert run_untrunc(X, 1, O.LAPLACE, 2.0, init[:1], batches, "fp64") == 4


def test_kmeanspp_and_early_stopping_terms():
    """k-means++ seeding feeds the table form; the last batch's objective of
    the table form equals the oracle's."""
    X, comp, _ = _gmm(3000, 8, 6, 0.3, seed=51)
    rng = np.random.default_rng(52)
    u = rng.random(6)
    model = _model(X, 6, 256, O.GAUSS, 4.0, "fp32")
    picks = model.init_kmeanspp(u).cpu().numpy()
    np.testing.assert_array_equal(picks, O.kmeanspp(X, O.GAUSS, 4.0, 6, u))
    orc = O.Oracle(X, 6, 0, O.GAUSS, 4.0)
    orc.init_centers(picks)
    for _ in range(4):
        B = rng.integers(0, 3000, 256).astype(np.int32)
        ref = orc.step(B, threads=4)
        g = model.step(B, want_objective=True)
        assert (g["labels"].cpu().numpy() == ref["labels"]).all()
        assert abs(model.last_batch_objective() - orc.objective(B)) <= 1e-5 * 2.0


def test_errors_of_the_table_form():
    from paper_2410_05902_amd import Model
    from paper_2410_05902_amd._lib import MbkkError
    X, comp, init = _gmm(500, 4, 3, 0.5, seed=53)
    Xd = torch.from_numpy(X).cuda()
    with pytest.raises(MbkkError):
        Model(Xd, k=3, b_max=64, window=0, tau=10)
    with pytest.raises(MbkkError):
        Model(Xd, k=3, b_max=64, window=0, precision="bf16x1")
    with pytest.raises(MbkkError):
        Model(Xd, k=3, b_max=64, window=0, precision="fp64", cross_impl="mfma")
    with pytest.raises(MbkkError):
        Model(Xd, k=3, b_max=64, window=0, kernel="laplace", cross_impl="mfma")
    model = Model(Xd, k=3, b_max=64, window=0, kernel_param=2.0)
    model.init_centers(init)
    with pytest.raises(MbkkError):
        model.get_state()
    with pytest.raises(MbkkError):
        model.objective_fwd(Xd[:8], 1.0)
    with pytest.raises(MbkkError):
        model.assign(np.array([0, 500], np.int32))
    with pytest.raises(MbkkError):
        model.step(np.array([1, -1, 2], np.int32))


def test_full_size_sampled_rows():
    """The Laplacian mixture at n = 4,000,000, d = 32, k = 1000, b = 8192 (the
    table form's benchmark workload): after two steps, the distances of
    sampled points of X to every center equal the oracle's."""
    wl = W.c5_laplace_mixture(seed=0)
    # one initial point per component: every label is decided by a wide margin
    first = np.full(wl.k, -1, np.int64)
    rows = np.arange(wl.n)
    first[wl.comp[::-1]] = rows[::-1]
    init = first.astype(np.int32)
    assert (init >= 0).all()
    orc = O.Oracle(wl.X, wl.k, 0, wl.kernel, wl.kernel_param)
    orc.init_centers(init)
    model = _model(wl.X, wl.k, wl.b, wl.kernel, wl.kernel_param, "fp32")
    model.init_centers(init)
    rng = np.random.default_rng(55)
    sample = np.concatenate([rng.integers(0, wl.n, 500), [0, wl.n - 1]]).astype(np.int32)
    for i in (1, 2):
        B = wl.batch(i)
        ref = orc.step(B, threads=8)
        lab = model.step(B)["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], MARGIN["fp32"])
        assert ag["on_margin"], ag["mismatches"][:8]
        if i == 1:
            np.testing.assert_array_equal(lab, ref["labels"])  # every margin is wide at step 1
        elif not (lab == ref["labels"]).all():
            break  # a near tie parted the trajectories after the compared state
        N = orc.norms()
        D = orc.distances(sample, threads=8)["D"]
        a = model.assign(sample, want_D=True)
        err = dist_rel_err(a["D"].cpu().numpy(), D, 1.0 + N[None, :])
        assert err.max() <= TOL["fp32"], f"after step {i}: {err.max():.3e}"
        np.testing.assert_allclose(model.center_norms(), N, rtol=1e-5, atol=1e-8)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_size_gaussian_mfma_sampled_rows(precision):
    """The Gaussian mixture at n = 1,000,000, d = 128, k = 100, b = 4096, window
    0 (the table update on MFMA, FP32 or BF16X3): after two steps, the
    distances of sampled points to every center equal the oracle's."""
    wl = W.c3_gaussian_mixture(seed=0)
    first = np.full(wl.k, -1, np.int64)
    rows = np.arange(wl.n)
    first[wl.comp[::-1]] = rows[::-1]
    init = first.astype(np.int32)
    assert (init >= 0).all()
    orc = O.Oracle(wl.X, wl.k, 0, wl.kernel, wl.kernel_param)
    orc.init_centers(init)
    model = _model(wl.X, wl.k, wl.b, wl.kernel, wl.kernel_param, precision)
    model.init_centers(init)
    rng = np.random.default_rng(56)
    sample = np.concatenate([rng.integers(0, wl.n, 500), [0, wl.n - 1]]).astype(np.int32)
    for i in (1, 2):
        B = wl.batch(i)
        ref = orc.step(B, threads=8)
        lab = model.step(B)["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
        assert ag["on_margin"], ag["mismatches"][:8]
        assert ag["all"] >= 0.999
        if not (lab == ref["labels"]).all():
            break
        N = orc.norms()
        D = orc.distances(sample, threads=8)["D"]
        a = model.assign(sample, want_D=True)
        err = dist_rel_err(a["D"].cpu().numpy(), D, 1.0 + N[None, :])
        assert err.max() <= TOL[precision], f"after step {i}: {err.max():.3e}"
        np.testing.assert_allclose(model.center_norms(), N, rtol=1e-5, atol=1e-8)


@pytest.mark.parametrize("d", [24, 64, 128])
def test_gauss_bf16x3_table(d):
    """BF16X3 (compensated split on MFMA) table update: distances within the
    BF16 tolerance (in practice far inside it) and the labels of every step
    equal the oracle's wherever the margin exceeds the form's error."""
    X, comp, init = _gmm(6000, d, 10, 0.3, seed=70 + d)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(71)
    batches = [rng.integers(0, 6000, 400).astype(np.int32) for _ in range(6)]
    same = run_untrunc(X, 10, O.GAUSS, 2 * sigma * sigma, init, batches, "bf16x3")
    assert same >= 4


@pytest.mark.parametrize("precision,impl", [("fp32", "auto"), ("fp32", "mfma"), ("fp64", "auto"), ("bf16x3", "auto")])
def test_tiny_data_and_single_point_batches(precision, impl):
    """n = 7 points (one partial row tile, table rows padded to 64), k = 2,
    batches of one point and of repeated points."""
    rng = np.random.default_rng(90)
    X = rng.standard_normal((7, 5)).astype(np.float32)
    init = np.array([0, 3], np.int32)
    orc = O.Oracle(X, 2, 0, O.GAUSS, 3.0)
    orc.init_centers(init)
    model = _model(X, 2, 4, O.GAUSS, 3.0, precision, impl=impl)
    model.init_centers(init)
    for B in ([6], [1, 1, 1], [2, 5, 6, 0], [4]):
        B = np.array(B, np.int32)
        ref = orc.step(B)
        lab = model.step(B)["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
        assert ag["on_margin"]
    allidx = np.arange(7, dtype=np.int32)
    ref = orc.distances(allidx)
    D = model.assign(allidx, want_D=True)["D"].cpu().numpy()
    err = dist_rel_err(D, ref["D"], 1.0 + ref["N"][None, :])
    assert err.max() <= TOL[precision]
