"""GPU path against the FP64 oracle, through the C ABI (libmbkk.so).

Lock-step protocol: before every compared iteration the GPU imports the
oracle's state (mbkk_set_state), so one near-tie cannot make the trajectories
diverge; the GPU's own update is then compared with the oracle's update of the
same iteration (slot contents, offsets, coefficients) whenever the labels of
that iteration agree.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import workloads as W
from tests._parity import agreement, dist_rel_err, oracle_state_to_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-5, "bf16x3": 1e-2, "bf16x1": 1e-2}
MARGIN = {"fp64": 1e-9, "fp32": 1e-4, "bf16x3": 1e-4, "bf16x1": 1e-2}


def _model(X, k, b_max, window, kernel, param, precision, impl="auto", lr="beta", tie=0.0, tau=0):
    from paper_2410_05902_amd import Model
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    return Model(Xd, k=k, b_max=b_max, window=window, kernel=kernel, kernel_param=param,
                 precision=precision, lr=lr, cross_impl=impl, tie_delta=tie, tau=tau)


KNAME = {O.GAUSS: "gauss", O.LAPLACE: "laplace", O.LINEAR: "linear", O.POLY2: "poly2"}


def lockstep(X, k, window, kind, param, init, batches, precision, impl="auto", lr=W.LR_BETA,
             b_max=None, check_state=True, threads=4, min_agree=1.0):
    """Runs the oracle and the GPU in lock-step; returns per-step stats."""
    b_max = b_max or max(len(B) for B in batches)
    lrname = {W.LR_BETA: "beta", W.LR_FULL: "full", W.LR_SKLEARN: "sklearn"}[lr]
    orc = O.Oracle(X, k, window, kind, param, lr)
    orc.init_centers(init)
    model = _model(X, k, b_max, window, KNAME[kind], param, precision, impl, lrname)
    model.init_centers(init)
    tol, mmin = TOL[precision], MARGIN[precision]
    stats = []
    for i, B in enumerate(batches, start=1):
        model.set_state(oracle_state_to_gpu(orc.state(), init, k, window, b_max))
        # centers' self norms: GPU Gram blocks vs the oracle's direct quadratic form
        Ng = model.center_norms()
        a = model.assign(B, want_D=True)
        ref = orc.step(B, threads=threads)
        No = ref["N"]
        np.testing.assert_allclose(Ng, No, rtol=max(tol, 1e-12), atol=1e-12 + tol * 1e-3)
        kxx = {O.GAUSS: 1.0, O.LAPLACE: 1.0}.get(kind)
        if kxx is None:
            x = X[B].astype(np.float64)
            sq = (x * x).sum(1)
            kxx = sq if kind == O.LINEAR else (sq + param) ** 2
        scale = np.broadcast_to(np.asarray(kxx).reshape(-1, 1), ref["D"].shape) + No[None, :]
        D = a["D"].cpu().numpy()
        err = dist_rel_err(D, ref["D"], scale)
        assert err.max() <= tol, f"step {i}: distance error {err.max():.3e} > {tol}"
        ag = agreement(a["labels"].cpu().numpy(), ref["labels"], ref["margin"], mmin)
        assert ag["on_margin"], f"step {i}: label mismatch on rows with margin >= {mmin}: {ag['mismatches'][:8]}"
        assert ag["all"] >= min_agree, f"step {i}: agreement {ag['all']:.5f}"
        stats.append(dict(err=float(err.max()), agree=ag["all"]))
    return orc, model, stats


def _step_and_compare_state(X, k, window, kind, param, init, batches, precision, impl="auto",
                            lr=W.LR_BETA, b_max=None, tau=0):
    """Lock-step on full iterations: import the oracle state, run one GPU step
    and one oracle step on the same batch, compare labels, min distance and the
    updated state."""
    b_max = b_max or max(len(B) for B in batches)
    lrname = {W.LR_BETA: "beta", W.LR_FULL: "full", W.LR_SKLEARN: "sklearn"}[lr]
    orc = O.Oracle(X, k, window, kind, param, lr, tau=tau)
    orc.init_centers(init)
    model = _model(X, k, b_max, window, KNAME[kind], param, precision, impl, lrname, tau=tau)
    model.init_centers(init)
    tol, mmin = TOL[precision], MARGIN[precision]
    compared = 0
    for i, B in enumerate(batches, start=1):
        model.set_state(oracle_state_to_gpu(orc.state(), init, k, window, b_max))
        g = model.step(B, want_objective=True)
        ref = orc.step(B, threads=4)
        lab = g["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], mmin)
        assert ag["on_margin"], f"step {i}: {ag['mismatches'][:8]}"
        mind = g["mind"].cpu().numpy().astype(np.float64)
        scale = 1.0 + ref["N"][ref["labels"]] if kind in (O.GAUSS, O.LAPLACE) else None
        if scale is not None:
            same = lab == ref["labels"]
            e = dist_rel_err(mind[same], ref["mind"][same], scale[same])
            assert e.max() <= max(tol, 2e-7), f"step {i}: min-distance error {e.max():.3e}"
            assert g["fbefore"] == pytest.approx(ref["fbefore"], rel=max(tol, 1e-6), abs=1e-9)
        if (lab == ref["labels"]).all():
            # second term of the early-stopping test: the batch under the updated centers
            assert model.last_batch_objective() == pytest.approx(orc.objective(B), rel=max(tol, 1e-6), abs=1e-9)
            sg = model.get_state()
            so = oracle_state_to_gpu(orc.state(), init, k, window, b_max)
            assert sg["iteration"] == so["iteration"]
            live = [((l - 1) % window) for l in range(max(1, i - window + 1), i + 1)]
            if tau == 0:
                for r in live:
                    assert sg["slot_b"][r] == so["slot_b"][r]
                    np.testing.assert_array_equal(sg["slot_off"][r], so["slot_off"][r])
                    np.testing.assert_array_equal(sg["slot_idx"][r, : so["slot_b"][r]],
                                                  so["slot_idx"][r, : so["slot_b"][r]])
            else:
                # the oracle drops a truncated center's points, the ring keeps
                # them at weight 0: compare each center's weighted points
                for r in live:
                    for c in range(k):
                        if so["coef"][c, 1 + r] != 0.0:
                            a = sg["slot_idx"][r, sg["slot_off"][r][c]: sg["slot_off"][r][c + 1]]
                            b = so["slot_idx"][r, so["slot_off"][r][c]: so["slot_off"][r][c + 1]]
                            np.testing.assert_array_equal(a, b)
            cols = ([0] if i <= window else []) + [1 + r for r in live]
            np.testing.assert_allclose(sg["coef"][:, cols], so["coef"][:, cols], rtol=1e-12, atol=1e-15)
            compared += 1
    assert compared >= len(batches) // 2
    return orc, model


# ---------------------------------------------------------------------------
# the 2-D blob workload in full: 20 iterations, k-means++ seeding
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    wl = W.c1_blobs(seed=0)
    init = O.kmeanspp(wl.X, wl.kernel, wl.kernel_param, wl.k, wl.kmeanspp_uniforms())
    return wl, init


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_distances_lockstep(c1, precision):
    wl, init = c1
    batches = [wl.batch(i) for i in range(1, wl.iterations + 1)]
    lockstep(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param, init, batches, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_steps_and_state(c1, precision):
    wl, init = c1
    batches = [wl.batch(i) for i in range(1, wl.iterations + 1)]
    _step_and_compare_state(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param, init, batches, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_free_running_trajectory(c1, precision):
    """Without state import: 20 GPU iterations give the oracle's labels on
    every row whose margin exceeds the precision's threshold."""
    wl, init = c1
    orc = O.Oracle(wl.X, wl.k, wl.window, wl.kernel, wl.kernel_param)
    orc.init_centers(init)
    model = _model(wl.X, wl.k, wl.b, wl.window, "gauss", wl.kernel_param, precision)
    model.init_centers(init)
    for i in range(1, wl.iterations + 1):
        B = wl.batch(i)
        ref = orc.step(B)
        g = model.step(B)
        lab = g["labels"].cpu().numpy()
        if precision == "fp64":
            np.testing.assert_array_equal(lab, ref["labels"])
        else:
            ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
            assert ag["on_margin"], ag["mismatches"]
    allidx = np.arange(wl.n, dtype=np.int32)
    assert model.objective(allidx) == pytest.approx(orc.objective(allidx), rel=TOL[precision] * 10)


def test_c1_kmeanspp_picks(c1):
    wl, init = c1
    model = _model(wl.X, wl.k, wl.b, wl.window, "gauss", wl.kernel_param, "fp64")
    picks = model.init_kmeanspp(wl.kmeanspp_uniforms()).cpu().numpy()
    np.testing.assert_array_equal(picks, init)
    u = np.random.default_rng(3).random(40)
    ref = O.kmeanspp(wl.X, wl.kernel, wl.kernel_param, 40, u)
    model = _model(wl.X, 40, wl.b, wl.window, "gauss", wl.kernel_param, "fp32")
    np.testing.assert_array_equal(model.init_kmeanspp(u).cpu().numpy(), ref)


# ---------------------------------------------------------------------------
# MFMA and BF16 forms, shapes of the larger workloads at reduced n
# ---------------------------------------------------------------------------

def _small_gmm(n, d, c, std, seed=0, scale=1.0, with_comp=False):
    rng = np.random.default_rng(seed)
    means = scale * rng.standard_normal((c, d))
    comp = rng.integers(0, c, n)
    X = (means[comp] + std * rng.standard_normal((n, d))).astype(np.float32)
    return (X, comp) if with_comp else X


def _one_per_component(comp, c):
    """The first point of every component: initial centers without shared or
    empty components, so that no exact tie decides a label."""
    return np.array([np.flatnonzero(comp == j)[0] for j in range(c)], np.int32)


@pytest.mark.parametrize("precision,impl", [("fp32", "mfma"), ("bf16x3", "mfma"), ("bf16x1", "mfma"),
                                            ("fp32", "direct"), ("fp64", "direct")])
def test_gmm128_lockstep(precision, impl):
    X = _small_gmm(12000, 128, 20, 0.3)
    sigma = W.median_pairwise_distance(X, 0)
    k, b, Wn = 20, 300, 3
    rng = np.random.default_rng(1)
    init = rng.choice(X.shape[0], k, replace=False).astype(np.int32)
    batches = [rng.integers(0, X.shape[0], b).astype(np.int32) for _ in range(Wn + 3)]
    agree = 0.999 if precision.startswith("bf16") else 1.0
    lockstep(X, k, Wn, O.GAUSS, 2 * sigma * sigma, init, batches, precision, impl,
             min_agree=agree if precision != "fp32" else 1.0)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_gmm128_steps_and_state(precision):
    X = _small_gmm(12000, 128, 20, 0.3, seed=2)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(4)
    init = rng.choice(X.shape[0], 20, replace=False).astype(np.int32)
    batches = [rng.integers(0, X.shape[0], 257).astype(np.int32) for _ in range(6)]
    _step_and_compare_state(X, 20, 3, O.GAUSS, 2 * sigma * sigma, init, batches, precision, "mfma")


def test_sparse784_mfma_fp32():
    """MNIST-shaped rows (d = 784, sparse prototypes in [0,1])."""
    wl = W.c2_sparse_prototypes(seed=0, n=6000)
    rng = np.random.default_rng(5)
    init = rng.choice(wl.n, wl.k, replace=False).astype(np.int32)
    batches = [rng.integers(0, wl.n, 200).astype(np.int32) for _ in range(5)]
    lockstep(wl.X, wl.k, 3, wl.kernel, wl.kernel_param, init, batches, "fp32", "mfma")


def test_laplace32_direct_lockstep():
    wl = W.c5_laplace_mixture(seed=0, n=20000, c=100)
    rng = np.random.default_rng(6)
    init = rng.choice(wl.n, 100, replace=False).astype(np.int32)
    batches = [rng.integers(0, wl.n, 700).astype(np.int32) for _ in range(wl.window + 2)]
    lockstep(wl.X, 100, wl.window, wl.kernel, wl.kernel_param, init, batches, "fp32")
    _step_and_compare_state(wl.X, 100, wl.window, wl.kernel, wl.kernel_param, init, batches, "fp32")


@pytest.mark.parametrize("kind,param", [(O.LINEAR, 0.0), (O.POLY2, 0.7)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_test_kernels_lockstep(kind, param, precision):
    X = _small_gmm(3000, 5, 4, 0.4, seed=7)
    rng = np.random.default_rng(8)
    init = rng.choice(3000, 4, replace=False).astype(np.int32)
    batches = [rng.integers(0, 3000, 100).astype(np.int32) for _ in range(6)]
    lockstep(X, 4, 2, kind, param, init, batches, precision)


# ---------------------------------------------------------------------------
# learning-rate rules, window 1, k = 1, edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lr", [W.LR_SKLEARN, W.LR_FULL])
def test_learning_rate_rules(lr):
    X = _small_gmm(4000, 8, 5, 0.3, seed=9)
    rng = np.random.default_rng(10)
    init = rng.choice(4000, 5, replace=False).astype(np.int32)
    batches = [rng.integers(0, 4000, 128).astype(np.int32) for _ in range(7)]
    _step_and_compare_state(X, 5, 3, O.GAUSS, 3.0, init, batches, "fp64", lr=lr)


def test_window_one_and_single_center():
    X = _small_gmm(2000, 4, 3, 0.3, seed=11)
    rng = np.random.default_rng(12)
    batches = [rng.integers(0, 2000, 64).astype(np.int32) for _ in range(5)]
    _step_and_compare_state(X, 3, 1, O.GAUSS, 2.0, np.array([0, 1, 2], np.int32), batches, "fp64")
    _step_and_compare_state(X, 1, 2, O.GAUSS, 2.0, np.array([5], np.int32), batches, "fp64")


def test_empty_cluster_and_duplicates():
    """A far-away initial center receives no points (alpha = 0); batches
    repeat indices."""
    X = _small_gmm(1000, 3, 2, 0.2, seed=13)
    X = np.vstack([X, np.full((1, 3), 50.0, np.float32)])
    init = np.array([0, 1, 1000], np.int32)
    base = np.random.default_rng(14).integers(0, 1000, 40).astype(np.int32)
    batches = [np.concatenate([base, base[:10]]) for _ in range(4)]
    _step_and_compare_state(X, 3, 2, O.GAUSS, 1.5, init, batches, "fp64")


@pytest.mark.parametrize("param", [1e-6, 1e8])
def test_bandwidth_extremes(param):
    X = _small_gmm(1500, 6, 3, 0.5, seed=15)
    rng = np.random.default_rng(16)
    init = rng.choice(1500, 3, replace=False).astype(np.int32)
    batches = [rng.integers(0, 1500, 90).astype(np.int32) for _ in range(4)]
    lockstep(X, 3, 2, O.GAUSS, param, init, batches, "fp64")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_ragged_batch_sizes_mfma(precision):
    """Batch sizes that are not multiples of the 128-row tile, down to b = 1
    (waves whose rows all lie past the batch still stage their share of the
    support)."""
    X = _small_gmm(5000, 64, 10, 0.4, seed=17)
    rng = np.random.default_rng(18)
    init = rng.choice(5000, 10, replace=False).astype(np.int32)
    batches = [rng.integers(0, 5000, b).astype(np.int32) for b in (1, 129, 255, 77, 300)]
    lockstep(X, 10, 2, O.GAUSS, 40.0, init, batches, precision, "mfma", b_max=300,
             min_agree=0.999 if precision == "bf16x3" else 1.0)


# ---------------------------------------------------------------------------
# free-running steps: the paths that only consecutive iterations take (the
# update writes the next segment offsets and the Gram task plan; the Gram
# work is folded into G by the next support layout), for the VALU Gram with
# two column rows per lane, both update kernels (k <= 512 and larger), the
# MFMA Gram and FP64
# ---------------------------------------------------------------------------

def free_run(X, k, window, kind, param, init, batches, precision, impl="auto", threads=4, tau=0):
    """GPU and oracle from the same initial centers, no state import: labels
    agree on rows with margin; while all labels agree, the self norms of the
    centers after the last step agree with the oracle's.  Returns the number
    of steps with identical labels."""
    orc = O.Oracle(X, k, window, kind, param, tau=tau)
    orc.init_centers(init)
    model = _model(X, k, max(len(B) for B in batches), window, KNAME[kind], param, precision, impl, tau=tau)
    model.init_centers(init)
    same = 0
    for B in batches:
        ref = orc.step(B, threads=threads)
        lab = model.step(B)["labels"].cpu().numpy()
        ag = agreement(lab, ref["labels"], ref["margin"], MARGIN[precision])
        assert ag["on_margin"], f"step {same + 1}: {ag['mismatches'][:8]}"
        if not (lab == ref["labels"]).all():
            return same  # a near tie parted the trajectories
        same += 1
    np.testing.assert_allclose(model.center_norms(), orc.norms(), rtol=max(TOL[precision], 1e-12),
                               atol=1e-12 + TOL[precision] * 1e-3)
    return same


def test_free_running_laplace_two_rows_per_lane():
    """d = 16 Laplacian FP32: direct cross kernel and VALU Gram with two rows per lane, k <= 512."""
    wl = W.c5_laplace_mixture(seed=1, n=12000, d=16, c=20)
    init = _one_per_component(wl.comp, 20)
    rng = np.random.default_rng(30)
    batches = [rng.integers(0, wl.n, 700).astype(np.int32) for _ in range(8)]
    assert free_run(wl.X, 20, 3, wl.kernel, 8.0, init, batches, "fp32") == 8


def test_free_running_large_k_general_update():
    """k = 600 with 32 chunks per batch: the general update kernel (counts in global memory)."""
    wl = W.c5_laplace_mixture(seed=2, n=30000, d=32, c=600)
    init = _one_per_component(wl.comp, 600)
    rng = np.random.default_rng(31)
    batches = [rng.integers(0, wl.n, 2048).astype(np.int32) for _ in range(4)]
    assert free_run(wl.X, 600, 2, wl.kernel, 20.0, init, batches, "fp32") == 4


@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
def test_free_running_mfma(precision):
    X, comp = _small_gmm(8000, 64, 12, 0.3, seed=32, with_comp=True)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(33)
    batches = [rng.integers(0, 8000, 512).astype(np.int32) for _ in range(8)]
    same = free_run(X, 12, 3, O.GAUSS, 2 * sigma * sigma, _one_per_component(comp, 12), batches, precision,
                    "mfma")
    assert same == 8


@pytest.mark.parametrize("k,b,window,steps", [(3, 2048, 3, 6), (2, 4096, 2, 4)])
def test_free_running_mfma_large_clusters(k, b, window, steps):
    """Clusters of 650-2100 rows: the Gram plan's 16 x 16 tasks outnumber the
    work kernel's 5120 waves, so the plan takes 2-4 (first case) or 8 (second)
    column tiles per task and each task loads its slot rows once for all of
    them; the self norms after the last step against the oracle's."""
    X, comp = _small_gmm(20000, 32, k, 0.3, seed=36, with_comp=True)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(37)
    batches = [rng.integers(0, 20000, b).astype(np.int32) for _ in range(steps)]
    same = free_run(X, k, window, O.GAUSS, 2 * sigma * sigma, _one_per_component(comp, k), batches, "fp32",
                    "mfma")
    assert same == steps


def test_free_running_fp64_direct():
    X, comp = _small_gmm(3000, 8, 6, 0.4, seed=34, with_comp=True)
    rng = np.random.default_rng(35)
    batches = [rng.integers(0, 3000, 200).astype(np.int32) for _ in range(8)]
    assert free_run(X, 6, 3, O.GAUSS, 4.0, _one_per_component(comp, 6), batches, "fp64", "direct") == 8


# ---------------------------------------------------------------------------
# the count truncation of Section 4.1 (tau) within the window
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,impl", [("fp32", "mfma"), ("bf16x3", "mfma"), ("fp32", "direct")])
def test_tau_free_running(precision, impl):
    """tau = 60 with about 21 points per center and batch: centers drop their
    older batches (and the initial point) well inside the 8-batch window."""
    X, comp = _small_gmm(6000, 32, 12, 0.3, seed=50, with_comp=True)
    sigma = W.median_pairwise_distance(X, 0)
    rng = np.random.default_rng(51)
    batches = [rng.integers(0, 6000, 256).astype(np.int32) for _ in range(10)]
    same = free_run(X, 12, 8, O.GAUSS, 2 * sigma * sigma, _one_per_component(comp, 12), batches, precision,
                    impl, tau=60)
    assert same == 10


def test_tau_state_lockstep():
    """Imported states and one step at a time: the coefficients after the
    count truncation equal the oracle's (dropped columns at 0)."""
    X, comp = _small_gmm(3000, 6, 5, 0.4, seed=52, with_comp=True)
    rng = np.random.default_rng(53)
    batches = [rng.integers(0, 3000, 90).astype(np.int32) for _ in range(8)]
    _step_and_compare_state(X, 5, 6, O.GAUSS, 3.0, _one_per_component(comp, 5), batches, "fp64", tau=40)


def test_tau_large_k_general_update():
    """k = 600: the general update kernel applies the count truncation."""
    wl = W.c5_laplace_mixture(seed=3, n=30000, d=32, c=600)
    init = _one_per_component(wl.comp, 600)
    rng = np.random.default_rng(54)
    batches = [rng.integers(0, wl.n, 2048).astype(np.int32) for _ in range(5)]
    assert free_run(wl.X, 600, 4, wl.kernel, 20.0, init, batches, "fp32", tau=6) == 5


@pytest.mark.parametrize("precision,impl", [("fp32", "mfma"), ("fp32", "direct"), ("bf16x3", "mfma")])
def test_early_stopping_fit(precision, impl):
    """Algorithm 2's stopping test: the improvement f_B(C_i) - f_B(C_{i+1}) of
    each batch agrees with the oracle's, and fit stops at the first step whose
    improvement falls below eps."""
    X, comp = _small_gmm(6000, 32, 12, 0.3, seed=60, with_comp=True)
    sigma = W.median_pairwise_distance(X, 0)
    kappa = 2 * sigma * sigma
    init = _one_per_component(comp, 12)
    rng = np.random.default_rng(61)
    batches = [rng.integers(0, 6000, 256).astype(np.int32) for _ in range(12)]
    orc = O.Oracle(X, 12, 4, O.GAUSS, kappa)
    orc.init_centers(init)
    gains_o = []
    for B in batches:
        ref = orc.step(B, threads=4)
        gains_o.append(ref["fbefore"] - orc.objective(B))
    gains_o = np.array(gains_o)
    # eps halfway between two improvements far apart, so rounding cannot move the stop
    order = np.sort(gains_o[2:8])
    gap = np.argmax(np.diff(order))
    eps = 0.5 * (order[gap] + order[gap + 1])
    stop_o = int(np.flatnonzero(gains_o < eps)[0]) + 1
    model = _model(X, 12, 256, 4, "gauss", kappa, precision, impl)
    model.init_centers(init)
    n, gains = model.fit([torch.from_numpy(B) for B in batches], eps)
    tol = max(TOL[precision], 1e-6)
    np.testing.assert_allclose(gains, gains_o[:n], rtol=0, atol=tol * 2.0)
    assert n == stop_o, (n, stop_o, gains, gains_o)
    # after the stop the entry point still scores the last batch used
    assert model.last_batch_objective() == pytest.approx(model.objective(batches[n - 1]), rel=1e-12)


def test_last_batch_objective_before_any_step_is_an_error():
    from paper_2410_05902_amd._lib import MbkkError
    X = _small_gmm(500, 8, 4, 0.4)
    model = _model(X, 4, 64, 2, "gauss", 4.0, "fp32")
    model.init_centers(np.arange(4, dtype=np.int32))
    with pytest.raises(MbkkError):
        model.last_batch_objective()


def test_agreement_scores():
    """Contingency table bit-exact, ARI and NMI of Section 6 against the oracle:
    assignments of a Gaussian mixture against its components (LDS table), many
    rows in many workgroups, and a table too large for LDS."""
    from oracle import scores
    from paper_2410_05902_amd._lib import MbkkError
    X, comp = _small_gmm(20000, 16, 10, 0.5, seed=70, with_comp=True)
    model = _model(X, 10, 4096, 2, "gauss", 8.0, "fp32")
    model.init_centers(_one_per_component(comp, 10))
    lab = model.assign(np.arange(20000))["labels"].cpu().numpy()
    rng = np.random.default_rng(71)
    big_u = rng.integers(0, 10, 3_000_000).astype(np.int32)
    cases = [(lab, comp, 10), (lab, comp % 3, 3), (big_u, (big_u * 7 + rng.integers(0, 3, big_u.size)) % 13, 13),
             (lab, rng.integers(0, 4000, lab.size), 4000), (lab[:2], comp[:2], 10),
             # one reference class; a table of k c = 32760 cells (counted in LDS) and of 32770 (global)
             (lab, np.zeros_like(comp), 1), (lab, rng.integers(0, 3276, lab.size), 3276),
             (lab, rng.integers(0, 3277, lab.size), 3277)]
    for u, v, c in cases:
        ari, nmi, table = model.agreement(u, v, c)
        n = scores.contingency(u, v, 10, c)
        np.testing.assert_array_equal(table.cpu().numpy(), n)
        assert ari == pytest.approx(scores.ari(n), rel=1e-12, abs=1e-12)
        assert nmi == pytest.approx(scores.nmi(n), rel=1e-12, abs=1e-12)
    assert model.agreement(lab, comp, 10)[0] > 0.5
    bad = comp.copy()
    bad[5] = 10
    with pytest.raises(MbkkError):
        model.agreement(lab, bad, 10)


def test_bad_index_and_nonfinite_are_errors():
    from paper_2410_05902_amd._lib import MbkkError, E_INDEX, E_NONFINITE
    X = _small_gmm(500, 4, 2, 0.3, seed=19)
    model = _model(X, 2, 64, 2, "gauss", 1.0, "fp32")
    model.init_centers([0, 1])
    with pytest.raises(MbkkError) as e:
        model.step(np.array([0, 3, 500], np.int32))
    assert e.value.code == E_INDEX
    with pytest.raises(MbkkError) as e:
        model.step(np.array([-1], np.int32))
    assert e.value.code == E_INDEX
    Xn = X.copy()
    Xn[7, 2] = np.nan
    model = _model(Xn, 2, 64, 2, "gauss", 1.0, "fp32")
    model.init_centers([0, 1])
    with pytest.raises(MbkkError) as e:
        model.step(np.array([3, 7], np.int32))
    assert e.value.code == E_NONFINITE


def test_bit_reproducible():
    X = _small_gmm(8000, 128, 16, 0.3, seed=20)
    rng = np.random.default_rng(21)
    init = rng.choice(8000, 16, replace=False).astype(np.int32)
    batches = [rng.integers(0, 8000, 512).astype(np.int32) for _ in range(5)]
    outs = []
    for _ in range(2):
        model = _model(X, 16, 512, 2, "gauss", 30.0, "bf16x3")
        model.init_centers(init)
        res = [model.step(B)["mind"].cpu().numpy() for B in batches]
        res.append(model.center_norms())
        outs.append(res)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
