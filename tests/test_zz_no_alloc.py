"""mbkk_create_static, the entry point that allocates nothing: its context keeps
the device state in the library's static per-GPU array.  Through the C ABI its
results must equal those of a context from mbkk_create on the same inputs, bit
for bit (same kernels, same launch order), on two contexts in a row, the
second with a smaller configuration (so the first one's contents are still in
the array when it starts).  Both are also checked against the FP64 oracle at
the precision forms' bar.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import _lib as L
from paper_2410_05902_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-2}


def _data(seed, n, d, c):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((c, d))
    X = (means[rng.integers(0, c, n)] + 0.3 * rng.standard_normal((n, d))).astype(np.float32)
    sigma = W.median_pairwise_distance(X, seed)
    return X, 2.0 * sigma * sigma


def _run(model, X, k, steps, seed, b):
    """k-means++ seeding, `steps` iterations, then an assignment of one more batch."""
    picks = model.init_kmeanspp(W.kmeanspp_uniforms(seed, k)).cpu().numpy()
    outs = []
    for i in range(1, steps + 1):
        B = W.batch_indices(seed, i, X.shape[0], b)
        o = model.step(B, want_objective=True)
        outs.append((o["labels"].cpu().numpy(), o["mind"].cpu().numpy(), o["fbefore"]))
    Bq = W.batch_indices(seed, steps + 1, X.shape[0], b)
    a = model.assign(Bq, want_D=True)
    return picks, outs, a, model.get_state(), model.center_norms(), Bq


@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
def test_static_workspace_matches_workspace_context(precision):
    from paper_2410_05902_amd import Model
    cases = [  # second case smaller: fewer rows, dimensions, centers and batch
        dict(seed=21, n=40000, d=96, c=24, k=24, b=2048, W=3, steps=6),
        dict(seed=22, n=6000, d=40, c=8, k=8, b=512, W=2, steps=5),
    ]
    for cs in cases:
        X, kappa = _data(cs["seed"], cs["n"], cs["d"], cs["c"])
        Xd = torch.from_numpy(X).cuda()
        kw = dict(k=cs["k"], b_max=cs["b"], window=cs["W"], kernel="gauss", kernel_param=kappa,
                  precision=precision)
        print(f"[no-alloc {precision}] n={cs['n']} d={cs['d']} k={cs['k']} b={cs['b']} W={cs['W']}",
              flush=True)
        ref_model = Model(Xd, **kw)
        ref = _run(ref_model, X, cs["k"], cs["steps"], cs["seed"], cs["b"])
        ref_model.close()
        st_model = Model(Xd, static_workspace=True, **kw)
        assert st_model.workspace is None
        got = _run(st_model, X, cs["k"], cs["steps"], cs["seed"], cs["b"])
        np.testing.assert_array_equal(got[0], ref[0])                  # k-means++ picks
        for (lg, mg, fg), (lr, mr, fr) in zip(got[1], ref[1]):
            np.testing.assert_array_equal(lg, lr)                       # labels
            np.testing.assert_array_equal(mg, mr)                       # min distances
            assert fg == fr                                             # batch objective
        for key in ("labels", "mind", "margin", "D"):
            np.testing.assert_array_equal(got[2][key].cpu().numpy(), ref[2][key].cpu().numpy())
        for key in ("iteration", "init_idx", "slot_b", "slot_idx", "slot_off", "coef", "cum"):
            np.testing.assert_array_equal(np.asarray(got[3][key]), np.asarray(ref[3][key]))
        np.testing.assert_array_equal(got[4], ref[4])                   # self norms
        # and the FP64 oracle on the final state, at the form's bar
        orc = O.Oracle(X, cs["k"], cs["W"], O.GAUSS, kappa)
        from tests._parity import oracle_from_gpu_state, dist_rel_err
        oracle_from_gpu_state(orc, got[3], cs["k"], cs["W"])
        r = orc.distances(got[5], threads=8)
        D = got[2]["D"].cpu().numpy()
        err = dist_rel_err(D, r["D"], 1.0 + r["N"][None, :])
        assert err.max() <= TOL[precision]
        lab = got[2]["labels"].cpu().numpy()
        sel = r["margin"] >= 1e-4
        assert (lab[sel] == r["labels"][sel]).all()
        st_model.close()


def test_static_workspace_limits():
    """One static context per device at a time, and configurations larger
    than the array are refused, both with clear errors and no allocation."""
    from paper_2410_05902_amd import Model
    X, kappa = _data(23, 3000, 16, 4)
    Xd = torch.from_numpy(X).cuda()
    kw = dict(k=4, b_max=256, window=2, kernel="gauss", kernel_param=kappa, precision="fp32")
    a = Model(Xd, static_workspace=True, **kw)
    with pytest.raises(L.MbkkError) as e:
        Model(Xd, static_workspace=True, **kw)
    assert e.value.code == L.E_STATE
    a.close()
    b = Model(Xd, static_workspace=True, **kw)   # free again after destroy
    b.close()
    big = L.Config(n=4_000_000, d=32, k=1000, b_max=8192, window=4, kernel=L.LAPLACE, kernel_param=4.0,
                   precision=L.FP32, lr=L.LR_BETA, cross_impl=L.CROSS_AUTO, tie_delta=0.0, validate=0, tau=0)
    ctx = C.c_void_p()
    rc = L.lib().mbkk_create_static(C.byref(big), None, C.byref(ctx))
    assert rc == L.E_WORKSPACE
    assert b"static array" in L.lib().mbkk_last_error(None)
