"""Differentiation form on the GPU (mbkk_objective_fwd / mbkk_objective_bwd and
the torch.autograd.Function) against the FP64 oracle's objective, its
closed-form gradient, and central finite differences of the oracle objective.

Both sides hold the same centers: the GPU runs a few iterations, and its state
(ring slots, coefficients) is handed to the oracle as explicit weighted
support entries."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2410_05902_amd import workloads as W

pytestmark = pytest.mark.gpu


def _entries(st, W_):
    """(center, point, weight) entries of a GPU state image."""
    cen, pts, wts = [], [], []
    k = st["coef"].shape[0]
    for j in range(k):
        c0 = st["coef"][j, 0]
        if c0 != 0.0:
            cen.append(j), pts.append(int(st["init_idx"][j])), wts.append(c0)
    for r in range(W_):
        off = st["slot_off"][r]
        for j in range(k):
            w = st["coef"][j, 1 + r]
            if w == 0.0:
                continue
            for p in st["slot_idx"][r, off[j]: off[j + 1]]:
                cen.append(j), pts.append(int(p)), wts.append(w)
    return np.array(cen, np.int32), np.array(pts, np.int32), np.array(wts, np.float64)


def _setup(wl, steps, precision="fp32", b_xb=None, noise=0.05):
    """GPU model after `steps` iterations, the oracle with the same centers,
    and a batch of coordinates near data points."""
    from paper_2410_05902_amd import Model
    X = wl.X
    Xd = torch.from_numpy(X).cuda()
    model = Model(Xd, k=wl.k, b_max=wl.b, window=wl.window, kernel="gauss", kernel_param=wl.kernel_param,
                  precision=precision)
    rng = np.random.default_rng(wl.seed + 17)
    init = rng.choice(wl.n, wl.k, replace=False).astype(np.int32)
    model.init_centers(init)
    for i in range(1, steps + 1):
        model.step(wl.batch(i))
    st = model.get_state()
    orc = O.Oracle(X, wl.k, wl.window, O.GAUSS, wl.kernel_param)
    orc.set_centers(*_entries(st, wl.window))
    b = b_xb or wl.b
    rows = rng.integers(0, wl.n, b)
    xb = (X[rows].astype(np.float64) + noise * rng.standard_normal((b, wl.d))).astype(np.float32)
    return model, orc, xb


def _small(seed=0):
    return W.c4_gaussian_mixture(seed=seed, n=20_000, b=1024)


@pytest.mark.parametrize("steps", [2, 6])
def test_forward_matches_oracle(steps):
    wl = _small()
    model, orc, xb = _setup(wl, steps)
    sigma = 1.3 * wl.sigma   # a bandwidth other than the model's own
    f, lab = model.objective_fwd(torch.from_numpy(xb).cuda(), sigma)
    fo, labo = orc.fobj_coords(xb.astype(np.float64), sigma)
    assert abs(f - fo) <= 1e-5 * abs(fo), (f, fo)
    agree = (lab.cpu().numpy() == labo).mean()
    assert agree >= 0.999, agree


def fp32_grad_bounds(X, xb, d, b, sigma, g, max_seg):
    """Bounds on the FP32-MFMA gradient's error, from its arithmetic (u = 2^-24):
      - d2 = |x|^2 + |y|^2 - 2 x.y with x.y on FP32 MFMA over dp products:
        |d d2| <= e2 = 2 (dp+1) u |x||y| + 4 u (|x|^2 + |y|^2);
      - so a kernel value has relative error eK <= e2 / (2 s^2) + 2u;
      - G = sum_e P_e y_e is an FP32 sum of at most S (longest support
        segment) terms with sum_e P_e = R <= 1 (weights sum to at most 1);
      - dX_t = c (x_t R - G_t), c = 2 g / (b s^2), so
        |d dX_t| <= c (eK (|x_t| + Ym) + S u Ym) + u |dX_t|, Ym = max |y_t|;
      - df/ds: per row -2 sum_e P_e d2_e / s^3 and dN_j / s^3 each move by at
        most (eK D2 + e2) / s^3 with D2 the largest d2, so
        |d ds| <= |g| 3 (eK D2 + e2) / s^3.
    Norms are bounded by the largest of the data and the coordinates."""
    u = 2.0 ** -24
    dp = (d + 31) // 32 * 32
    nx = float(np.sqrt((xb.astype(np.float64) ** 2).sum(1).max()))
    ny = float(np.sqrt((X.astype(np.float64) ** 2).sum(1).max()))
    e2 = 2 * (dp + 1) * u * nx * ny + 4 * u * (nx * nx + ny * ny)
    eK = e2 / (2 * sigma * sigma) + 2 * u
    ym = float(np.abs(X).max())
    c = 2 * abs(g) / (b * sigma * sigma)
    bX = c * (eK * (np.abs(xb.astype(np.float64)) + ym) + max_seg * u * ym)
    D2 = (nx + ny) ** 2
    bS = abs(g) * 3 * (eK * D2 + e2) / sigma ** 3
    return bX, bS


def _max_seg(st, W_):
    k = st["coef"].shape[0]
    seg = (st["coef"][:, 0] != 0).astype(int)
    for r in range(W_):
        seg = seg + np.diff(st["slot_off"][r]) * (st["coef"][:, 1 + r] != 0)
    return int(seg.max())


@pytest.mark.parametrize("precision,steps", [("fp32", 2), ("fp32", 6), ("bf16x3", 6), ("fp64", 6)])
def test_backward_matches_oracle_gradient(precision, steps):
    """FP32 / BF16 contexts run the backward on FP32 MFMA (bounded by its
    arithmetic, fp32_grad_bounds); the FP64 context on the VALU in FP64."""
    wl = _small()
    model, orc, xb = _setup(wl, steps, precision=precision)
    sigma = 0.8 * wl.sigma
    _, labo = orc.fobj_coords(xb.astype(np.float64), sigma)
    dXo, dso = orc.fobj_grad(xb.astype(np.float64), sigma, labo)
    g = 1.7
    dX, ds = model.objective_bwd(torch.from_numpy(xb).cuda(), sigma, torch.from_numpy(labo).cuda(), g)
    dX = dX.cpu().numpy().astype(np.float64)
    err = np.abs(dX - g * dXo)
    rel = err.max() / np.abs(g * dXo).max()
    rel_s = abs(ds - g * dso) / abs(g * dso)
    print(f"[grad {precision} steps={steps}] dX error {rel:.2e} of max, dsigma error {rel_s:.2e}", flush=True)
    if precision == "fp64":
        assert rel <= 1e-6, rel
        assert rel_s <= 1e-9, (ds, g * dso)
    else:
        bX, bS = fp32_grad_bounds(wl.X, xb, wl.d, len(xb), sigma, g, _max_seg(model.get_state(), wl.window))
        assert (err <= bX + 2.0 ** -24 * np.abs(g * dXo)).all(), float((err / bX).max())
        assert abs(ds - g * dso) <= bS, (ds, g * dso, bS)


def test_backward_without_forward_is_identical():
    """The backward reuses the forward's self norms at the same bandwidth and
    state; run alone it makes them itself, with the same bits."""
    wl = _small(seed=3)
    model, orc, xb = _setup(wl, 5, b_xb=512)
    x = torch.from_numpy(xb).cuda()
    _, lab = model.objective_fwd(x, wl.sigma)
    dX1, ds1 = model.objective_bwd(x, wl.sigma, lab)
    model.step(wl.batch(6))          # a new state: the cached norms are stale
    model.set_state(model.get_state())
    _, lab2 = model.objective_fwd(x, 1.1 * wl.sigma)   # cache at another bandwidth
    st = model.get_state()
    from paper_2410_05902_amd import Model
    other = Model(torch.from_numpy(wl.X).cuda(), k=wl.k, b_max=wl.b, window=wl.window, kernel="gauss",
                  kernel_param=wl.kernel_param)
    other.set_state(st)
    dXa, dsa = model.objective_bwd(x, wl.sigma, lab)   # cache miss: recomputed
    dXb, dsb = other.objective_bwd(x, wl.sigma, lab)   # no forward at all
    assert torch.equal(dXa, dXb) and dsa == dsb
    assert not torch.equal(dXa, dX1)                   # the state did change


def test_backward_matches_finite_differences():
    """Central differences (h = 1e-3) of the FP64 oracle objective, along sigma
    and along a random unit direction in the space of all batch coordinates.
    Rows whose label changes within the step are left out (the objective has a
    kink there), on both sides."""
    wl = _small(seed=1)
    model, orc, xb = _setup(wl, 6, b_xb=512)
    sigma = wl.sigma
    h = 1e-3
    rng = np.random.default_rng(5)
    u = rng.standard_normal(xb.shape)
    u /= np.linalg.norm(u)
    x64 = xb.astype(np.float64)
    _, lab = orc.fobj_coords(x64, sigma)
    keep = np.ones(len(xb), bool)
    for xs, ss in ((x64, sigma + h), (x64, sigma - h), (x64 + h * u, sigma), (x64 - h * u, sigma)):
        keep &= orc.fobj_coords(xs, ss)[1] == lab
    assert keep.mean() > 0.95
    xb, x64, u, lab = xb[keep], x64[keep], u[keep], lab[keep]
    dX, ds = model.objective_bwd(torch.from_numpy(xb).cuda(), sigma, torch.from_numpy(lab).cuda(), 1.0)
    dX = dX.cpu().numpy().astype(np.float64)
    fd_s = (orc.fobj_coords(x64, sigma + h)[0] - orc.fobj_coords(x64, sigma - h)[0]) / (2 * h)
    assert abs(ds - fd_s) <= 1e-4 * abs(fd_s), (ds, fd_s)
    fd_u = (orc.fobj_coords(x64 + h * u, sigma)[0] - orc.fobj_coords(x64 - h * u, sigma)[0]) / (2 * h)
    an_u = float((dX * u).sum())
    assert abs(an_u - fd_u) <= 1e-4 * abs(fd_u), (an_u, fd_u)


def test_autograd_function():
    from paper_2410_05902_amd.autograd import batch_objective
    wl = _small(seed=2)
    model, orc, xb = _setup(wl, 5, b_xb=256)
    x = torch.from_numpy(xb).cuda().requires_grad_(True)
    s = torch.tensor(wl.sigma, dtype=torch.float64, requires_grad=True)
    f = batch_objective(model, x, s)
    (2.5 * f).backward()
    f2, lab = model.objective_fwd(x.detach(), wl.sigma)
    assert float(f.detach()) == f2
    dX, ds = model.objective_bwd(x.detach(), wl.sigma, lab, 2.5)
    assert torch.equal(x.grad, dX)
    assert float(s.grad) == ds
    # a gradient step on sigma lowers or keeps the objective for a small step
    assert np.isfinite(float(s.grad))


def test_full_size_c4():
    """The differentiation-form workload at full size: n = 100,000, d = 64,
    k = 50, b = 2048, W = 4, after W + 2 iterations."""
    wl = W.make("c4")
    model, orc, xb = _setup(wl, wl.window + 2)
    x64 = xb.astype(np.float64)
    f, lab = model.objective_fwd(torch.from_numpy(xb).cuda(), wl.sigma)
    fo, labo = orc.fobj_coords(x64, wl.sigma)
    assert abs(f - fo) <= 1e-5 * abs(fo), (f, fo)
    assert (lab.cpu().numpy() == labo).mean() >= 0.999
    dXo, dso = orc.fobj_grad(x64, wl.sigma, labo)
    dX, ds = model.objective_bwd(torch.from_numpy(xb).cuda(), wl.sigma, torch.from_numpy(labo).cuda(), 1.0)
    dX = dX.cpu().numpy().astype(np.float64)
    err = np.abs(dX - dXo)
    print(f"[grad full size] dX error {err.max() / np.abs(dXo).max():.2e} of max, "
          f"dsigma error {abs(ds - dso) / abs(dso):.2e}", flush=True)
    bX, bS = fp32_grad_bounds(wl.X, xb, wl.d, len(xb), wl.sigma, 1.0, _max_seg(model.get_state(), wl.window))
    assert (err <= bX + 2.0 ** -24 * np.abs(dXo)).all()
    assert abs(ds - dso) <= bS
    # and the central differences (h = 1e-3) of the FP64 objective along sigma,
    # at 1e-4, on the rows whose label stays within the step
    h = 1e-3
    keep = (orc.fobj_coords(x64, wl.sigma + h)[1] == labo) & (orc.fobj_coords(x64, wl.sigma - h)[1] == labo)
    assert keep.mean() > 0.95
    xk = np.ascontiguousarray(x64[keep])
    fd = (orc.fobj_coords(xk, wl.sigma + h)[0] - orc.fobj_coords(xk, wl.sigma - h)[0]) / (2 * h)
    _, dsk = model.objective_bwd(torch.from_numpy(xb[keep]).cuda(), wl.sigma,
                                 torch.from_numpy(labo[keep]).cuda(), 1.0)
    assert abs(dsk - fd) <= 1e-4 * abs(fd), (dsk, fd)


def test_errors():
    from paper_2410_05902_amd import Model
    from paper_2410_05902_amd._lib import MbkkError
    wl = _small()
    Xd = torch.from_numpy(wl.X).cuda()
    lap = Model(Xd, k=wl.k, b_max=256, window=2, kernel="laplace", kernel_param=1.0)
    lap.init_centers(np.arange(wl.k))
    xb = Xd[:16].clone()
    with pytest.raises(MbkkError):
        lap.objective_fwd(xb, 1.0)
    m = Model(Xd, k=wl.k, b_max=256, window=2, kernel="gauss", kernel_param=wl.kernel_param)
    with pytest.raises(MbkkError):   # before init
        m.objective_fwd(xb, 1.0)
    m.init_centers(np.arange(wl.k))
    with pytest.raises(MbkkError):
        m.objective_fwd(xb, 0.0)
    bad = xb.clone()
    bad[3, 5] = float("nan")
    with pytest.raises(MbkkError):
        m.objective_fwd(bad, 1.0)
    lab = torch.full((16,), wl.k, dtype=torch.int32, device="cuda")
    with pytest.raises(MbkkError):
        m.objective_bwd(xb, 1.0, lab)
    # the model still steps normally afterwards, at its own bandwidth
    out = m.step(np.arange(100, 356), want_objective=True)
    assert np.isfinite(out["fbefore"])
