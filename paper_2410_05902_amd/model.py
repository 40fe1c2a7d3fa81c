"""Python face of the library: one run of truncated mini-batch kernel k-means
on one GPU.  PyTorch supplies device memory (data, workspace, outputs) and the
stream; every step of the computation runs in libmbkk's HIP kernels."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_KERNELS = {"gauss": L.GAUSS, "laplace": L.LAPLACE, "linear": L.LINEAR, "poly2": L.POLY2}
_PREC = {"fp32": L.FP32, "fp64": L.FP64, "bf16x3": L.BF16X3, "bf16x1": L.BF16X1}
_LR = {"beta": L.LR_BETA, "full": L.LR_FULL, "sklearn": L.LR_SKLEARN}
_IMPL = {"auto": L.CROSS_AUTO, "direct": L.CROSS_DIRECT, "mfma": L.CROSS_MFMA}


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Model:
    """Implicit centers held as weights over the points of their last
    `window` batches (Eq. 1), updated one batch at a time (Algorithm 2).
    window = 0: untruncated (Algorithm 1), with the centers held as the table
    of cross terms <phi(x), C_j> of every point (Appendix A).

    X: (n, d) float32 CUDA tensor, borrowed for the lifetime of the model.
    static_workspace: keep the device state in the library's static array
    (mbkk_create_static: no allocation; one such model per device at a time)
    instead of a workspace tensor.
    """

    def __init__(self, X: torch.Tensor, k: int, b_max: int, window: int, kernel="gauss",
                 kernel_param: float = 1.0, precision="fp32", lr="beta", cross_impl="auto",
                 tie_delta: float = 0.0, validate: bool = True, stream: Optional[torch.cuda.Stream] = None,
                 tau: int = 0, static_workspace: bool = False):
        if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
            raise ValueError("X must be a row-major float32 CUDA tensor")
        self.X = X
        self.device = X.device
        self.k, self.b_max, self.window = int(k), int(b_max), int(window)
        self.cfg = L.Config(n=X.shape[0], d=X.shape[1], k=self.k, b_max=self.b_max, window=self.window,
                            kernel=_code(_KERNELS, kernel), kernel_param=float(kernel_param),
                            precision=_code(_PREC, precision), lr=_code(_LR, lr),
                            cross_impl=_code(_IMPL, cross_impl), tie_delta=float(tie_delta),
                            validate=1 if validate else 0, tau=int(tau))
        lib = L.lib()
        nbytes = C.c_size_t()
        L.check(lib.mbkk_workspace_size(C.byref(self.cfg), C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                L.check(lib.mbkk_create_static(C.byref(self.cfg), C.c_void_p(self.stream.cuda_stream),
                                               C.byref(ctx)))
        else:
            raw = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            shift = (-raw.data_ptr()) % 256
            self._raw = raw
            self.workspace = raw[shift: shift + self.workspace_bytes]
            L.check(lib.mbkk_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()),
                                    self.workspace_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self._ctx = ctx
        L.check(lib.mbkk_set_data(ctx, C.c_void_p(X.data_ptr()), X.stride(0)), ctx)

    def close(self):
        """Destroys the context (also done on garbage collection)."""
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and L._lib is not None:
            L._lib.mbkk_destroy(ctx)
            self._ctx = None

    def __del__(self):
        self.close()

    # -- helpers ------------------------------------------------------------
    def _idx(self, idx) -> torch.Tensor:
        if isinstance(idx, torch.Tensor):
            t = idx.to(device=self.device, dtype=torch.int32)
        else:
            t = torch.as_tensor(np.asarray(idx, dtype=np.int32), device=self.device)
        return t.contiguous()

    def _chk(self, rc):
        L.check(rc, self._ctx)

    # -- API ----------------------------------------------------------------
    def init_centers(self, idx):
        t = self._idx(idx)
        assert t.numel() == self.k
        self._chk(L.lib().mbkk_init_centers(self._ctx, _ptr(t)))
        self._keep = t

    def init_kmeanspp(self, u) -> torch.Tensor:
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape[0] >= self.k
        out = torch.empty(self.k, dtype=torch.int32, device=self.device)
        self._chk(L.lib().mbkk_init_kmeanspp(self._ctx, u.ctypes.data_as(C.c_void_p), _ptr(out)))
        return out

    def step(self, batch, want_objective: bool = False):
        t = self._idx(batch)
        b = t.numel()
        labels = torch.empty(b, dtype=torch.int32, device=self.device)
        mind = torch.empty(b, dtype=torch.float32, device=self.device)
        f = C.c_double()
        self._chk(L.lib().mbkk_step(self._ctx, _ptr(t), b, _ptr(labels), _ptr(mind),
                                    C.byref(f) if want_objective else None))
        self._keep = t
        out = dict(labels=labels, mind=mind)
        if want_objective:
            out["fbefore"] = float(f.value)
        return out

    def step_noout(self, batch: torch.Tensor):
        """One iteration without copying outputs (benchmark path)."""
        self._chk(L.lib().mbkk_step(self._ctx, _ptr(batch), batch.numel(), None, None, None))

    def assign(self, idx, want_D: bool = False):
        t = self._idx(idx)
        m = t.numel()
        labels = torch.empty(m, dtype=torch.int32, device=self.device)
        mind = torch.empty(m, dtype=torch.float32, device=self.device)
        margin = torch.empty(m, dtype=torch.float32, device=self.device)
        D = torch.empty((m, self.k), dtype=torch.float64, device=self.device) if want_D else None
        self._chk(L.lib().mbkk_assign(self._ctx, _ptr(t), m, _ptr(labels), _ptr(mind), _ptr(margin), _ptr(D)))
        self._keep = t
        return dict(labels=labels, mind=mind, margin=margin, D=D)

    def objective(self, idx) -> float:
        t = self._idx(idx)
        f = C.c_double()
        self._chk(L.lib().mbkk_objective(self._ctx, _ptr(t), t.numel(), C.byref(f)))
        return float(f.value)

    def last_batch_objective(self) -> float:
        """f of the most recent batch under the centers after its update."""
        f = C.c_double()
        self._chk(L.lib().mbkk_last_batch_objective(self._ctx, C.byref(f)))
        return float(f.value)

    def fit(self, batches, eps: float):
        """Run steps over `batches` (an iterable of index tensors) until the
        early-stopping test of Algorithms 1 and 2 fires: the objective of the
        batch just used drops by less than eps across its update, i.e.
        f_B(C_i) - f_B(C_{i+1}) < eps.  Returns the number of steps taken and
        the per-step improvements."""
        gains = []
        for batch in batches:
            fb = self.step(batch, want_objective=True)["fbefore"]
            gains.append(fb - self.last_batch_objective())
            if gains[-1] < eps:
                break
        return len(gains), gains

    def agreement(self, labels, truth, c: int):
        """Adjusted Rand index and normalised mutual information of `labels`
        (in [0, k)) against reference labels `truth` (in [0, c)); returns
        (ari, nmi, contingency table [k x c])."""
        lab = self._idx(labels)
        tru = self._idx(truth)
        if lab.numel() != tru.numel():
            raise ValueError("labels and truth differ in length")
        table = torch.empty((self.k, c), dtype=torch.int64, device=self.device)
        ari, nmi = C.c_double(), C.c_double()
        self._chk(L.lib().mbkk_agreement(self._ctx, _ptr(lab), _ptr(tru), lab.numel(), c, _ptr(table),
                                         C.byref(ari), C.byref(nmi)))
        self._keep = (lab, tru)
        return float(ari.value), float(nmi.value), table

    def center_norms(self) -> np.ndarray:
        N = np.empty(self.k, dtype=np.float64)
        self._chk(L.lib().mbkk_center_norms(self._ctx, N.ctypes.data_as(C.c_void_p)))
        return N

    def _state_buffers(self):
        W, k, bm = self.window, self.k, self.b_max
        bufs = dict(init_idx=np.zeros(k, np.int32), slot_b=np.zeros(W, np.int32),
                    slot_idx=np.zeros(W * bm, np.int32), slot_off=np.zeros(W * (k + 1), np.int32),
                    coef=np.zeros(k * (W + 1), np.float64), cum=np.zeros(k, np.float64))
        return bufs

    @staticmethod
    def _state_struct(bufs, it, k, W, bm):
        def p(a, ct):
            return a.ctypes.data_as(C.POINTER(ct))
        return L.State(iteration=it, k=k, window=W, b_max=bm,
                       init_idx=p(bufs["init_idx"], C.c_int32), slot_b=p(bufs["slot_b"], C.c_int32),
                       slot_idx=p(bufs["slot_idx"], C.c_int32), slot_off=p(bufs["slot_off"], C.c_int32),
                       coef=p(bufs["coef"], C.c_double), cum=p(bufs["cum"], C.c_double))

    def get_state(self) -> dict:
        bufs = self._state_buffers()
        s = self._state_struct(bufs, 0, self.k, self.window, self.b_max)
        self._chk(L.lib().mbkk_get_state(self._ctx, C.byref(s)))
        W, k, bm = self.window, self.k, self.b_max
        return dict(iteration=int(s.iteration), init_idx=bufs["init_idx"], slot_b=bufs["slot_b"],
                    slot_idx=bufs["slot_idx"].reshape(W, bm), slot_off=bufs["slot_off"].reshape(W, k + 1),
                    coef=bufs["coef"].reshape(k, W + 1), cum=bufs["cum"])

    def set_state(self, st: dict):
        W, k, bm = self.window, self.k, self.b_max
        bufs = dict(init_idx=np.ascontiguousarray(st["init_idx"], np.int32).reshape(k),
                    slot_b=np.ascontiguousarray(st["slot_b"], np.int32).reshape(W),
                    slot_idx=np.ascontiguousarray(st["slot_idx"], np.int32).reshape(W * bm),
                    slot_off=np.ascontiguousarray(st["slot_off"], np.int32).reshape(W * (k + 1)),
                    coef=np.ascontiguousarray(st["coef"], np.float64).reshape(k * (W + 1)),
                    cum=np.ascontiguousarray(st["cum"], np.float64).reshape(k))
        s = self._state_struct(bufs, int(st["iteration"]), k, W, bm)
        self._chk(L.lib().mbkk_set_state(self._ctx, C.byref(s)))

    def rescore_count(self, reset: bool = False) -> int:
        """Rows re-scored in FP64 (BF16 forms) since creation or the last reset."""
        n = C.c_int64()
        self._chk(L.lib().mbkk_rescore_count(self._ctx, C.byref(n), 1 if reset else 0))
        return int(n.value)

    def selfnorm_error_bound(self) -> float:
        """Bound on the error of a center's self norm (Gaussian MFMA forms)."""
        v = C.c_double()
        self._chk(L.lib().mbkk_selfnorm_error_bound(self._ctx, C.byref(v)))
        return float(v.value)

    def set_timing(self, enable: bool):
        self._chk(L.lib().mbkk_set_timing(self._ctx, 1 if enable else 0))

    def get_timing(self):
        ms, n = C.c_double(), C.c_int64()
        self._chk(L.lib().mbkk_get_timing(self._ctx, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)

    # -- differentiation form (Gaussian kernel, bandwidth sigma) --------------
    def _coords(self, xb: torch.Tensor) -> torch.Tensor:
        if not (xb.is_cuda and xb.dtype == torch.float32 and xb.dim() == 2 and xb.shape[1] == self.X.shape[1]):
            raise ValueError("xb must be a (b, d) float32 CUDA tensor")
        return xb.contiguous()

    def objective_fwd(self, xb: torch.Tensor, sigma: float):
        """f(xb, sigma): the batch objective of Section 3 with the bandwidth-form
        Gaussian kernel exp(-||x-y||^2 / (2 sigma^2)) against the current
        centers.  Returns (f, labels)."""
        x = self._coords(xb)
        labels = torch.empty(x.shape[0], dtype=torch.int32, device=self.device)
        f = C.c_double()
        self._chk(L.lib().mbkk_objective_fwd(self._ctx, _ptr(x), x.shape[0], float(sigma), _ptr(labels),
                                             C.byref(f)))
        return float(f.value), labels

    def objective_bwd(self, xb: torch.Tensor, sigma: float, labels: torch.Tensor, g: float = 1.0):
        """Gradient of g * f at fixed labels: (dX (b, d) float32, dsigma float)."""
        x = self._coords(xb)
        lab = labels.to(device=self.device, dtype=torch.int32).contiguous()
        dX = torch.empty_like(x)
        ds = C.c_double()
        self._chk(L.lib().mbkk_objective_bwd(self._ctx, _ptr(x), x.shape[0], float(sigma), _ptr(lab), float(g),
                                             _ptr(dX), C.byref(ds)))
        return dX, float(ds.value)
