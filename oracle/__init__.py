"""ctypes binding of the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module.  The product package never imports it.

The binding only marshals arguments; every number is computed in oracle.c.
Rows of a distance evaluation are independent, so ``distances`` may split them
across threads (ctypes releases the GIL); that changes no value.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GAUSS, LAPLACE, LINEAR, POLY2 = 0, 1, 2, 3
LR_BETA, LR_FULL, LR_SKLEARN = 0, 1, 2


def build() -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.orc_kernel.restype = D
        L.orc_kernel.argtypes = [C.c_int, D, P, P, C.c_int]
        L.orc_create.restype = P
        L.orc_create.argtypes = [P, I64, I32, I32, I32, I32, D, I32]
        L.orc_destroy.argtypes = [P]
        L.orc_set_tau.restype = C.c_int
        L.orc_set_tau.argtypes = [P, I32]
        L.orc_init_centers.restype = C.c_int
        L.orc_init_centers.argtypes = [P, P]
        L.orc_set_centers.restype = C.c_int
        L.orc_set_centers.argtypes = [P, I64, P, P, P]
        L.orc_center_norms.argtypes = [P, P]
        L.orc_distances_n.restype = C.c_int
        L.orc_distances_n.argtypes = [P, P, P, I64, P, P, P, P]
        L.orc_terms.restype = C.c_int
        L.orc_terms.argtypes = [P, P, I64, P, P]
        L.orc_objective.restype = D
        L.orc_objective.argtypes = [P, P, I64]
        L.orc_update.restype = C.c_int
        L.orc_update.argtypes = [P, P, I32, P, P, P]
        L.orc_iteration.restype = I64
        L.orc_iteration.argtypes = [P]
        L.orc_cum.argtypes = [P, P]
        L.orc_state_size.argtypes = [P, P, P]
        L.orc_state_export.argtypes = [P, P, P, P, P, P]
        L.orc_set_terms.restype = C.c_int
        L.orc_set_terms.argtypes = [P, I64, I64, P, P, P, P, P, P]
        L.orc_kmeanspp.restype = C.c_int
        L.orc_kmeanspp.argtypes = [P, I64, I32, I32, D, I32, P, P]
        L.orc_fobj_coords.restype = D
        L.orc_fobj_coords.argtypes = [P, P, I32, D, P]
        L.orc_fobj_grad.restype = C.c_int
        L.orc_fobj_grad.argtypes = [P, P, I32, D, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def kernel(kind: int, param: float, u, v) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_kernel(kind, param, _p(u), _p(v), u.shape[0])


def kmeanspp(X: np.ndarray, kind: int, param: float, k: int, u: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape[0] >= k
    out = np.empty(k, dtype=np.int32)
    rc = lib().orc_kmeanspp(_p(X), X.shape[0], X.shape[1], kind, param, k, _p(u), _p(out))
    assert rc == 0
    return out


class Oracle:
    """One run of truncated mini-batch kernel k-means, in FP64 on one core."""

    def __init__(self, X: np.ndarray, k: int, window: int, kernel: int, param: float,
                 lr: int = LR_BETA, tau: int = 0):
        self.X = np.ascontiguousarray(X, dtype=np.float32)   # kept alive: borrowed by C
        self.k, self.window, self.kernel, self.param, self.lr = k, window, kernel, param, lr
        self.tau = tau
        self._m = lib().orc_create(_p(self.X), self.X.shape[0], self.X.shape[1], k, window,
                                   kernel, param, lr)
        if not self._m:
            raise ValueError("invalid oracle configuration")
        if tau and lib().orc_set_tau(self._m, tau) != 0:
            raise ValueError("invalid tau")

    def __del__(self):
        m, self._m = getattr(self, "_m", None), None
        if m and _lib is not None:
            _lib.orc_destroy(m)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def iteration(self) -> int:
        return int(lib().orc_iteration(self._m))

    def init_centers(self, idx):
        idx = _i32(idx)
        assert idx.shape[0] == self.k
        if lib().orc_init_centers(self._m, _p(idx)) != 0:
            raise ValueError("initial index out of range")

    def set_centers(self, centers, points, coefs):
        c, p = _i32(centers), _i32(points)
        w = np.ascontiguousarray(coefs, dtype=np.float64)
        if lib().orc_set_centers(self._m, c.shape[0], _p(c), _p(p), _p(w)) != 0:
            raise ValueError("bad center entries")

    def norms(self) -> np.ndarray:
        N = np.empty(self.k, dtype=np.float64)
        lib().orc_center_norms(self._m, _p(N))
        return N

    def distances(self, idx, threads: int = 1, N=None, want_D: bool = True):
        idx = _i32(idx)
        m = idx.shape[0]
        N = self.norms() if N is None else np.ascontiguousarray(N, dtype=np.float64)
        D = np.empty((m, self.k), dtype=np.float64) if want_D else None
        lab = np.empty(m, dtype=np.int32)
        mind = np.empty(m, dtype=np.float64)
        marg = np.empty(m, dtype=np.float64)

        def run(lo, hi):
            sl = slice(lo, hi)
            rc = lib().orc_distances_n(
                self._m, _p(N), _p(idx[sl]), hi - lo,
                None if D is None else _p(D[sl]), _p(lab[sl]), _p(mind[sl]), _p(marg[sl]))
            if rc != 0:
                raise ValueError("index out of range")

        threads = max(1, min(threads, m))
        if threads == 1:
            run(0, m)
        else:
            cuts = np.linspace(0, m, threads + 1).astype(int)
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(lambda t: run(cuts[t], cuts[t + 1]), range(threads)))
        return dict(D=D, labels=lab, mind=mind, margin=marg, N=N)

    def terms(self, idx):
        idx = _i32(idx)
        P = np.empty((idx.shape[0], self.k), dtype=np.float64)
        N = np.empty(self.k, dtype=np.float64)
        if lib().orc_terms(self._m, _p(idx), idx.shape[0], _p(P), _p(N)) != 0:
            raise ValueError("index out of range")
        return P, N

    def objective(self, idx) -> float:
        idx = _i32(idx)
        return float(lib().orc_objective(self._m, _p(idx), idx.shape[0]))

    def update(self, batch, labels):
        batch, labels = _i32(batch), _i32(labels)
        cnt = np.empty(self.k, dtype=np.int32)
        alpha = np.empty(self.k, dtype=np.float64)
        if lib().orc_update(self._m, _p(batch), batch.shape[0], _p(labels), _p(cnt), _p(alpha)) != 0:
            raise ValueError("bad batch or labels")
        return cnt, alpha

    def step(self, batch, threads: int = 1, want_D: bool = True):
        """One iteration of Algorithm 2: assignment on C_i, then the update."""
        batch = _i32(batch)
        out = self.distances(batch, threads=threads, want_D=want_D)
        out["fbefore"] = float(out["mind"].mean())
        out["counts"], out["alpha"] = self.update(batch, out["labels"])
        return out

    def state(self):
        """Every term of every center: (center, tag, coef, points)."""
        L = lib()
        nt, ne = C.c_int64(), C.c_int64()
        L.orc_state_size(self._m, C.byref(nt), C.byref(ne))
        tc = np.empty(nt.value, dtype=np.int32)
        tt = np.empty(nt.value, dtype=np.int64)
        tw = np.empty(nt.value, dtype=np.float64)
        tn = np.empty(nt.value, dtype=np.int32)
        pts = np.empty(max(ne.value, 1), dtype=np.int32)
        L.orc_state_export(self._m, _p(tc), _p(tt), _p(tw), _p(tn), _p(pts))
        cum = np.empty(self.k, dtype=np.float64)
        L.orc_cum(self._m, _p(cum))
        return dict(iteration=self.iteration, term_center=tc, term_tag=tt, term_coef=tw,
                    term_npts=tn, points=pts[: ne.value], cum=cum)

    def set_state(self, st: dict):
        """Resumes from a state in the layout of state(): the iteration counter,
        every term of every center with its batch tag, and the running counts."""
        tc = _i32(st["term_center"])
        tt = np.ascontiguousarray(st["term_tag"], dtype=np.int64)
        tw = np.ascontiguousarray(st["term_coef"], dtype=np.float64)
        tn = _i32(st["term_npts"])
        pts = _i32(st["points"])
        cum = np.ascontiguousarray(st["cum"], dtype=np.float64)
        assert tc.shape == tt.shape == tw.shape == tn.shape and int(tn.sum()) == pts.shape[0]
        if lib().orc_set_terms(self._m, int(st["iteration"]), tc.shape[0], _p(tc), _p(tt), _p(tw), _p(tn),
                               _p(pts), _p(cum)) != 0:
            raise ValueError("bad state")

    def center_entries(self):
        """Flattened (center, point, coefficient) entries of the current centers."""
        s = self.state()
        rep = s["term_npts"].astype(np.int64)
        return (np.repeat(s["term_center"], rep), s["points"], np.repeat(s["term_coef"], rep))

    def fobj_coords(self, xb: np.ndarray, sigma: float):
        xb = np.ascontiguousarray(xb, dtype=np.float64)
        lab = np.empty(xb.shape[0], dtype=np.int32)
        f = lib().orc_fobj_coords(self._m, _p(xb), xb.shape[0], sigma, _p(lab))
        return float(f), lab

    def fobj_grad(self, xb: np.ndarray, sigma: float, labels):
        xb = np.ascontiguousarray(xb, dtype=np.float64)
        labels = _i32(labels)
        dX = np.empty_like(xb)
        ds = C.c_double()
        if lib().orc_fobj_grad(self._m, _p(xb), xb.shape[0], sigma, _p(labels), _p(dX),
                               C.byref(ds)) != 0:
            raise ValueError("bad labels")
        return dX, float(ds.value)
