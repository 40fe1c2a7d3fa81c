"""Quality comparison of learning rates, truncation and precision forms.

Section 6 compares the learning rate of Section 5 (alpha = sqrt(b_j / b))
with the count-based rate (alpha = b_j / sum of b_j so far), truncated with
untruncated mini-batch kernel k-means, by the adjusted Rand index and the
normalised mutual information against the true labels, after a fixed number
of iterations without a stopping test.  This harness runs that comparison on
the seeded synthetic workloads (the paper's datasets are not available): each
configuration starts from the same kernel k-means++ seeding and takes the
same batches; it then assigns every point and scores the labels against the
generating components with the library's own contingency kernel.

    python -m paper_2410_05902_amd.quality --workload c4 --iterations 50

prints one JSON line per configuration.
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Iterable, Optional

import numpy as np

from . import workloads as W

KNAME = {W.GAUSS: "gauss", W.LAPLACE: "laplace"}


def run_config(wl: W.Workload, X, lr: str, window: int, precision: str, iterations: int,
               b: Optional[int] = None) -> dict:
    """One configuration of the comparison; X is wl.X on the GPU."""
    import torch
    from .model import Model

    b = b or wl.b
    model = Model(X, k=wl.k, b_max=b, window=window, kernel=KNAME[wl.kernel], kernel_param=wl.kernel_param,
                  precision=precision, lr=lr, validate=False)
    model.init_kmeanspp(wl.kmeanspp_uniforms())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(1, iterations + 1):
        model.step_noout(torch.from_numpy(wl.batch(i, b)).to(X.device))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    allidx = torch.arange(wl.n, dtype=torch.int32, device=X.device)
    labels = model.assign(allidx)["labels"]
    c = int(wl.comp.max()) + 1
    ari, nmi, _ = model.agreement(labels, torch.from_numpy(wl.comp.astype(np.int32)).to(X.device), c)
    f = model.objective(allidx)
    return {"workload": wl.name, "lr": lr, "window": window, "precision": precision, "b": b,
            "iterations": iterations, "ari": ari, "nmi": nmi, "objective_all": f,
            "ms_per_step": (t1 - t0) * 1e3 / iterations}


def compare(wl: W.Workload, iterations: int, lrs: Iterable[str] = ("beta", "sklearn"),
            windows: Optional[Iterable[int]] = None, precisions: Iterable[str] = ("fp32",),
            b: Optional[int] = None) -> list:
    import torch

    X = torch.from_numpy(wl.X).cuda()
    windows = list(windows) if windows is not None else [wl.window, 0]
    out = []
    for prec in precisions:
        for window in windows:
            if window == 0 and prec == "bf16x1":
                continue  # the table form runs in FP32, FP64 or BF16X3
            for lr in lrs:
                out.append(run_config(wl, X, lr, window, prec, iterations, b))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="c4", choices=sorted(W.CONFIGS))
    ap.add_argument("--iterations", type=int, default=50)
    ap.add_argument("--batch", type=int, default=None, help="batch size (default: the workload's)")
    ap.add_argument("--windows", default=None, help="comma-separated windows (0 = untruncated)")
    ap.add_argument("--precisions", default="fp32")
    ap.add_argument("--lrs", default="beta,sklearn")
    args = ap.parse_args(argv)
    wl = W.make(args.workload)
    windows = [int(w) for w in args.windows.split(",")] if args.windows else None
    for r in compare(wl, args.iterations, args.lrs.split(","), windows, args.precisions.split(","), args.batch):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
