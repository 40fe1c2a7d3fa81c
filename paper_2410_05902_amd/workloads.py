"""Seeded synthetic workloads for mini-batch kernel k-means.

This module only draws inputs: data matrices, batch index tuples, initial
indices, the uniforms that kernel k-means++ consumes, and the Gaussian
bandwidth set by the median heuristic.  It holds none of the method's
arithmetic (no kernel evaluation, no distance, no center update), so both the
HIP path and the FP64 CPU oracle can draw from it without sharing any code
that computes a result.

The paper evaluates on MNIST (70000 x 784, 10 classes), PenDigits, Letters and
HAR (Section 6).  None of these datasets is available here; the workloads below
are synthetic stand-ins with the shapes and structure of those experiments, and
the larger shapes of the scaling configurations.

All randomness comes from numpy ``Generator(PCG64)`` streams derived from one
seed through ``SeedSequence``; independent streams are used for the data, the
bandwidth sample, the initial centers and the batches, so that e.g. changing
the number of steps never changes the data.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Kernel families.  The numbering is the one used by the C ABI (include/mbkk.h)
# and by the oracle; it is a plain enumeration, not arithmetic.
GAUSS = 0     # K(x,y) = exp(-||x-y||_2^2 / kappa)          (Section 6)
LAPLACE = 1   # K(x,y) = exp(-||x-y||_1 / sigma)            (named in the abstract)
LINEAR = 2    # K(x,y) = <x,y>                               (test kernel)
POLY2 = 3     # K(x,y) = (<x,y> + c)^2                       (test kernel)

# Learning-rate rules.
LR_BETA = 0      # alpha = sqrt(b_i^j / b)   (Section 5, rate of Schwartzman 2023)
LR_FULL = 1      # alpha = 1 if b_i^j > 0     (b = n reduces the method to Lloyd)
LR_SKLEARN = 2   # alpha = b_i^j / sum_{l<=i} b_l^j  (count-based rate, goes to 0)

_STREAM_DATA, _STREAM_SIGMA, _STREAM_INIT, _STREAM_BATCH = 1, 2, 3, 4


def _rng(seed: int, *stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *stream])))


@dataclasses.dataclass
class Workload:
    """One configuration: data, kernel, window and batch geometry."""

    name: str
    X: np.ndarray            # (n, d) float32, C-contiguous
    comp: np.ndarray         # (n,) int32 generating component of each row
    k: int
    b: int
    window: int              # W: centers keep their last W batches (0 = all)
    kernel: int
    kernel_param: float      # kappa (GAUSS), sigma (LAPLACE), c (POLY2)
    sigma: Optional[float]   # bandwidth before conversion, where one exists
    seed: int
    iterations: int = 20
    lr: int = LR_BETA

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    def batch(self, i: int, b: Optional[int] = None) -> np.ndarray:
        """Batch B_i: b indices drawn uniformly with repetition (Algorithm 1)."""
        return batch_indices(self.seed, i, self.n, self.b if b is None else b)

    def kmeanspp_uniforms(self) -> np.ndarray:
        return kmeanspp_uniforms(self.seed, self.k)

    def random_init(self) -> np.ndarray:
        return random_init(self.seed, self.n, self.k)


def batch_indices(seed: int, i: int, n: int, b: int) -> np.ndarray:
    """Indices of batch i (1-based): uniform over [0, n) with repetition."""
    return _rng(seed, _STREAM_BATCH, int(i)).integers(0, n, size=b, dtype=np.int64).astype(np.int32)


def kmeanspp_uniforms(seed: int, k: int) -> np.ndarray:
    """The k uniforms in [0, 1) that one run of k-means++ consumes, one per pick."""
    return _rng(seed, _STREAM_INIT, 0).random(k)


def random_init(seed: int, n: int, k: int) -> np.ndarray:
    """k distinct indices, uniformly at random (used where k-means++ is too slow
    for the single-threaded oracle)."""
    return _rng(seed, _STREAM_INIT, 1).choice(n, size=k, replace=False).astype(np.int32)


def median_pairwise_distance(X: np.ndarray, seed: int, m: int = 1000) -> float:
    """Median heuristic for the Gaussian bandwidth: m rows sampled without
    replacement, the median of all m(m-1)/2 Euclidean distances between them."""
    m = min(m, X.shape[0])
    rows = _rng(seed, _STREAM_SIGMA).choice(X.shape[0], size=m, replace=False)
    Y = X[rows].astype(np.float64)
    sq = (Y * Y).sum(1)
    g = Y @ Y.T
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * g, 0.0)
    iu = np.triu_indices(m, 1)
    return float(np.median(np.sqrt(d2[iu])))


def _shuffle(X: np.ndarray, comp: np.ndarray, rng: np.random.Generator):
    perm = rng.permutation(X.shape[0])
    return np.ascontiguousarray(X[perm]), np.ascontiguousarray(comp[perm])


def _sizes(n: int, c: int) -> np.ndarray:
    base = np.full(c, n // c, dtype=np.int64)
    base[: n - base.sum()] += 1
    return base


def gaussian_blobs(n: int, d: int, c: int, means: np.ndarray, std: float,
                   rng: np.random.Generator):
    sizes = _sizes(n, c)
    comp = np.repeat(np.arange(c, dtype=np.int32), sizes)
    X = means[comp] + std * rng.standard_normal((n, d))
    return _shuffle(X.astype(np.float32), comp, rng)


def c1_blobs(seed: int = 0, n: int = 2000) -> Workload:
    """Three isotropic 2-D blobs, means U[-5,5]^2, std 1, equal sizes; k=3,
    b=256, Gaussian sigma=1 (kappa=2 sigma^2), last 4 batches, 20 iterations."""
    rng = _rng(seed, _STREAM_DATA)
    means = rng.uniform(-5.0, 5.0, size=(3, 2))
    X, comp = gaussian_blobs(n, 2, 3, means, 1.0, rng)
    sigma = 1.0
    return Workload("blobs2d_n2000_k3_b256", X, comp, k=3, b=256, window=4, kernel=GAUSS,
                    kernel_param=2.0 * sigma * sigma, sigma=sigma, seed=seed, iterations=20)


def c2_sparse_prototypes(seed: int = 0, n: int = 70000, d: int = 784) -> Workload:
    """MNIST-shaped stand-in: 10 random sparse prototypes (20% of coordinates
    U[0,1]), points = prototype + N(0, 0.1^2) noise clipped to [0,1]; k=10,
    b=1024, Gaussian with the median heuristic, last 8 batches."""
    rng = _rng(seed, _STREAM_DATA)
    c = 10
    protos = np.zeros((c, d))
    nnz = int(round(0.2 * d))
    for j in range(c):
        cols = rng.choice(d, size=nnz, replace=False)
        protos[j, cols] = rng.uniform(0.0, 1.0, size=nnz)
    sizes = _sizes(n, c)
    comp = np.repeat(np.arange(c, dtype=np.int32), sizes)
    X = np.clip(protos[comp] + 0.1 * rng.standard_normal((n, d)), 0.0, 1.0).astype(np.float32)
    X, comp = _shuffle(X, comp, rng)
    sigma = median_pairwise_distance(X, seed)
    return Workload(f"sparseproto_n{n}_d{d}_k10_b1024", X, comp, k=c, b=1024, window=8,
                    kernel=GAUSS, kernel_param=2.0 * sigma * sigma, sigma=sigma, seed=seed)


def c3_gaussian_mixture(seed: int = 0, n: int = 1_000_000, d: int = 128, c: int = 100,
                        b: int = 4096) -> Workload:
    """100 Gaussian components in 128-D, means N(0, I), std 0.3; k=100, b=4096,
    Gaussian kernel with the median heuristic, last 4 batches."""
    rng = _rng(seed, _STREAM_DATA)
    means = rng.standard_normal((c, d))
    X, comp = gaussian_blobs(n, d, c, means, 0.3, rng)
    sigma = median_pairwise_distance(X, seed)
    return Workload(f"gmm_n{n}_d{d}_k{c}_b{b}", X, comp, k=c, b=b, window=4, kernel=GAUSS,
                    kernel_param=2.0 * sigma * sigma, sigma=sigma, seed=seed)


def c4_gaussian_mixture(seed: int = 0, n: int = 100_000, d: int = 64, c: int = 50,
                        b: int = 2048) -> Workload:
    """50 components in 64-D, means N(0, 2I), std 0.5; k=50, b=2048, Gaussian
    kernel with the median heuristic, last 4 batches (differentiation form)."""
    rng = _rng(seed, _STREAM_DATA)
    means = np.sqrt(2.0) * rng.standard_normal((c, d))
    X, comp = gaussian_blobs(n, d, c, means, 0.5, rng)
    sigma = median_pairwise_distance(X, seed)
    return Workload(f"gmm_n{n}_d{d}_k{c}_b{b}", X, comp, k=c, b=b, window=4, kernel=GAUSS,
                    kernel_param=2.0 * sigma * sigma, sigma=sigma, seed=seed)


def c5_laplace_mixture(seed: int = 0, n: int = 4_000_000, d: int = 32, c: int = 1000,
                       b: int = 8192) -> Workload:
    """1000 components in 32-D, means U[-10,10]^32, std 0.4; k=1000, b=8192,
    Laplacian kernel exp(-||x-y||_1 / 4), last 4 batches."""
    rng = _rng(seed, _STREAM_DATA)
    means = rng.uniform(-10.0, 10.0, size=(c, d))
    X, comp = gaussian_blobs(n, d, c, means, 0.4, rng)
    return Workload(f"l1mix_n{n}_d{d}_k{c}_b{b}", X, comp, k=c, b=b, window=4, kernel=LAPLACE,
                    kernel_param=4.0, sigma=4.0, seed=seed)


CONFIGS = {
    "c1": c1_blobs,
    "c2": c2_sparse_prototypes,
    "c3": c3_gaussian_mixture,
    "c4": c4_gaussian_mixture,
    "c5": c5_laplace_mixture,
}


def make(name: str, **kw) -> Workload:
    return CONFIGS[name](**kw)
