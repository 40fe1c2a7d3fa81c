"""Agreement scores of a clustering with reference labels, as reported in
Section 6 of the paper (adjusted Rand index, normalised mutual information).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: plain numpy in FP64,
written from the definitions, for the tests to check the library against.

- contingency: n[i, j] = number of rows with label i and reference label j.
- ari: the Rand index counts pairs of rows that both labelings put together;
  the adjusted form subtracts its expectation under random labelings with the
  same cluster sizes and divides by (mean of the two together-pair counts
  minus that expectation).  Both labelings trivial in the same way (the
  denominator vanishes) gives 1.
- nmi: mutual information I(U; V) over the mean of the entropies
  (H(U) + H(V)) / 2, natural logarithms; 1 when both labelings are a single
  cluster.
"""
from __future__ import annotations

import numpy as np


def contingency(u, v, k: int, c: int) -> np.ndarray:
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    n = np.zeros((k, c), dtype=np.int64)
    np.add.at(n, (u, v), 1)
    return n


def _pairs(x):
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) / 2.0


def ari(n: np.ndarray) -> float:
    n = np.asarray(n, dtype=np.float64)
    total = n.sum()
    together_both = _pairs(n).sum()
    together_u = _pairs(n.sum(axis=1)).sum()
    together_v = _pairs(n.sum(axis=0)).sum()
    expected = together_u * together_v / _pairs(total)
    top = 0.5 * (together_u + together_v)
    if top == expected:
        return 1.0
    return float((together_both - expected) / (top - expected))


def _entropy(p):
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


def nmi(n: np.ndarray) -> float:
    n = np.asarray(n, dtype=np.float64)
    total = n.sum()
    pij = n / total
    pu, pv = pij.sum(axis=1), pij.sum(axis=0)
    hu, hv = _entropy(pu), _entropy(pv)
    if hu == 0.0 and hv == 0.0:
        return 1.0
    mi = 0.0
    for i, j in zip(*np.nonzero(n)):
        mi += pij[i, j] * np.log(pij[i, j] / (pu[i] * pv[j]))
    return float(max(mi, 0.0) / (0.5 * (hu + hv)))
