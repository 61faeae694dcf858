"""Seeded matrix-completion instances (the recipe of the matrix completion
experiments of Sec. 6): ground truth M = U V^T with U (n1 x r) and V (n2 x r)
i.i.d. standard Gaussian, and m = ceil(gamma r (n - r)) entries observed
uniformly at random without repetition, n = n1 + n2, gamma = r log n.

Only data is drawn here: the observed values are entries of the ground truth.
"""

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Completion:
    n1: int
    n2: int
    r: int
    U: np.ndarray     # n1 x r
    V: np.ndarray     # n2 x r
    rows: np.ndarray  # int64, sorted by (row, col), unique pairs
    cols: np.ndarray  # int64
    vals: np.ndarray  # float64, M[rows, cols]

    @property
    def n(self) -> int:
        return self.n1 + self.n2

    @property
    def m(self) -> int:
        return int(self.rows.shape[0])


def sample_count(n1, n2, r):
    """m = ceil(gamma r (n - r)) with gamma = r log(n1 + n2), at most n1 n2."""
    n = n1 + n2
    return int(min(n1 * n2, math.ceil(r * math.log(n) * r * (n - r))))


def completion_instance(n1, n2, r, seed, m=None):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n1, r))
    V = rng.standard_normal((n2, r))
    total = n1 * n2
    m = sample_count(n1, n2, r) if m is None else int(min(m, total))
    if m > total // 2:
        keys = np.sort(rng.choice(total, size=m, replace=False)).astype(np.int64)
    else:
        keys = np.unique(rng.integers(0, total, size=m + m // 8 + 16, dtype=np.int64))
        while keys.shape[0] < m:
            keys = np.unique(np.concatenate([keys, rng.integers(0, total, size=m, dtype=np.int64)]))
        keys = np.sort(rng.choice(keys, size=m, replace=False))
    rows = keys // n2
    cols = keys % n2
    vals = np.einsum("ij,ij->i", U[rows], V[cols])
    return Completion(n1, n2, r, U, V, rows, cols, vals)
