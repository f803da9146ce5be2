"""FP64 oracle for the Mantel test between two distance matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (section III) uses the Mantel test to ask whether two distance
matrices are correlated, with Pearson's or Spearman's coefficient and a
non-parametric (permutation) p-value, without writing the procedure out.
The standard procedure is taken as the definition:

* x, y: the condensed (upper-triangle) forms of the two matrices;
* statistic r = Pearson correlation of x and y; Spearman's is Pearson's on
  the ranks of x and of y (ties get the average of their ranks);
* each permutation pi reorders the samples of the first matrix, rows and
  columns together: x'_ij = x_{pi(i) pi(j)}; r_pi = the same statistic on x', y;
* p = (#{permutations at least as extreme} + 1) / (permutations + 1), where
  "at least as extreme" is |r_pi| >= |r| (two-sided), r_pi >= r (greater) or
  r_pi <= r (less).

The permutations are inputs (rows of an int array), drawn by the caller.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

ALTERNATIVES = ("two-sided", "greater", "less")


def pearson(x: np.ndarray, y: np.ndarray) -> float:
    """sum (x - mean x)(y - mean y) / sqrt(sum (x - mean x)^2 sum (y - mean y)^2)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xc = x - x.mean()
    yc = y - y.mean()
    den = np.sqrt((xc * xc).sum() * (yc * yc).sum())
    return float((xc * yc).sum() / den) if den > 0 else 0.0


def average_ranks(v: np.ndarray) -> np.ndarray:
    """Ranks 1..m of v in increasing order; a run of equal values shares the
    mean of the ranks it spans."""
    v = np.asarray(v, dtype=np.float64)
    order = np.argsort(v, kind="stable")
    sv = v[order]
    ranks = np.empty(v.size, dtype=np.float64)
    start = 0
    m = v.size
    while start < m:
        end = start
        while end + 1 < m and sv[end + 1] == sv[start]:
            end += 1
        ranks[order[start:end + 1]] = 0.5 * (start + end) + 1.0
        start = end + 1
    return ranks


def permuted_condensed(x: np.ndarray, n: int, perm: np.ndarray) -> np.ndarray:
    """Condensed form of x'_ij = x_{perm(i) perm(j)}."""
    full = np.zeros((n, n), dtype=np.float64)
    iu = np.triu_indices(n, 1)
    full[iu] = x
    full = full + full.T
    p = np.asarray(perm, dtype=np.int64)
    return full[np.ix_(p, p)][iu]


def mantel(x: np.ndarray, y: np.ndarray, n: int, method: str, perms: np.ndarray,
           alternative: str = "two-sided") -> Tuple[float, float, np.ndarray]:
    """(statistic, p-value, statistics of each permutation)."""
    if method not in ("pearson", "spearman"):
        raise ValueError("method must be pearson or spearman")
    if alternative not in ALTERNATIVES:
        raise ValueError("unknown alternative")
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if method == "spearman":
        x = average_ranks(x)
        y = average_ranks(y)
    r = pearson(x, y)
    stats = np.array([pearson(permuted_condensed(x, n, p), y) for p in perms], dtype=np.float64)
    if alternative == "two-sided":
        count = int(np.sum(np.abs(stats) >= abs(r)))
    elif alternative == "greater":
        count = int(np.sum(stats >= r))
    else:
        count = int(np.sum(stats <= r))
    return r, (count + 1) / (len(stats) + 1), stats
