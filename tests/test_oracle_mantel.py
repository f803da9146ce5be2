"""Pins of the Mantel oracle (oracle/mantel.py).

* Pearson and Spearman statistics against scipy.stats (a separate library
  implementation);
* closed forms: y = a x + b gives r = 1 (a > 0) or -1 (a < 0); Spearman is 1
  for any increasing transform;
* average ranks with ties against scipy.stats.rankdata;
* the permuted condensed form against a direct double loop;
* p-values against exhaustive enumeration of all 4! relabellings of a 4-sample
  matrix, for all three alternatives; the identity permutation gives r itself.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import mantel as om


def _rand_dm(n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.normal(size=(n, 3))
    iu = np.triu_indices(n, 1)
    return np.sqrt(((pts[:, None] - pts[None]) ** 2).sum(-1))[iu]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_statistics_match_scipy(seed):
    x = _rand_dm(30, seed)
    y = x + np.random.default_rng(seed + 10).normal(scale=0.3, size=x.size)
    assert om.pearson(x, y) == pytest.approx(stats.pearsonr(x, y)[0], abs=1e-13)
    rx, ry = om.average_ranks(x), om.average_ranks(y)
    assert om.pearson(rx, ry) == pytest.approx(stats.spearmanr(x, y)[0], abs=1e-13)


def test_closed_forms():
    x = _rand_dm(20, 4)
    assert om.pearson(x, 3.0 * x + 2.0) == pytest.approx(1.0, abs=1e-14)
    assert om.pearson(x, -0.5 * x + 9.0) == pytest.approx(-1.0, abs=1e-14)
    ex = np.exp(x)
    assert om.pearson(om.average_ranks(x), om.average_ranks(ex)) == pytest.approx(1.0, abs=1e-14)


def test_average_ranks_ties():
    v = np.array([3.0, 1.0, 3.0, 2.0, 3.0, 1.0, 7.0])
    assert np.array_equal(om.average_ranks(v), stats.rankdata(v, method="average"))


def test_permuted_condensed():
    n = 7
    x = _rand_dm(n, 5)
    perm = np.random.default_rng(6).permutation(n)
    full = np.zeros((n, n))
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            full[i, j] = full[j, i] = x[k]
            k += 1
    want = [full[perm[i], perm[j]] for i in range(n) for j in range(i + 1, n)]
    assert np.array_equal(om.permuted_condensed(x, n, perm), np.array(want))


@pytest.mark.parametrize("method", ["pearson", "spearman"])
@pytest.mark.parametrize("alternative", ["two-sided", "greater", "less"])
def test_exhaustive_p_value(method, alternative):
    n = 4
    x = np.array([1.0, 4.0, 2.0, 6.0, 3.0, 5.0])
    y = np.array([2.0, 3.0, 1.0, 5.0, 4.0, 6.0])
    perms = np.array(list(itertools.permutations(range(n))))
    r, p, st = om.mantel(x, y, n, method, perms, alternative)
    if method == "spearman":
        x, y = om.average_ranks(x), om.average_ranks(y)
    assert st[0] == pytest.approx(r, abs=1e-15)          # identity first
    # brute force over the 24 relabellings
    full = np.zeros((n, n))
    full[np.triu_indices(n, 1)] = x
    full = full + full.T
    vals = []
    for pm in itertools.permutations(range(n)):
        xp = [full[pm[i], pm[j]] for i in range(n) for j in range(i + 1, n)]
        vals.append(np.corrcoef(xp, y)[0, 1])
    vals = np.array(vals)
    if alternative == "two-sided":
        c = np.sum(np.abs(vals) >= abs(r) - 1e-12)
    elif alternative == "greater":
        c = np.sum(vals >= r - 1e-12)
    else:
        c = np.sum(vals <= r + 1e-12)
    assert p == pytest.approx((c + 1) / 25)
    assert 1 / 25 <= p <= 1.0
