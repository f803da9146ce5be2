"""Pins of the PCoA oracle (oracle/pcoa.py) against closed forms and invariants.

* equilateral triangle of side s: the centred matrix has eigenvalues s^2/2,
  s^2/2, 0 (three points at radius s/sqrt(3), hand derivation);
* Euclidean points X: B equals Xc Xc^T (Xc centred), so the nonzero
  eigenvalues are those of the small matrix Xc^T Xc and the coordinates
  reproduce every pairwise distance;
* trace(B) = sum_{i<j} d_ij^2 / n, summed independently;
* the randomized method with a full-width test matrix is exact; with a
  narrow one it converges on the top eigenvalues of a UniFrac matrix.
"""
import numpy as np
import pytest

import synth
from oracle import core
from oracle import pcoa


def _condensed(points):
    n = points.shape[0]
    iu = np.triu_indices(n, 1)
    diff = points[:, None, :] - points[None, :, :]
    return np.sqrt((diff ** 2).sum(-1))[iu]


def test_equilateral_triangle():
    s = 1.7
    vals, coords, tr = pcoa.pcoa_exact(np.array([s, s, s]), 3, 3)
    assert np.allclose(vals, [s * s / 2, s * s / 2, 0.0], atol=1e-12)
    assert abs(tr - s * s) < 1e-12          # 3 pairs * s^2 / 3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_euclidean_points_recovered(seed):
    rng = np.random.default_rng(seed)
    n, k = 40, 3
    x = rng.normal(size=(n, k)) * np.array([5.0, 2.0, 0.5]) + rng.normal(size=k) * 10
    d = _condensed(x)
    vals, coords, tr = pcoa.pcoa_exact(d, n, 6)
    xc = x - x.mean(axis=0)
    want = np.sort(np.linalg.eigvalsh(xc.T @ xc))[::-1]
    assert np.allclose(vals[:k], want, rtol=1e-10)
    assert np.all(np.abs(vals[k:]) < 1e-8 * want[0])
    assert np.allclose(_condensed(coords[:, :k]), d, atol=1e-9)
    assert abs(tr - want.sum()) < 1e-9 * want.sum()


def test_trace_closed_form():
    rng = np.random.default_rng(5)
    n = 30
    d = rng.uniform(0, 1, size=n * (n - 1) // 2)
    _, _, tr = pcoa.pcoa_exact(d, n, 2)
    total = 0.0
    for v in d:
        total += v * v
    assert abs(tr - total / n) < 1e-12 * max(1.0, total)


def test_sign_convention():
    rng = np.random.default_rng(7)
    n = 25
    d = rng.uniform(0, 1, size=n * (n - 1) // 2)
    _, coords, _ = pcoa.pcoa_exact(d, n, 4)
    for k in range(4):
        i = int(np.argmax(np.abs(coords[:, k])))
        assert coords[i, k] > 0


@pytest.fixture(scope="module")
def c1_weighted():
    tree, table = synth.config("C1", n_samples=160)
    d = core.dm(tree, table, "weighted_normalized")[0]
    return d, table.n_samples


def test_randomized_full_width_is_exact(c1_weighted):
    d, n = c1_weighted
    omega = np.random.default_rng(3).normal(size=(n, n))
    v1, c1, t1 = pcoa.pcoa_randomized(d, n, 8, omega, power_iters=0)
    v0, c0, t0 = pcoa.pcoa_exact(d, n, 8)
    assert np.allclose(v1, v0, rtol=1e-10, atol=1e-12 * abs(v0[0]))
    assert np.allclose(np.abs(c1), np.abs(c0), atol=1e-8)
    assert t1 == pytest.approx(t0, rel=1e-14)


def test_randomized_converges_on_top_eigenvalues(c1_weighted):
    """UniFrac spectra decay slowly (C1: 3.26, 2.04, 1.71, 1.24, ...), so the
    subspace iteration converges geometrically in the number of passes; the
    Ritz values approach the true eigenvalues from below."""
    d, n = c1_weighted
    v0, _, _ = pcoa.pcoa_exact(d, n, 5)
    errs = []
    for q in range(6):
        omega = np.random.default_rng(4).normal(size=(n, 20))
        v1, _, _ = pcoa.pcoa_randomized(d, n, 5, omega, power_iters=q)
        assert np.all(v1 <= v0 * (1 + 1e-12) + 1e-15)
        errs.append(np.abs(v1[:3] - v0[:3]) / v0[:3])
    for a, b in zip(errs, errs[1:]):
        assert np.all(b <= a * 1.0000001)
    assert np.all(errs[-1] < 1e-6)


def test_randomized_rank_deficient():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(30, 2))
    d = _condensed(x)
    omega = rng.normal(size=(30, 8))
    v1, c1, _ = pcoa.pcoa_randomized(d, 30, 4, omega, power_iters=1)
    v0, c0, _ = pcoa.pcoa_exact(d, 30, 4)
    assert np.allclose(v1[:2], v0[:2], rtol=1e-10)
    assert np.all(np.abs(v1[2:]) < 1e-8 * v0[0])
    assert np.allclose(_condensed(c1[:, :2]), d, atol=1e-9)
