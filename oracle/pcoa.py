"""FP64 oracle for principal coordinates analysis of a distance matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes PCoA as part of the UniFrac job (section II) without
printing the method.  Classical PCoA (Gower's principal coordinates, i.e.
classical multidimensional scaling) is taken as the definition:

* A = -d^2 / 2 elementwise, B = J A J with J = I - 11^T / n (double centring);
  B_ij = A_ij - r_i - r_j + g with r the row means of A and g their mean;
* the eigenpairs (lambda_k, v_k) of B in decreasing order of lambda;
* coordinates v_k * sqrt(lambda_k) (zero where lambda_k <= 0);
* the sum of all eigenvalues is trace(B) = -n g.

``pcoa_exact`` is that definition (a full symmetric eigendecomposition).
``pcoa_randomized`` takes the steps of randomized subspace iteration with a
Rayleigh-Ritz projection (Halko, Martinsson and Tropp, "Finding structure
with randomness", SIAM Review 2011, Algorithms 4.4 and 5.3), the method a
top-k PCoA of a large matrix uses, on the explicit B, with library QR and
eigh as its steps.  The caller passes the Gaussian test matrix Omega.

Sign convention of an eigenvector (the decomposition fixes it only up to
sign): the entry of largest magnitude is made positive; among equal
magnitudes the first index counts.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def square(condensed: np.ndarray, n: int) -> np.ndarray:
    """Full symmetric n x n matrix from the condensed upper triangle (row major)."""
    d = np.zeros((n, n), dtype=np.float64)
    iu = np.triu_indices(n, 1)
    d[iu] = np.asarray(condensed, dtype=np.float64)
    return d + d.T


def centred(condensed: np.ndarray, n: int) -> np.ndarray:
    """B = J (-d^2/2) J, formed with the centring matrix J = I - 11^T/n."""
    a = -0.5 * square(condensed, n) ** 2
    j = np.eye(n) - np.full((n, n), 1.0 / n)
    return j @ a @ j


def fix_signs(v: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (first on ties)."""
    v = np.array(v, dtype=np.float64, copy=True)
    for k in range(v.shape[1]):
        i = int(np.argmax(np.abs(v[:, k])))
        if v[i, k] < 0:
            v[:, k] = -v[:, k]
    return v


def _coords(vals: np.ndarray, vecs: np.ndarray) -> np.ndarray:
    return fix_signs(vecs) * np.sqrt(np.maximum(vals, 0.0))


def pcoa_exact(condensed: np.ndarray, n: int, dims: int) -> Tuple[np.ndarray, np.ndarray, float]:
    """(eigenvalues[dims] decreasing, coordinates[n, dims], trace of B)."""
    b = centred(condensed, n)
    w, v = np.linalg.eigh(b)
    order = np.argsort(-w, kind="stable")[:dims]
    return w[order], _coords(w[order], v[:, order]), float(np.trace(b))


def pcoa_randomized(condensed: np.ndarray, n: int, dims: int, omega: np.ndarray,
                    power_iters: int) -> Tuple[np.ndarray, np.ndarray, float]:
    """Randomized subspace iteration on B with test matrix omega (n x l, l >= dims).

    Y = B Omega; Q = orth(Y); q times: Q = orth(B Q); then the Rayleigh-Ritz
    step T = Q^T B Q = W diag(lambda) W^T and V = Q W.  orth() keeps the
    directions of Y whose singular values exceed 1e-12 of the largest (a basis
    of the numerical range), so rank-deficient B is handled.
    """
    b = centred(condensed, n)

    def orth(y):
        u, s, _ = np.linalg.svd(y, full_matrices=False)
        keep = s > 1e-12 * s[0] if s.size and s[0] > 0 else np.zeros(0, dtype=bool)
        return u[:, keep]

    q = orth(b @ np.asarray(omega, dtype=np.float64))
    for _ in range(power_iters):
        q = orth(b @ q)
    t = q.T @ b @ q
    t = 0.5 * (t + t.T)
    w, wv = np.linalg.eigh(t)
    order = np.argsort(-w, kind="stable")[:dims]
    vals = w[order]
    vecs = q @ wv[:, order]
    if vals.size < dims:   # rank below dims: the remaining axes are zero
        vals = np.concatenate([vals, np.zeros(dims - vals.size)])
        vecs = np.concatenate([vecs, np.zeros((n, dims - vecs.shape[1]))], axis=1)
    return vals, _coords(vals, vecs), float(np.trace(b))
