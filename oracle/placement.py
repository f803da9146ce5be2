"""FP64 oracle of the learned placement encoder -- TEST INFRASTRUCTURE ONLY.

The paper's introduction motivates placing new sample collections into the
context of existing data.  The encoder that does it here is a map from a
sample's embedded proportions to a low-dimensional space whose Euclidean
distances approximate weighted-normalized UniFrac; exact UniFrac re-ranks its
nearest candidates.  Definitions written out plainly:

* projection: y_v = l_v u_v over the non-root branches (so ||y_a - y_b||_1 is
  the weighted-normalized numerator); x = R y with R[d, v] = sign/2 at the
  (node, dim) pairs drawn by ``synth.sparse_projection``.
* MLP: h_0 = x; h_l = relu(h_{l-1} W_l^T + b_l) for hidden layers; z = h_{L-1} W_L^T + b_L.
* loss over pairs (a, b) with target d: mean_p (w_p (||z_a - z_b||_2 - d_p))^2
  with w_p = 1 (absolute) or 1 / max(d_p, floor) (relative error).
* Adam with bias correction.
* kNN: exact squared Euclidean distances, ties broken by the smaller index.

``bf16_storage=True`` rounds the tensors the GPU stores in bfloat16 (inputs,
hidden activations, the loss gradient dZ and the hidden-layer gradients) at
the same points, everything else in FP64 -- the kernel's precision model.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import unifrac


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as FP64."""
    return unifrac._round_bf16_f64(np.asarray(x, dtype=np.float64))


def project(tree, table, dims, signs, out_dim: int, scale: float = 1.0) -> np.ndarray:
    """x[s] = scale * sum over non-root branches v of l_v u_sv * signs[v, j] / 2 at dims[v, j]."""
    u, a, length, nonroot = unifrac.embedding(tree, table)
    y = u * length[None, :]
    x = np.zeros((u.shape[0], out_dim))
    for j in range(dims.shape[1]):
        w = np.where(nonroot, signs[:, j].astype(np.float64) / 2.0, 0.0)
        for s in range(u.shape[0]):
            np.add.at(x[s], dims[:, j], y[s] * w)
    return x * scale


def forward(x: np.ndarray, params: Sequence[Tuple[np.ndarray, np.ndarray]], bf16_storage=False,
            skip=None):
    """Returns (hs, z): hs[0] = x, hs[l] = hidden activation l, z = output (FP64);
    skip: optional linear path S, z = MLP(x) + S x."""
    rnd = bf16 if bf16_storage else (lambda t: t)
    h = rnd(np.asarray(x, dtype=np.float64))
    hs = [h]
    L = len(params)
    for l, (w, b) in enumerate(params):
        a = h @ np.asarray(w, np.float64).T + np.asarray(b, np.float64)
        if l < L - 1:
            h = rnd(np.maximum(a, 0.0))
            hs.append(h)
        else:
            z = a
    if skip is not None:
        z = z + hs[0] @ np.asarray(skip, np.float64).T
    return hs, z


def loss_and_grads(x, params, pair_a, pair_b, target, bf16_storage=False, rel_floor=0.0,
                   skip=None):
    """Mean pair loss and its gradients [(dW_l, db_l)] (+ dS if skip) (FP64).

    rel_floor > 0: relative error, each pair weighted by 1 / max(d, rel_floor)."""
    rnd = bf16 if bf16_storage else (lambda t: t)
    rows = np.concatenate([pair_a, pair_b])
    hs, z = forward(np.asarray(x)[rows], params, bf16_storage, skip)
    p = len(pair_a)
    diff = z[:p] - z[p:]
    delta = np.sqrt((diff * diff).sum(axis=1))
    t = np.asarray(target, np.float64)
    w = 1.0 / np.maximum(t, rel_floor) if rel_floor > 0 else np.ones_like(t)
    r = (delta - t) * w
    loss = float(np.mean(r * r))
    coef = np.where(delta > 0, 2.0 * r * w / np.where(delta > 0, delta, 1.0), 0.0) / p
    dza = coef[:, None] * diff
    dz = rnd(np.concatenate([dza, -dza]))
    grads: List[Tuple[np.ndarray, np.ndarray]] = [None] * len(params)
    if skip is not None:
        grads.append((dz.T @ hs[0], None))
    g = dz
    for l in range(len(params) - 1, -1, -1):
        w = np.asarray(params[l][0], np.float64)
        grads[l] = (g.T @ hs[l], g.sum(axis=0))
        if l > 0:
            g = rnd((g @ w) * (hs[l] > 0))
    return loss, grads


def _backward(dz, hs, params, bf16_storage=False, skip=None):
    """Parameter gradients [(dW_l, db_l)] (+ (dS, None) if skip) for the output
    gradient dz of rows whose activations are hs (FP64)."""
    rnd = bf16 if bf16_storage else (lambda t: t)
    grads: List[Tuple[np.ndarray, np.ndarray]] = [None] * len(params)
    if skip is not None:
        grads.append((dz.T @ hs[0], None))
    g = dz
    for l in range(len(params) - 1, -1, -1):
        w = np.asarray(params[l][0], np.float64)
        grads[l] = (g.T @ hs[l], g.sum(axis=0))
        if l > 0:
            g = rnd((g @ w) * (hs[l] > 0))
    return grads


def softplus(x):
    """log(1 + e^x), without overflow."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def triplet_loss_and_grads(x, params, anchor, near, far, d_near, d_far, rank_weight, tau,
                           bf16_storage=False, skip=None, dist_weight=1.0):
    """Mean over triples (a, p, n) of the distance-regression terms of both pairs
    plus a ranking term that asks the encoder to place p closer to a than n:

        e_p = ||z_a - z_p||,  e_n = ||z_a - z_n||
        L = mean_t [ alpha ((e_p - d_p)^2 + (e_n - d_n)^2)
                     + lam * tau * softplus((e_p - e_n) / tau) ]

    (alpha = dist_weight, lam = rank_weight, tau = temperature).  Returns
    (loss, grads) as loss_and_grads does; rows are anchors, then near ends, then
    far ends."""
    rnd = bf16 if bf16_storage else (lambda t: t)
    rows = np.concatenate([anchor, near, far])
    hs, z = forward(np.asarray(x)[rows], params, bf16_storage, skip)
    T = len(anchor)
    za, zp, zn = z[:T], z[T:2 * T], z[2 * T:]
    dap, dan = za - zp, za - zn
    ep = np.sqrt((dap * dap).sum(axis=1))
    en = np.sqrt((dan * dan).sum(axis=1))
    tp, tn = np.asarray(d_near, np.float64), np.asarray(d_far, np.float64)
    s = (ep - en) / tau
    loss = float(np.mean(dist_weight * ((ep - tp) ** 2 + (en - tn) ** 2) +
                         rank_weight * tau * softplus(s)))
    # dL/de_p and dL/de_n of each triple (divided by T for the mean)
    gp = (2.0 * dist_weight * (ep - tp) + rank_weight * sigmoid(s)) / T
    gn = (2.0 * dist_weight * (en - tn) - rank_weight * sigmoid(s)) / T
    cp = np.where(ep > 0, gp / np.where(ep > 0, ep, 1.0), 0.0)[:, None] * dap
    cn = np.where(en > 0, gn / np.where(en > 0, en, 1.0), 0.0)[:, None] * dan
    dz = rnd(np.concatenate([cp + cn, -cp, -cn]))
    return loss, _backward(dz, hs, params, bf16_storage, skip)


def triplet_loss_only(x, params, anchor, near, far, d_near, d_far, rank_weight, tau,
                      skip=None, dist_weight=1.0) -> float:
    return triplet_loss_and_grads(x, params, anchor, near, far, d_near, d_far, rank_weight, tau,
                                  skip=skip, dist_weight=dist_weight)[0]


def loss_only(x, params, pair_a, pair_b, target, rel_floor=0.0) -> float:
    return loss_and_grads(x, params, pair_a, pair_b, target, rel_floor=rel_floor)[0]


def adam(param, grad, m, v, lr, b1, b2, eps, step, weight_decay=0.0):
    """One Adam update (FP64) with decoupled weight decay; returns (param, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return param - lr * (mh / (np.sqrt(vh) + eps) + weight_decay * param), m, v


def pca_basis(x, k: int):
    """Top-k principal directions of the rows of x: eigenvectors of the covariance
    (1/n) (x - mean)^T (x - mean) with the k largest eigenvalues, returned as
    (basis [k][d], eigenvalues [k]) in descending order (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    xc = x - x.mean(axis=0, keepdims=True)
    cov = xc.T @ xc / x.shape[0]
    w, v = np.linalg.eigh(cov)
    order = np.argsort(-w, kind="stable")[:k]
    return v[:, order].T, w[order]


def knn(zq: np.ndarray, zr: np.ndarray, k: int):
    """Exact k nearest references per query (squared Euclidean, ties -> smaller index)."""
    d = ((zq[:, None, :].astype(np.float64) - zr[None, :, :]) ** 2).sum(axis=2)
    idx = np.lexsort((np.broadcast_to(np.arange(zr.shape[0]), d.shape), d), axis=1)[:, :k]
    return idx, np.take_along_axis(d, idx, axis=1)


def topk_rows(values: np.ndarray, k: int):
    """k smallest per row, ties -> smaller column index."""
    v = np.asarray(values, dtype=np.float64)
    cols = np.broadcast_to(np.arange(v.shape[1]), v.shape)
    idx = np.lexsort((cols, v), axis=1)[:, :k]
    return idx, np.take_along_axis(v, idx, axis=1)


def recall_at_k(found: np.ndarray, exact_d: np.ndarray, k: int) -> float:
    """Tie-tolerant recall: found[q] (k reference ids) counts a hit when its
    exact distance is <= the exact k-th smallest distance of row q."""
    kth = np.sort(exact_d, axis=1)[:, k - 1]
    got = np.take_along_axis(exact_d, found, axis=1)
    return float(np.mean(got <= kth[:, None] + 0.0))
