"""Plain FP64 definitions of the UniFrac distances (test oracle only).

The paper (section II) names the measure and its two variants -- unweighted and
weighted normalized -- and says they are computed "striped" over all sample
pairs; it does not print the formulas.  The definitions used here are the
standard ones of the UniFrac literature, restated:

* A rooted tree with root r; every other node v has a branch of length
  l_v >= 0 to its parent.  The root has no branch (its length is ignored).
* Sample s has integer counts x[s, t] >= 0 on the tips t, total T_s > 0.
* Embedded count of node v: c[s, v] = sum of x[s, t] over tips t under v
  (v itself if v is a tip).  Proportion u[s, v] = c[s, v] / T_s.
  Presence a[s, v] = 1 if c[s, v] > 0 else 0 (decided on the integer count).
* unweighted:          d_U(i, j) = sum_v l_v |a_iv - a_jv| / sum_v l_v max(a_iv, a_jv)
* weighted normalized: d_W(i, j) = sum_v l_v |u_iv - u_jv| / sum_v l_v (u_iv + u_jv)
  (sums over non-root v).  A zero denominator gives d = 0.

Everything is FP64 and written for clarity, not speed.
"""
from __future__ import annotations

from typing import Iterable, Tuple

import numpy as np


class TreeError(ValueError):
    pass


class TableError(ValueError):
    pass


# ---------------------------------------------------------------------------
# tree
# ---------------------------------------------------------------------------
def validate_tree(parent, length) -> Tuple[np.ndarray, np.ndarray, int]:
    """Check a parent-array tree; return (parent, length, root).

    Exactly one root (parent -1); every other parent id in range; lengths of
    non-root nodes finite and >= 0; every node reachable from the root (which
    also rules out cycles).
    """
    parent = np.asarray(parent, dtype=np.int64)
    length = np.asarray(length, dtype=np.float64)
    m = parent.shape[0]
    if m < 1 or length.shape != (m,):
        raise TreeError("parent/length shape mismatch or empty tree")
    roots = np.nonzero(parent == -1)[0]
    if roots.size != 1:
        raise TreeError("tree must have exactly one root")
    root = int(roots[0])
    others = np.arange(m) != root
    if np.any((parent[others] < 0) | (parent[others] >= m)):
        raise TreeError("parent id out of range")
    if np.any(parent[others] == np.arange(m)[others]):
        raise TreeError("node is its own parent")
    lo = length[others]
    if np.any(~np.isfinite(lo)) or np.any(lo < 0):
        raise TreeError("branch lengths must be finite and >= 0")
    order = postorder(parent, root)
    if order.shape[0] != m:
        raise TreeError("tree is not connected (or has a cycle)")
    return parent, length, root


def _children(parent: np.ndarray):
    m = parent.shape[0]
    kids = [[] for _ in range(m)]
    for v in range(m):               # children kept in increasing id order
        p = int(parent[v])
        if p >= 0:
            kids[p].append(v)
    return kids


def postorder(parent, root=None) -> np.ndarray:
    """Iterative depth-first postorder (children before parents, root last)."""
    parent = np.asarray(parent, dtype=np.int64)
    if root is None:
        root = int(np.nonzero(parent == -1)[0][0])
    kids = _children(parent)
    out = []
    stack = [(root, 0)]
    seen = 0
    while stack:
        v, k = stack.pop()
        if k < len(kids[v]):
            stack.append((v, k + 1))
            stack.append((kids[v][k], 0))
            seen += 1
            if seen > parent.shape[0]:
                break
        else:
            out.append(v)
    return np.asarray(out, dtype=np.int64)


def tips_of(parent) -> np.ndarray:
    """Boolean mask of the tips (nodes without children)."""
    parent = np.asarray(parent, dtype=np.int64)
    has_child = np.zeros(parent.shape[0], dtype=bool)
    has_child[parent[parent >= 0]] = True
    return ~has_child


# ---------------------------------------------------------------------------
# table + embedding
# ---------------------------------------------------------------------------
def _dense_counts(parent, indptr, tips, counts) -> np.ndarray:
    """Validate the CSR table and return dense counts [n_samples, n_nodes]."""
    parent = np.asarray(parent, dtype=np.int64)
    indptr = np.asarray(indptr, dtype=np.int64)
    tips = np.asarray(tips, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    m = parent.shape[0]
    n = indptr.shape[0] - 1
    if n < 0 or indptr[0] != 0 or np.any(np.diff(indptr) < 0) or \
            indptr[-1] != tips.shape[0] or tips.shape != counts.shape:
        raise TableError("malformed CSR table")
    is_tip = tips_of(parent)
    if np.any((tips < 0) | (tips >= m)):
        raise TableError("feature id out of range")
    if not np.all(is_tip[tips]):
        raise TableError("feature mapped to an internal node")
    if np.any(counts < 0):
        raise TableError("negative count")
    x = np.zeros((n, m), dtype=np.int64)
    for s in range(n):
        a, b = int(indptr[s]), int(indptr[s + 1])
        t = tips[a:b]
        if np.unique(t).shape[0] != t.shape[0]:
            raise TableError("duplicate feature in a sample")
        x[s, t] = counts[a:b]
    if np.any(x.sum(axis=1) <= 0):
        raise TableError("sample with zero total count")
    return x


def embed_counts(tree, table) -> Tuple[np.ndarray, np.ndarray]:
    """Embedded counts c[s, v] (int64) by a postorder pass, and totals T_s."""
    parent, _, root = validate_tree(tree.parent, tree.length)
    c = _dense_counts(parent, table.indptr, table.tips, table.counts)
    for v in postorder(parent, root):
        p = int(parent[v])
        if p >= 0:
            c[:, p] += c[:, v]
    return c, c[:, root].copy()


def embedding(tree, table):
    """(u, a, l, nonroot): proportions, presence, lengths, non-root mask."""
    parent, length, root = validate_tree(tree.parent, tree.length)
    c, total = embed_counts(tree, table)
    u = c.astype(np.float64) / total.astype(np.float64)[:, None]
    a = (c > 0).astype(np.float64)
    nonroot = np.arange(parent.shape[0]) != root
    return u, a, length, nonroot


def _pair_terms(u, a, l, i, j, variant):
    if variant == "unweighted":
        num = np.sum(l * np.abs(a[i] - a[j]))
        den = np.sum(l * np.maximum(a[i], a[j]))
    elif variant == "weighted_normalized":
        num = np.sum(l * np.abs(u[i] - u[j]))
        den = np.sum(l * (u[i] + u[j]))
    else:
        raise ValueError("variant must be 'unweighted' or 'weighted_normalized'")
    return num, den


def dm(tree, table, variant: str) -> np.ndarray:
    """Full distance matrix in condensed order (row-major upper triangle)."""
    u, a, length, nonroot = embedding(tree, table)
    u, a, l = u[:, nonroot], a[:, nonroot], length[nonroot]
    n = u.shape[0]
    out = np.zeros(n * (n - 1) // 2, dtype=np.float64)
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            num, den = _pair_terms(u, a, l, i, j, variant)
            out[k] = num / den if den > 0 else 0.0
            k += 1
    return out


def dm_pairs(tree, table, pairs: Iterable[Tuple[int, int]], variant: str) -> np.ndarray:
    """Distances for a list of (i, j) sample pairs, embedding only those samples."""
    import synth  # input plumbing only (row subset); no method arithmetic
    pairs = np.asarray(list(pairs), dtype=np.int64).reshape(-1, 2)
    rows = np.unique(pairs.reshape(-1))
    sub = synth.subset_rows(table, rows)
    u, a, length, nonroot = embedding(tree, sub)
    u, a, l = u[:, nonroot], a[:, nonroot], length[nonroot]
    pos = {int(r): k for k, r in enumerate(rows)}
    out = np.zeros(pairs.shape[0], dtype=np.float64)
    for k, (i, j) in enumerate(pairs):
        num, den = _pair_terms(u, a, l, pos[int(i)], pos[int(j)], variant)
        out[k] = num / den if den > 0 else 0.0
    return out


# ---------------------------------------------------------------------------
# output layouts and PCoA inputs
# ---------------------------------------------------------------------------
def condensed_index(n: int, i: int, j: int) -> int:
    """Position of pair (i, j), i != j, in the row-major upper triangle."""
    if i > j:
        i, j = j, i
    return n * i - i * (i + 1) // 2 + (j - i - 1)


def n_stripes(n: int) -> int:
    """Stripe count: pairs (i, i+s+1 mod n) for s < floor(n/2) cover all pairs."""
    return n // 2


def stripe_partner(n: int, s: int, i: int) -> int:
    return (i + s + 1) % n


def to_stripes(condensed: np.ndarray, n: int, s_begin: int, s_end: int) -> np.ndarray:
    """Stripe-major layout [s_end - s_begin, n]: entry (s, i) = d(i, (i+s+1) mod n)."""
    out = np.zeros((s_end - s_begin, n), dtype=condensed.dtype)
    for s in range(s_begin, s_end):
        for i in range(n):
            out[s - s_begin, i] = condensed[condensed_index(n, i, stripe_partner(n, s, i))]
    return out


def pcoa_means(condensed: np.ndarray, n: int) -> Tuple[np.ndarray, float]:
    """Row means r_i of A = -d^2/2 (diagonal zero included) and the grand mean.

    These are the centring terms of principal coordinates analysis (Gower):
    the centred matrix is A_ij - r_i - r_j + g.
    """
    d = np.zeros((n, n), dtype=np.float64)
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            d[i, j] = d[j, i] = condensed[k]
            k += 1
    a = -0.5 * d * d
    r = a.mean(axis=1)
    return r, float(r.mean())


def gram_split_bf16(length: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Split FP64 lengths into hi + lo bfloat16 values (round to nearest even).

    hi = bf16(l), lo = bf16(l - hi); returned as the FP64 values they encode.
    Used to state the exact result the split-precision Gram path is aiming at.
    """
    l = np.asarray(length, dtype=np.float64)
    hi = _round_bf16_f64(l)
    lo = _round_bf16_f64(l - hi)
    return hi, lo


def _round_bf16_f64(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), exactly.

    bfloat16 keeps 8 significant bits.  For a normal x = m * 2^e with
    1 <= m < 2, the grid spacing is 2^(e-7); values are rounded on that grid.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    m, e = np.frexp(x[nz])           # x = m * 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)          # bfloat16 subnormal grid below 2^-126
    scaled = np.ldexp(x[nz], 8 - e)  # 8 significant bits left of the point
    out[nz] = np.ldexp(np.rint(scaled), e - 8)   # np.rint rounds half to even
    return out
