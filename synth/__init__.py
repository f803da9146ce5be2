"""Seeded synthetic inputs: random rooted trees and sparse sample x tip count tables.

This module is shared by the oracle and by the GPU library's tests and bench.
It only draws random inputs; it computes nothing of the UniFrac method itself.

Workload laws (the paper measures on the Earth Microbiome Project tables, which
are not available here; these synthetic laws stand in for them):

* tree topology: random merge (coalescent) -- repeatedly join two uniformly
  chosen lineages under a new parent.  Tips get ids 0..n-1, internal nodes get
  ids n..2n-2 in creation order, the root is 2n-2.  Depth grows like log n.
* branch lengths: i.i.d. Exponential(mean) for every non-root node; the root's
  entry is 0 and is ignored by the method.
* "uniform" tables: exactly ``nnz`` distinct tips per sample, uniform without
  replacement.
* "zipf" tables: tip popularity ~ rank^-s over all tips with a seeded random
  rank->tip permutation; i.i.d. draws until ``nnz`` distinct tips are seen.
* counts: round(LogNormal(mu=2, sigma=1.5)) + 1 per (sample, tip).
* rarefaction: subsampling without replacement (multivariate hypergeometric)
  to an exact depth; samples with fewer reads are dropped.

A table is returned as CSR: ``indptr`` (n_samples+1), ``tips`` (tree node id of
each nonzero), ``counts`` (int64 > 0); all int64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = [
    "Tree", "Table", "gen_tree", "gen_table_uniform", "gen_table_zipf",
    "rarefy", "subset_rows", "config", "CONFIGS",
]


@dataclasses.dataclass
class Tree:
    parent: np.ndarray   # int64 [n_nodes], -1 for the root
    length: np.ndarray   # float64 [n_nodes], >= 0
    n_tips: int

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])


@dataclasses.dataclass
class Table:
    indptr: np.ndarray   # int64 [n_samples+1]
    tips: np.ndarray     # int64 [nnz] tree node ids
    counts: np.ndarray   # int64 [nnz] > 0

    @property
    def n_samples(self) -> int:
        return int(self.indptr.shape[0] - 1)

    def dense(self, n_nodes: int) -> np.ndarray:
        """Dense [n_samples, n_nodes] int64 count matrix (small inputs only)."""
        out = np.zeros((self.n_samples, n_nodes), dtype=np.int64)
        rows = np.repeat(np.arange(self.n_samples), np.diff(self.indptr))
        np.add.at(out, (rows, self.tips), self.counts)
        return out


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def gen_tree(n_tips: int, mean_len: float, seed: int) -> Tree:
    """Random-merge rooted binary tree with Exponential(mean_len) branch lengths."""
    if n_tips < 1:
        raise ValueError("n_tips must be >= 1")
    rng = _rng(seed, 1)
    n_nodes = 2 * n_tips - 1
    parent = np.full(n_nodes, -1, dtype=np.int64)
    m = np.arange(n_tips, 1, -1, dtype=np.float64)          # lineages before each merge
    ua = np.floor(rng.random(n_tips - 1) * m).astype(np.int64)
    ub = np.floor(rng.random(n_tips - 1) * (m - 1)).astype(np.int64)
    lineages: List[int] = list(range(n_tips))
    nxt = n_tips
    for k in range(n_tips - 1):
        a = int(ua[k])
        b = int(ub[k])
        if b >= a:
            b += 1
        la, lb = lineages[a], lineages[b]
        parent[la] = nxt
        parent[lb] = nxt
        # remove the two picked lineages (swap-with-last), then add the new one
        hi, lo = (a, b) if a > b else (b, a)
        lineages[hi] = lineages[-1]
        lineages.pop()
        lineages[lo] = lineages[-1]
        lineages.pop()
        lineages.append(nxt)
        nxt += 1
    length = rng.exponential(mean_len, size=n_nodes)
    length[n_nodes - 1] = 0.0
    return Tree(parent=parent, length=length, n_tips=n_tips)


def _counts(rng: np.random.Generator, size: int) -> np.ndarray:
    return (np.rint(rng.lognormal(2.0, 1.5, size=size)) + 1).astype(np.int64)


def gen_table_uniform(n_samples: int, tip_ids: np.ndarray, nnz: int, seed: int) -> Table:
    """Exactly ``nnz`` distinct tips per sample, uniform without replacement."""
    rng = _rng(seed, 2)
    tip_ids = np.asarray(tip_ids, dtype=np.int64)
    n = tip_ids.shape[0]
    if nnz > n:
        raise ValueError("nnz exceeds the number of tips")
    keys = rng.random((n_samples, n))
    pick = np.argpartition(keys, nnz - 1, axis=1)[:, :nnz]
    pick.sort(axis=1)
    tips = tip_ids[pick].reshape(-1)
    counts = _counts(rng, n_samples * nnz)
    indptr = np.arange(n_samples + 1, dtype=np.int64) * nnz
    return Table(indptr=indptr, tips=tips, counts=counts)


def _alias(p: np.ndarray):
    """Walker alias table for O(1) draws from a discrete law."""
    n = p.shape[0]
    q = p * n
    alias = np.zeros(n, dtype=np.int64)
    small = list(np.nonzero(q < 1.0)[0])
    large = list(np.nonzero(q >= 1.0)[0])
    while small and large:
        s = small.pop()
        g = large.pop()
        alias[s] = g
        q[g] -= 1.0 - q[s]
        (small if q[g] < 1.0 else large).append(g)
    for rest in (small, large):
        for s in rest:
            q[s] = 1.0
    return alias, q


def gen_table_zipf(n_samples: int, tip_ids: np.ndarray, nnz: int, seed: int,
                   s: float = 1.1, batch: int = 1024) -> Table:
    """Zipf(s) tip popularity; i.i.d. draws per sample until ``nnz`` distinct tips."""
    rng = _rng(seed, 3)
    tip_ids = np.asarray(tip_ids, dtype=np.int64)
    n = tip_ids.shape[0]
    if nnz > n:
        raise ValueError("nnz exceeds the number of tips")
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    alias, q = _alias(w / w.sum())
    rank_to_tip = tip_ids[rng.permutation(n)]
    rows = []
    draws = max(4 * nnz, 64)
    done = 0
    while done < n_samples:
        b = min(batch, n_samples - done)
        need = np.arange(b)
        out = np.empty((b, nnz), dtype=np.int64)
        d = draws
        while need.size:
            i = rng.integers(0, n, size=(need.size, d))
            u = rng.random((need.size, d))
            r = np.where(u < q[i], i, alias[i])
            order = np.argsort(r, axis=1, kind="stable")
            rs = np.take_along_axis(r, order, 1)
            first_sorted = np.ones_like(rs, dtype=bool)
            first_sorted[:, 1:] = rs[:, 1:] != rs[:, :-1]
            first = np.zeros_like(first_sorted)
            np.put_along_axis(first, order, first_sorted, 1)
            c = np.cumsum(first, axis=1, dtype=np.int64)
            ok = c[:, -1] >= nnz
            sel = first & (c <= nnz)
            okr = np.nonzero(ok)[0]
            if okr.size:
                out[need[okr]] = r[okr][sel[okr]].reshape(okr.size, nnz)
            need = need[~ok]
            d *= 2
        tips = np.sort(rank_to_tip[out], axis=1)
        rows.append(tips)
        done += b
    tips = np.concatenate(rows, axis=0).reshape(-1)
    counts = _counts(rng, n_samples * nnz)
    indptr = np.arange(n_samples + 1, dtype=np.int64) * nnz
    return Table(indptr=indptr, tips=tips, counts=counts)


def rarefy(table: Table, depth: int, seed: int) -> Table:
    """Subsample each sample without replacement to exactly ``depth`` reads.

    Samples with fewer than ``depth`` reads are dropped; zero entries removed.
    """
    rng = _rng(seed, 4)
    indptr, tips, counts = table.indptr, table.tips, table.counts
    out_ptr = [0]
    out_tips = []
    out_counts = []
    for r in range(table.n_samples):
        a, b = int(indptr[r]), int(indptr[r + 1])
        c = counts[a:b]
        if int(c.sum()) < depth:
            continue
        sub = rng.multivariate_hypergeometric(c, depth)
        keep = sub > 0
        out_tips.append(tips[a:b][keep])
        out_counts.append(sub[keep].astype(np.int64))
        out_ptr.append(out_ptr[-1] + int(keep.sum()))
    if out_tips:
        t = np.concatenate(out_tips)
        c = np.concatenate(out_counts)
    else:
        t = np.zeros(0, np.int64)
        c = np.zeros(0, np.int64)
    return Table(indptr=np.asarray(out_ptr, dtype=np.int64), tips=t, counts=c)


def subset_rows(table: Table, rows) -> Table:
    """Table restricted to the given sample rows (in the given order)."""
    rows = np.asarray(rows, dtype=np.int64)
    lens = table.indptr[rows + 1] - table.indptr[rows]
    indptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    idx = np.concatenate([np.arange(table.indptr[r], table.indptr[r + 1]) for r in rows]) \
        if rows.size else np.zeros(0, np.int64)
    return Table(indptr=indptr, tips=table.tips[idx], counts=table.counts[idx])


# ---------------------------------------------------------------------------
# The five workloads.  Sizes and laws follow the configurations the project is
# measured on; C1 is small enough for the oracle to finish in seconds.
# ---------------------------------------------------------------------------
CONFIGS = {
    "C1": dict(n_tips=1000, mean_len=0.1, n_samples=256, nnz=50, law="uniform", seed=101),
    "C2": dict(n_tips=200000, mean_len=0.05, n_samples=25000, nnz=1000, law="zipf", seed=102),
    "C3": dict(n_tips=200000, mean_len=0.05, n_samples=50000, nnz=1000, law="zipf", seed=103),
    "C4": dict(n_tips=100000, mean_len=0.05, n_tables=64, n_min=2000, n_max=20000,
               nnz=1000, law="zipf", depth=5000, seed=104),
    "C5": dict(n_tips=200000, mean_len=0.05, n_ref=25000, n_query=10000, nnz=1000,
               law="zipf", seed=102, query_seed=105),
}


def config(name: str, n_samples: Optional[int] = None, n_tips: Optional[int] = None):
    """Generate (tree, table) for C1/C2/C3, optionally scaled down.

    The tree seed and the table seed are the configuration's seed on separate
    streams, so a scaled-down table on the full tree reuses the same tree.
    """
    c = CONFIGS[name]
    nt = int(n_tips if n_tips is not None else c["n_tips"])
    ns = int(n_samples if n_samples is not None else c["n_samples"])
    tree = gen_tree(nt, c["mean_len"], c["seed"])
    tip_ids = np.arange(nt, dtype=np.int64)
    nnz = min(c["nnz"], nt)
    if c["law"] == "uniform":
        table = gen_table_uniform(ns, tip_ids, nnz, c["seed"])
    else:
        table = gen_table_zipf(ns, tip_ids, nnz, c["seed"])
    return tree, table


def _one_batch_table(args):
    n, n_tips, nnz, depth, tseed = args
    t = gen_table_zipf(int(n), np.arange(n_tips, dtype=np.int64), min(nnz, n_tips), tseed)
    return rarefy(t, depth, tseed)


def batch_tables(n_tips: int = 100000, n_tables: int = 64, n_min: int = 2000,
                 n_max: int = 20000, nnz: int = 1000, depth: int = 5000,
                 seed: int = 104, processes: int = 1):
    """Tree + ``n_tables`` rarefied tables of uneven size (the batching workload).

    Table r uses its own seed, so the result does not depend on ``processes``
    (worker processes are forked; call this before any GPU is initialised).
    """
    tree = gen_tree(n_tips, CONFIGS["C4"]["mean_len"], seed)
    rng = _rng(seed, 5)
    sizes = rng.integers(n_min, n_max + 1, size=n_tables)
    jobs = [(int(n), n_tips, nnz, depth, seed * 1000 + r) for r, n in enumerate(sizes)]
    if processes > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            tables = pool.map(_one_batch_table, jobs, chunksize=1)
    else:
        tables = [_one_batch_table(j) for j in jobs]
    return tree, tables


# ---------------------------------------------------------------------------
# Random inputs of the learned placement encoder.  The encoder's random
# numbers are drawn here and passed to both the GPU library and the oracle.
# ---------------------------------------------------------------------------
def sparse_projection(n_nodes: int, out_dim: int = 4096, per_node: int = 4, seed: int = 7):
    """A fixed sparse random projection: node v (by id) feeds ``per_node``
    distinct output dims with signs +-1 (the projection weight is sign/2).
    Returns (dims int32 [n_nodes, per_node], signs int8 [n_nodes, per_node])."""
    rng = _rng(seed, 6)
    dims = rng.integers(0, out_dim, size=(n_nodes, per_node)).astype(np.int32)
    while True:                         # redraw the rows that repeat a dim
        srt = np.sort(dims, axis=1)
        dup = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not dup.any():
            break
        dims[dup] = rng.integers(0, out_dim, size=(int(dup.sum()), per_node))
    signs = np.where(rng.random((n_nodes, per_node)) < 0.5, -1, 1).astype(np.int8)
    return dims, signs


def bf16_grid(x: np.ndarray) -> np.ndarray:
    """Values already on the bfloat16 grid (truncate float32 mantissas), so that
    random inputs are exactly representable by either side."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return f.view(np.float32)


def mlp_init(dims, seed: int = 11):
    """He-uniform initial weights on the bfloat16 grid and zero biases.
    dims = (d0, d1, ..., dL); returns [(W1 [d1, d0], b1), ...] as float32."""
    rng = _rng(seed, 7)
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        bound = np.sqrt(6.0 / a)
        w = bf16_grid(rng.uniform(-bound, bound, size=(b, a)).astype(np.float32))
        out.append((w, np.zeros(b, dtype=np.float32)))
    return out


def placement_pairs(n: int, n_uniform: int, neighbours: np.ndarray, n_near: int, seed: int = 13):
    """Training pairs: ``n_uniform`` uniform random pairs (i != j) plus ``n_near``
    pairs drawn from each sample's nearest-neighbour lists ``neighbours`` [n, k]."""
    rng = _rng(seed, 8)
    a = rng.integers(0, n, size=n_uniform)
    b = (a + rng.integers(1, n, size=n_uniform)) % n
    k = neighbours.shape[1]
    rows = rng.integers(0, n, size=n_near)
    cols = rng.integers(0, k, size=n_near)
    a2 = rows
    b2 = neighbours[rows, cols]
    pa = np.concatenate([a, a2]).astype(np.int32)
    pb = np.concatenate([b, b2]).astype(np.int32)
    perm = rng.permutation(pa.shape[0])
    return pa[perm], pb[perm]


def placement_triplets(n: int, neighbours: np.ndarray, n_triplets: int, near_k: int = 10,
                       far_lo: int = 10, seed: int = 14):
    """Training triples (anchor, near, far) for the ranking loss: anchors uniform;
    near drawn from the anchor's ``near_k`` nearest neighbours; far, for half of
    the triples, from its neighbours ranked ``far_lo`` .. k-1 (``neighbours`` is
    [n, k], nearest first), for the other half uniform among the other samples."""
    rng = _rng(seed, 9)
    k = neighbours.shape[1]
    a = rng.integers(0, n, size=n_triplets)
    near = neighbours[a, rng.integers(0, near_k, size=n_triplets)]
    far = neighbours[a, rng.integers(far_lo, k, size=n_triplets)]
    half = n_triplets // 2
    far[half:] = (a[half:] + rng.integers(1, n, size=n_triplets - half)) % n
    return a.astype(np.int32), near.astype(np.int32), far.astype(np.int32)


def gaussian_matrix(rows: int, cols: int, seed: int = 17) -> np.ndarray:
    """Standard normal entries on the bfloat16 grid (a Johnson-Lindenstrauss map
    when scaled), float32 [rows, cols]."""
    rng = _rng(seed, 9)
    return bf16_grid(rng.standard_normal(size=(rows, cols)).astype(np.float32))
