"""Seeded generators: determinism and the laws they are meant to follow."""
import numpy as np

import synth


def test_tree_shape_and_determinism():
    t1 = synth.gen_tree(500, 0.1, seed=7)
    t2 = synth.gen_tree(500, 0.1, seed=7)
    assert np.array_equal(t1.parent, t2.parent) and np.array_equal(t1.length, t2.length)
    assert t1.n_nodes == 999
    assert (t1.parent == -1).sum() == 1 and t1.parent[-1] == -1
    nonroot = t1.parent >= 0
    # creation order: every parent id is larger than its child id
    assert np.all(t1.parent[nonroot] > np.nonzero(nonroot)[0])
    # binary: every internal node has exactly two children
    kids = np.bincount(t1.parent[nonroot], minlength=t1.n_nodes)
    assert np.all(kids[:500] == 0) and np.all(kids[500:] == 2)
    assert np.all(t1.length[nonroot] >= 0)
    big = synth.gen_tree(20000, 0.05, seed=3)
    assert abs(big.length[:-1].mean() - 0.05) < 0.002


def test_tree_depth_is_logarithmic():
    t = synth.gen_tree(20000, 0.05, seed=11)
    depth = np.zeros(t.n_nodes, np.int64)
    for v in range(t.n_nodes - 2, -1, -1):       # parents have larger ids
        depth[v] = depth[t.parent[v]] + 1
    assert depth[:20000].mean() < 4 * np.log(20000)


def test_uniform_table():
    tab = synth.gen_table_uniform(64, np.arange(1000), 50, seed=5)
    assert tab.n_samples == 64
    assert np.all(np.diff(tab.indptr) == 50)
    for s in range(64):
        row = tab.tips[tab.indptr[s]:tab.indptr[s + 1]]
        assert np.unique(row).size == 50
    assert tab.counts.min() >= 1
    tab2 = synth.gen_table_uniform(64, np.arange(1000), 50, seed=5)
    assert np.array_equal(tab.tips, tab2.tips) and np.array_equal(tab.counts, tab2.counts)


def test_zipf_table_popularity():
    tab = synth.gen_table_zipf(200, np.arange(20000), 300, seed=9)
    assert np.all(np.diff(tab.indptr) == 300)
    for s in range(0, 200, 17):
        row = tab.tips[tab.indptr[s]:tab.indptr[s + 1]]
        assert np.unique(row).size == 300
    freq = np.bincount(tab.tips, minlength=20000)
    # a popular head: some tips are in nearly every sample, most in very few
    assert freq.max() >= 190 and np.median(freq) <= 5


def test_counts_law():
    tab = synth.gen_table_uniform(400, np.arange(1000), 50, seed=1)
    lc = np.log(tab.counts.astype(float))
    assert 1.6 < np.median(lc) < 2.4


def test_rarefy():
    tab = synth.gen_table_zipf(50, np.arange(5000), 200, seed=2)
    r = synth.rarefy(tab, 1000, seed=3)
    tot = np.add.reduceat(r.counts, r.indptr[:-1])
    assert np.all(tot == 1000)
    assert r.n_samples <= 50
    r2 = synth.rarefy(tab, 1000, seed=3)
    assert np.array_equal(r.counts, r2.counts)
    # counts never exceed the originals
    orig = tab.dense(5000)
    kept = np.nonzero(np.add.reduceat(tab.counts, tab.indptr[:-1]) >= 1000)[0]
    rd = r.dense(5000)
    assert np.all(rd <= orig[kept])
