"""Sparse-aware weighted-normalized path (UF_FP32_SPLIT) through the C ABI.

* threshold 1.0: no branch is dense, every pair contribution goes through the
  exact fixed-point min-form: |d - d_oracle| <= 1e-10 (2^-40 quantisation of
  each l*u value, sums exact in integers);
* default and 0.0 thresholds: the dense part is the FP32 stripe kernel, so the
  FP32 tolerance (1e-4) applies;
* stripe ranges merge bit for bit; repeated runs are bit-identical (integer
  atomics commute).
"""
import numpy as np
import pytest

import synth
from oracle import core
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _emb(tree, table):
    import paper_2107_05397_amd as uf
    t = uf.Tree(tree.parent, tree.length)
    return uf.Embedding(t, uf.Table(t, table.indptr, table.tips, table.counts))


@pytest.fixture
def threshold():
    import paper_2107_05397_amd as uf
    yield uf.set_split_threshold
    uf.set_split_threshold(0.05)


@pytest.mark.parametrize("n", [2, 3, 64, 129, 256, 301])
@pytest.mark.parametrize("thr,tol", [(1.0, 1e-10), (0.05, 1e-4), (0.0, 1e-4), (0.3, 1e-4)])
def test_split_matches_oracle(n, thr, tol, threshold):
    import torch
    import paper_2107_05397_amd as uf
    threshold(thr)
    tree = synth.gen_tree(400, 0.1, seed=n)
    table = synth.gen_table_zipf(n, np.arange(400), 40, seed=n + 7)
    emb = _emb(tree, table)
    d, rm, gm = uf.dm(emb, "weighted_normalized", "fp32_split", row_means=True)
    torch.cuda.synchronize()
    want = core.dm(tree, table, "weighted_normalized")[0]
    err = np.abs(d.cpu().numpy() - want)
    print(f"[split n={n} thr={thr}] max|err|={err.max():.3e}", uf.split_stats(emb))
    assert err.max() <= tol


def test_split_stripes_merge_bitwise_and_repeat(threshold):
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.05)
    tree = synth.gen_tree(500, 0.1, seed=5)
    table = synth.gen_table_zipf(300, np.arange(500), 50, seed=6)
    emb = _emb(tree, table)
    full, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split")
    again, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split")
    n = 300
    S = uf.n_stripes(n)
    buf = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float64, device="cuda")
    for a, b in ((0, 7), (7, 100), (100, S)):
        uf.dm_stripes(emb, "weighted_normalized", "fp32_split", a, b, layout="condensed", out=buf)
    torch.cuda.synchronize()
    assert torch.equal(full, again)
    assert torch.equal(full, buf)


def test_split_stats_partition(threshold):
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(300, 0.1, seed=8)
    table = synth.gen_table_zipf(100, np.arange(300), 30, seed=9)
    emb = _emb(tree, table)
    threshold(1.0)
    nd, nl, npairs = uf.split_stats(emb)
    assert nd == 0 and nl > 0 and npairs > 0
    threshold(0.0)
    nd0, nl0, np0 = uf.split_stats(emb)
    assert nl0 == 0 and np0 == 0 and nd0 > 0
