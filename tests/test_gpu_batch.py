"""Batched tables (many rarefied replicates on one tree), persistent kernel,
hipGraph replay and the autotuner -- through the C ABI.

Per table the batch must equal the single-table FP32 weighted-normalized call
bit for bit (the per-pair branch order is the same; FP32 partial sums are
stored and reloaded unchanged between chunks) and the FP64 oracle within the
FP32 tolerance (1e-4).  Graph replays, eager launches, every autotuner
candidate and chunked runs must all give identical bits.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import core
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _tables():
    tree = synth.gen_tree(300, 0.05, seed=31)
    tips = np.arange(300)
    out = []
    for r, n in enumerate([2, 3, 129, 300, 517, 40, 1, 260]):
        t = synth.gen_table_zipf(n, tips, 60, seed=500 + r)
        t = synth.rarefy(t, 400, seed=600 + r)
        out.append(t)
    return tree, out


@pytest.fixture(scope="module")
def batch():
    import paper_2107_05397_amd as uf
    tree, tables = _tables()
    ut = uf.Tree(tree.parent, tree.length)
    uts = [uf.Table(ut, t.indptr, t.tips, t.counts) for t in tables]
    b = uf.Batch(ut, uts)
    return tree, tables, ut, uts, b


def _copy(outs):
    return [o.clone() for o in outs]


def test_batch_matches_single_tables_and_oracle(batch):
    import torch
    import paper_2107_05397_amd as uf
    tree, tables, ut, uts, b = batch
    outs = _copy(b.run(use_graph=True))
    torch.cuda.synchronize()
    for r, (t, tu) in enumerate(zip(tables, uts)):
        n = t.n_samples
        if n < 2:
            continue
        emb = uf.Embedding(ut, tu)
        single, _, _ = uf.dm(emb, "weighted_normalized", "fp32", out_dtype=torch.float32)
        torch.cuda.synchronize()
        assert torch.equal(outs[r], single[: n * (n - 1) // 2]), r
        want = core.dm(tree, t, "weighted_normalized")[0]
        err = np.abs(outs[r].cpu().numpy().astype(np.float64) - want)
        print(f"[batch table {r} n={n}] max|err|={err.max():.3e}")
        assert err.max() <= 1e-4


def test_graph_replay_eager_and_autotune_identical(batch, tmp_path):
    import torch
    tree, tables, ut, uts, b = batch
    ref = _copy(b.run(use_graph=True))
    x = torch.randn(512, 512, device="cuda")
    for _ in range(2):
        y = x @ x                        # unrelated work between replays
        got = b.run(use_graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c) for a, c in zip(ref, got))
    eager = b.run(use_graph=False)
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(ref, eager))
    del y
    path = str(tmp_path / "tune.json")
    ms = b.autotune(path)
    assert ms > 0 and os.path.exists(path)
    text = open(path).read()
    data = json.loads(text)
    entry = next(iter(data["gfx950"]["weighted_normalized_fp32"].values()))
    assert entry["stage_branches"] in (8, 16, 32) and 1 <= entry["wgs_per_cu"] <= 5
    assert entry["tile_stripes"] in (64, 128, 256)
    cfg = b.config()
    assert (cfg[0], cfg[1], cfg[3]) == (entry["stage_branches"], entry["wgs_per_cu"],
                                        entry["tile_stripes"])
    # every tile size and stage size (each kernel), at one and two blocks per CU
    for ts in (64, 128, 256):
        for ks in (8, 16, 32):
            for w in (1, 2):
                if ks == 32 and w == 2:
                    continue   # one block per CU only (LDS)
                b.set_config(ks, w, ts)
                got = b.run(use_graph=True)
                torch.cuda.synchronize()
                assert all(torch.equal(a, c) for a, c in zip(ref, got)), (ks, w, ts)
    import paper_2107_05397_amd as uf
    with pytest.raises(uf.UFError):
        b.set_config(32, 2, 128)   # two blocks of 96 KiB do not fit in 160 KiB of LDS
    with pytest.raises(uf.UFError):
        b.set_config(16, 2, 96)    # no such tile


def test_chunked_batch_identical(batch):
    import torch
    import paper_2107_05397_amd as uf
    tree, tables, ut, uts, b = batch
    ref = _copy(b.run(use_graph=True))
    try:
        uf.set_chunk_nodes(40)
        b2 = uf.Batch(ut, uts)
        assert b2.config()[2] == 40
        got = b2.run(use_graph=True)
        torch.cuda.synchronize()
    finally:
        uf.set_chunk_nodes(0)
    assert all(torch.equal(a, c) for a, c in zip(ref, got))


def test_tune_cache_is_read_back(batch, tmp_path):
    import paper_2107_05397_amd as uf
    tree, tables, ut, uts, b = batch
    mean_n = np.mean([t.n_samples for t in tables])
    bucket = int(np.ceil(np.log2(mean_n)))
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({"gfx950": {"weighted_normalized_fp32": {
        f"n_bucket_{bucket}": {"stage_branches": 8, "wgs_per_cu": 3, "ms": 1.0}}}}))
    b2 = uf.Batch(ut, uts, tune_cache=str(path))
    assert b2.config()[:2] == (8, 3) and b2.config()[3] == 128   # no tile entry: 128
    path.write_text(json.dumps({"gfx950": {"weighted_normalized_fp32": {
        f"n_bucket_{bucket}": {"stage_branches": 16, "wgs_per_cu": 1, "tile_stripes": 256,
                               "ms": 1.0}}}}))
    b3 = uf.Batch(ut, uts, tune_cache=str(path))
    assert b3.config()[:2] == (16, 1) and b3.config()[3] == 256
    ref = _copy(b.run(use_graph=True))
    got = b3.run(use_graph=True)
    import torch
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(ref, got))


def test_split_mode_matches_single_split_calls(tmp_path):
    """Sparse-split mode: every table equals uf_dm_weighted_normalized(UF_FP32_SPLIT)
    on that table alone, bit for bit, and the oracle within 1e-4; graph replays
    (with unrelated work between them), eager runs and every stream count agree."""
    import torch
    import paper_2107_05397_amd as uf
    tree, tables = _tables()
    ut = uf.Tree(tree.parent, tree.length)
    uts = [uf.Table(ut, t.indptr, t.tips, t.counts) for t in tables]
    b = uf.Batch(ut, uts)
    b.set_precision("fp32_split")
    ref = _copy(b.run(use_graph=True))
    torch.cuda.synchronize()
    for r, (t, tu) in enumerate(zip(tables, uts)):
        n = t.n_samples
        if n < 2:
            continue
        emb = uf.Embedding(ut, tu)
        single, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split", out_dtype=torch.float32)
        torch.cuda.synchronize()
        assert torch.equal(ref[r], single[: n * (n - 1) // 2]), r
        want = core.dm(tree, t, "weighted_normalized")[0]
        err = np.abs(ref[r].cpu().numpy().astype(np.float64) - want)
        print(f"[batch split table {r} n={n}] max|err|={err.max():.3e}")
        assert err.max() <= 1e-4
    x = torch.randn(512, 512, device="cuda")
    for _ in range(3):
        y = x @ x
        got = b.run(use_graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c) for a, c in zip(ref, got))
    eager = b.run(use_graph=False)
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(ref, eager))
    del y
    ms = b.autotune()
    assert ms > 0
    got = b.run(use_graph=True)
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(ref, got))
    b.set_precision("fp32")
    dense = b.run(use_graph=True)
    torch.cuda.synchronize()
    for r, t in enumerate(tables):
        if t.n_samples >= 2:
            assert torch.max(torch.abs(dense[r] - ref[r])).item() <= 2e-4


def test_c4_scale_tables_match_single_calls_and_oracle():
    """Three rarefied tables of the batching workload's law at its scale (the
    100,000-tip tree, 2,000-3,000 samples, depth 5,000): the batch equals the
    single-table FP32 call bit for bit, at the default and at the smallest and
    largest tile, and sampled pairs equal the FP64 oracle within 1e-4."""
    import torch
    import oracle
    import paper_2107_05397_amd as uf
    tree, tables = synth.batch_tables(n_tables=3, n_min=2000, n_max=3000, seed=104)
    ut = uf.Tree(tree.parent, tree.length)
    uts = [uf.Table(ut, t.indptr, t.tips, t.counts) for t in tables]
    b = uf.Batch(ut, uts)
    print("C4-scale tables", [t.n_samples for t in tables], "config", b.config(), flush=True)
    ref = _copy(b.run(use_graph=True))
    torch.cuda.synchronize()
    for ts in (64, 256):
        b.set_config(16, 1, ts)
        got = b.run(use_graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c) for a, c in zip(ref, got)), ts
    rng = np.random.default_rng(7)
    for r, (t, tu) in enumerate(zip(tables, uts)):
        n = t.n_samples
        emb = uf.Embedding(ut, tu)
        single, _, _ = uf.dm(emb, "weighted_normalized", "fp32", out_dtype=torch.float32)
        torch.cuda.synchronize()
        assert torch.equal(ref[r], single[: n * (n - 1) // 2]), r
        ii = rng.choice(n, size=16, replace=False)
        pairs = [(int(min(a, c)), int(max(a, c))) for a, c in zip(ii[:8], ii[8:])]
        want = oracle.dm_pairs(tree, t, pairs, "weighted_normalized")
        idx = torch.tensor([uf.condensed_index(n, a, c) for a, c in pairs], device="cuda")
        got = ref[r][idx].double().cpu().numpy()
        err = np.abs(got - want)
        print(f"[C4-scale table {r} n={n}] sampled max|err| {err.max():.3e}", flush=True)
        assert err.max() <= 1e-4
