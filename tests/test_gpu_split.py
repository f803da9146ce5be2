"""Sparse-aware paths through the C ABI: UF_FP32_SPLIT (weighted normalized) and
UF_MFMA_SPLIT (unweighted).

* threshold 1.0: no branch is dense, every pair contribution goes through the
  exact fixed-point sums: |d - d_oracle| <= 1e-10 (2^-40 quantisation of each
  term, sums exact in integers).  The unweighted split uses the lengths
  l_hi + l_lo of the MFMA path, so its oracle runs on those lengths;
* fixed thresholds 0.05, 0.3 and 0.0: the dense part is the FP32 stripe kernel or the
  MFMA Gram, so the FP32 tolerance (1e-4) applies;
* stripe ranges merge bit for bit; repeated runs are bit-identical (integer
  atomics commute).
"""
import numpy as np
import pytest

import oracle
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
    uf.set_split_threshold(None)


SPLIT = {"weighted_normalized": "fp32_split", "unweighted": "mfma_split"}


@pytest.mark.parametrize("variant", sorted(SPLIT))
@pytest.mark.parametrize("n", [2, 3, 64, 129, 256, 301])
@pytest.mark.parametrize("thr,tol", [(1.0, 1e-10), (0.05, 1e-4), (0.0, 1e-4), (0.3, 1e-4)])
def test_split_matches_oracle(variant, n, thr, tol, threshold):
    import torch
    import paper_2107_05397_amd as uf
    threshold(thr, variant)
    tree = synth.gen_tree(400, 0.1, seed=n)
    table = synth.gen_table_zipf(n, np.arange(400), 40, seed=n + 7)
    emb = _emb(tree, table)
    d, rm, gm = uf.dm(emb, variant, SPLIT[variant], row_means=True)
    torch.cuda.synchronize()
    ref_tree = tree
    if variant == "unweighted" and thr == 1.0:
        hi, lo = oracle.gram_split_bf16(tree.length)
        ref_tree = synth.Tree(tree.parent.copy(), hi + lo, tree.n_tips)
    want = core.dm(ref_tree, table, variant)[0]
    err = np.abs(d.cpu().numpy() - want)
    print(f"[split {variant} n={n} thr={thr}] max|err|={err.max():.3e}", uf.split_stats(emb, variant))
    assert err.max() <= tol


@pytest.mark.parametrize("variant", sorted(SPLIT))
def test_split_stripes_merge_bitwise_and_repeat(variant, threshold):
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.05)
    tree = synth.gen_tree(500, 0.1, seed=5)
    table = synth.gen_table_zipf(300, np.arange(500), 50, seed=6)
    emb = _emb(tree, table)
    full, _, _ = uf.dm(emb, variant, SPLIT[variant])
    again, _, _ = uf.dm(emb, variant, SPLIT[variant])
    n = 300
    S = uf.n_stripes(n)
    buf = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float64, device="cuda")
    for a, b in ((0, 7), (7, 100), (100, S)):
        uf.dm_stripes(emb, variant, SPLIT[variant], a, b, layout="condensed", out=buf)
    torch.cuda.synchronize()
    assert torch.equal(full, again)
    if variant == "weighted_normalized":
        assert torch.equal(full, buf)
    else:
        # the MFMA tiles covering a stripe range differ with the range, so the FP32
        # Gram partial sums may be added in another order
        assert torch.max(torch.abs(full - buf)).item() < 1e-5


def _fp32_forcing(tree, table):
    """Sample 0 reduced to one tip whose root path has lengths 1e-12: the
    fixed-point bound of the weighted dense pass fails, so it runs in FP32."""
    t = int(table.tips[table.indptr[0]])
    v = t
    while tree.parent[v] >= 0:
        tree.length[v] = 1e-12
        v = int(tree.parent[v])
    table.tips = np.concatenate([[t], table.tips[table.indptr[1]:]])
    table.counts = np.concatenate([[5], table.counts[table.indptr[1]:]])
    table.indptr = np.concatenate([[0], table.indptr[1:] - table.indptr[1] + 1])


@pytest.mark.parametrize("dense_kind", ["band_wn_u32", "band_wn_f32"])
def test_merge_and_search_embeddings_agree_bitwise(dense_kind, threshold):
    """The dense chunk of the weighted split is embedded by a forward merge when
    every sample total is below 2^32, else by one binary search per element.
    Multiplying every count by 2^32 keeps each relative abundance c/T bit for bit,
    so the two paths must give the same matrix bit for bit, for the fixed-point
    and the FP32 dense pass, and the oracle's within the FP32 tolerance."""
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.2, "weighted_normalized")
    tree = synth.gen_tree(500, 0.1, seed=31)
    table = synth.gen_table_zipf(300, np.arange(500), 60, seed=32)
    if dense_kind == "band_wn_f32":
        _fp32_forcing(tree, table)
    big = synth.Table(indptr=table.indptr.copy(), tips=table.tips.copy(),
                      counts=table.counts.astype(np.int64) * (1 << 32))
    got = []
    for tb in (table, big):
        emb = _emb(tree, tb)
        assert uf.split_stats(emb, "weighted_normalized")[0] > 0
        d, used = _dense_kernel_used(uf, emb)
        torch.cuda.synchronize()
        assert used == {dense_kind}
        got.append(d.cpu().numpy())
    assert np.array_equal(got[0], got[1])
    err = np.abs(got[0] - core.dm(tree, table, "weighted_normalized")[0]).max()
    print(f"[merge vs search embedding, {dense_kind}] max|err|={err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("variant", sorted(SPLIT))
def test_two_segment_slots_exact_and_mergeable(variant, threshold):
    """N = 41,000: floor(N/2) = 20,500 stripes exceed one slot workgroup's LDS row,
    so each sample's lists are walked in two segments.  A full-range call takes
    the segment boundary from the counts the list entries carry; stripe-range
    calls find their edges by search.  With no dense branch (threshold 1) both
    give the same integers, so the pieces merge bit for bit, and sampled pairs
    match the oracle within the 2^-40 quantisation (the unweighted lengths are
    l_hi + l_lo, as in the split)."""
    import torch
    import paper_2107_05397_amd as uf
    n = 41000
    threshold(1.0, variant)
    tree = synth.gen_tree(3000, 0.1, seed=41)
    table = synth.gen_table_zipf(n, np.arange(3000), 12, seed=42)
    emb = _emb(tree, table)
    assert uf.split_stats(emb, variant)[0] == 0
    full, _, _ = uf.dm(emb, variant, SPLIT[variant])
    S = uf.n_stripes(n)
    buf = torch.full_like(full, -1.0)
    for a, b in ((0, 7), (7, 12000), (12000, S)):
        uf.dm_stripes(emb, variant, SPLIT[variant], a, b, layout="condensed", out=buf)
    torch.cuda.synchronize()
    assert torch.equal(full, buf)
    del buf
    rng = np.random.default_rng(43)
    pairs = rng.integers(0, n, size=(3000, 2))
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    idx = torch.tensor([uf.condensed_index(n, int(i), int(j)) for i, j in pairs], device="cuda")
    got = full[idx].cpu().numpy()
    ref_tree = tree
    if variant == "unweighted":
        hi, lo = oracle.gram_split_bf16(tree.length)
        ref_tree = synth.Tree(tree.parent.copy(), hi + lo, tree.n_tips)
    want = oracle.dm_pairs(ref_tree, table, pairs, variant)
    err = np.abs(got - want).max()
    print(f"[two-segment slots {variant}] max|err|={err:.3e}")
    assert err <= 1e-10


def test_weighted_split_stripe_range_at_70000_samples(threshold):
    """N = 70,000 with no dense branch: a stripe-range call (the first 64
    stripes) through the weighted split; sampled pairs match the oracle within
    the 2^-40 quantisation of the list values (1e-10)."""
    import torch
    import paper_2107_05397_amd as uf
    n = 70000
    threshold(1.0, "weighted_normalized")
    tree = synth.gen_tree(3000, 0.1, seed=71)
    table = synth.gen_table_zipf(n, np.arange(3000), 12, seed=72)
    emb = _emb(tree, table)
    out, _ = uf.dm_stripes(emb, "weighted_normalized", "fp32_split", 0, 64)
    torch.cuda.synchronize()
    st = out.cpu().numpy().reshape(64, n)
    rng = np.random.default_rng(73)
    ss = rng.integers(0, 64, size=400)
    ii = rng.integers(0, n, size=400)
    pairs = [(int(i), int((i + s + 1) % n)) for s, i in zip(ss, ii)]
    want = oracle.dm_pairs(tree, table, pairs, "weighted_normalized")
    err = np.abs(st[ss, ii] - want).max()
    print(f"[weighted split, N={n}, stripes 0-63] max|err|={err:.3e}")
    assert err <= 1e-10


def test_mfma_split_exact_with_integer_lengths(threshold):
    """Integer lengths < 256 are exact in bf16 and their FP32 Gram sums stay below
    2^24, so the dense MFMA part is exact too: the split equals the oracle."""
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.1)
    tree = synth.gen_tree(400, 1.0, seed=12)
    rng = np.random.default_rng(0)
    tree.length[:] = rng.integers(1, 256, size=tree.n_nodes).astype(float)
    table = synth.gen_table_zipf(150, np.arange(400), 30, seed=13)
    emb = _emb(tree, table)
    nd, nl, npairs = uf.split_stats(emb, "unweighted")
    assert nd > 0 and npairs > 0
    want = core.dm(tree, table, "unweighted")[0]
    d, _, _ = uf.dm(emb, "unweighted", "mfma_split")
    torch.cuda.synchronize()
    err = np.abs(d.cpu().numpy() - want).max()
    print(f"[mfma_split integer lengths] max|err|={err:.3e}")
    assert err < 1e-12


def test_split_rejects_wrong_variant():
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(50, 0.1, seed=1)
    table = synth.gen_table_uniform(10, np.arange(50), 5, seed=2)
    emb = _emb(tree, table)
    with pytest.raises(uf.UFError):
        uf.dm(emb, "weighted_normalized", "mfma_split")
    with pytest.raises(uf.UFError):
        uf.dm(emb, "unweighted", "fp32_split")


def test_split_stats_partition(threshold):
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(300, 0.1, seed=8)
    table = synth.gen_table_zipf(100, np.arange(300), 30, seed=9)
    emb = _emb(tree, table)
    for variant in SPLIT:
        threshold(1.0, variant)
        nd, nl, npairs = uf.split_stats(emb, variant)
        assert nd == 0 and nl > 0 and npairs > 0
        threshold(0.0, variant)
        nd0, nl0, np0 = uf.split_stats(emb, variant)
        assert nl0 == 0 and np0 == 0 and nd0 > 0


def test_auto_threshold_per_variant(threshold):
    """The automatic dense set follows the cost model: branches touched by more
    samples are dense first, and the cheaper dense kernel (MFMA, unweighted)
    takes at least as many branches as the stripe kernel (weighted)."""
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(3000, 0.05, seed=21)
    table = synth.gen_table_zipf(2000, np.arange(3000), 100, seed=22)
    emb = _emb(tree, table)
    threshold(None)
    nd_w, _, np_w = uf.split_stats(emb, "weighted_normalized")
    nd_u, _, np_u = uf.split_stats(emb, "unweighted")
    threshold(0.0)
    nd_all = uf.split_stats(emb, "unweighted")[0]
    print(f"[auto split] weighted dense={nd_w} pairs={np_w}; unweighted dense={nd_u} pairs={np_u}; "
          f"touched={nd_all}")
    assert 0 < nd_w <= nd_u < nd_all
    assert np_u <= np_w
    with pytest.raises(uf.UFError):
        uf.set_split_threshold(1.5)


def _dense_kernel_used(uf, emb):
    uf.profile_reset()
    uf.profile_enable(True)
    try:
        d, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split")
    finally:
        uf.profile_enable(False)
    used = {k for k in ("band_wn_u32", "band_wn_f32") if uf.profile_read(k)[1] > 0}
    return d, used


def test_weighted_dense_pass_fixed_point(threshold):
    """Homogeneous sample masses: the dense weighted pass runs in 32-bit fixed point
    and stays within its stated bound (1e-5) of the oracle."""
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.1, "weighted_normalized")
    tree = synth.gen_tree(600, 0.1, seed=31)
    table = synth.gen_table_zipf(257, np.arange(600), 60, seed=32)
    emb = _emb(tree, table)
    assert uf.split_stats(emb, "weighted_normalized")[0] > 0
    d, used = _dense_kernel_used(uf, emb)
    torch.cuda.synchronize()
    err = np.abs(d.cpu().numpy() - core.dm(tree, table, "weighted_normalized")[0]).max()
    print(f"[fixed-point dense pass] kernels={used} max|err|={err:.3e}")
    assert used == {"band_wn_u32"}
    assert err <= 1e-5


def test_weighted_dense_pass_falls_back_to_fp32(threshold):
    """A sample whose whole mass sits on near-zero branch lengths makes the fixed-point
    bound fail; the dense pass then runs in FP32 and still meets the FP32 tolerance."""
    import torch
    import paper_2107_05397_amd as uf
    threshold(0.1, "weighted_normalized")
    tree = synth.gen_tree(600, 0.1, seed=33)
    table = synth.gen_table_zipf(200, np.arange(600), 60, seed=34)
    _fp32_forcing(tree, table)
    emb = _emb(tree, table)
    d, used = _dense_kernel_used(uf, emb)
    torch.cuda.synchronize()
    err = np.abs(d.cpu().numpy() - core.dm(tree, table, "weighted_normalized")[0]).max()
    print(f"[fp32 fallback dense pass] kernels={used} max|err|={err:.3e}")
    assert used == {"band_wn_f32"}
    assert err <= 1e-4


@pytest.mark.parametrize("variant", sorted(SPLIT))
def test_prepare_rebuild_is_bitwise_equal(variant, threshold):
    """A split rebuilt from the device-resident table (uf_embedding_prepare, as a
    benchmark step does) gives the same bits as the one built on first use, and
    lists ranked by the LDS bitmap and by pairwise comparison agree."""
    import os
    import torch
    import paper_2107_05397_amd as uf
    threshold(1.0, variant)          # every shared branch in the lists: long lists too
    tree = synth.gen_tree(500, 0.1, seed=31)
    table = synth.gen_table_zipf(301, np.arange(500), 40, seed=32)
    emb = _emb(tree, table)
    d0, _, _ = uf.dm(emb, variant, SPLIT[variant])
    torch.cuda.synchronize()
    emb.prepare(scalars=True, split_weighted=True, split_unweighted=True)
    d1, _, _ = uf.dm(emb, variant, SPLIT[variant])
    os.environ["UF_SPLIT_SORT"] = "pairwise"
    try:
        emb.prepare(scalars=False, split_weighted=True, split_unweighted=True)
        d2, _, _ = uf.dm(emb, variant, SPLIT[variant])
        torch.cuda.synchronize()
    finally:
        del os.environ["UF_SPLIT_SORT"]
    assert torch.equal(d0, d1) and torch.equal(d0, d2)
    _, n_lists, n_pairs = uf.split_stats(emb, variant)
    assert n_lists > 0 and n_pairs > 301 * 300 // 2    # lists longer than 64 members exist


def test_threshold_changes_while_computing(threshold):
    """One thread computes split matrices while another switches the threshold:
    each call keeps the split it started with alive, so every result is a valid
    matrix (equal to the oracle within the split tolerance)."""
    import threading
    import torch
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(400, 0.1, seed=41)
    table = synth.gen_table_zipf(200, np.arange(400), 40, seed=42)
    emb = _emb(tree, table)
    want = core.dm(tree, table, "weighted_normalized")[0]
    errors, stop = [], threading.Event()
    # the workspace size depends on the split's dense set, hence on the threshold
    # another thread may change at any moment: the caller provides one large
    # enough for every threshold it uses
    need = 0
    for f in (0.05, 0.3, 1.0):
        threshold(f, "weighted_normalized")
        need = max(need, uf.workspace_size(emb, "weighted_normalized", "fp32_split"))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")

    def flip():
        k = 0
        while not stop.is_set():
            threshold((0.05, 0.3, 1.0)[k % 3], "weighted_normalized")
            uf.split_stats(emb, "weighted_normalized")
            k += 1

    th = threading.Thread(target=flip)
    th.start()
    try:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            for _ in range(20):
                d, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split", stream=stream,
                                workspace=ws)
                stream.synchronize()
                errors.append(float(np.abs(d.cpu().numpy() - want).max()))
    finally:
        stop.set()
        th.join()
    print("max errors", max(errors))
    assert max(errors) <= 1e-4
