"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (per pair, d_o = oracle):
* FP64 path: |d - d_o| <= 1e-6 |d_o| + 1e-12 (the FP64 target).
* FP32 stripe kernels: |d - d_o| <= 1e-4.  Derivation: each prescaled value
  l*u is rounded once to FP32 (relative 2^-24) and the numerator is a
  sequential FP32 sum over the branches; with K nonzero terms the error is
  below (K + 1) * 2^-24 in d in the worst case and ~sqrt(K) * 2^-24 typically.
  For the test inputs K <= ~2e4, so the typical error is ~1e-5 and 1e-4 holds
  with margin; the measured maximum is printed.
* MFMA split-BF16 Gram path: |d - d_o| <= 1e-4 absolute (the MFMA target).
* Integer branch lengths (exact in BF16, l_lo = 0) with Gram sums below 2^24
  make the MFMA path exact: 1e-12.
Union of stripe ranges vs the full call, repeated runs and chunked runs of the
vector-ALU kernels are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import core
from tests import _util
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

VARIANTS = ("unweighted", "weighted_normalized")
PRECISIONS = {"unweighted": ("fp64", "fp32", "mfma"), "weighted_normalized": ("fp64", "fp32")}
TOL_ABS = {"fp32": 1e-4, "mfma": 1e-4}


def _uf():
    import paper_2107_05397_amd as uf
    return uf


def _emb(tree, table):
    uf = _uf()
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    return uf.Embedding(t, tb)


def _check(got, want, precision, what=""):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - want)
    if precision == "fp64":
        bad = err > 1e-6 * np.abs(want) + 1e-12
    else:
        bad = err > TOL_ABS[precision]
    print(f"[{what} {precision}] n={want.size} max|err|={err.max() if err.size else 0:.3e}", flush=True)
    assert not bad.any(), (what, precision, float(err.max()), int(bad.sum()))
    return float(err.max()) if err.size else 0.0


@pytest.fixture(scope="module")
def c1():
    tree, table = synth.config("C1")
    want = {v: core.dm(tree, table, v)[0] for v in VARIANTS}
    return tree, table, _emb(tree, table), want


@pytest.mark.parametrize("variant,precision", [(v, p) for v in VARIANTS for p in PRECISIONS[v]])
def test_c1_full_matrix(c1, variant, precision):
    import torch
    uf = _uf()
    tree, table, emb, want = c1
    n = table.n_samples
    d, rm, gm = uf.dm(emb, variant, precision, row_means=True)
    torch.cuda.synchronize()
    _check(d.cpu().numpy(), want[variant], precision, f"C1 {variant}")
    r_o, g_o = oracle.pcoa_means(want[variant], n)
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert np.allclose(rm.cpu().numpy(), r_o, rtol=0, atol=tol)
    assert abs(float(gm.cpu()[0]) - g_o) <= tol


@pytest.mark.parametrize("n", [2, 3, 5, 64, 127, 128, 129, 255, 257, 300])
def test_ragged_sample_counts(n):
    import torch
    uf = _uf()
    tree = synth.gen_tree(150, 0.2, seed=n)
    table = synth.gen_table_uniform(n, np.arange(150), 12, seed=n + 1)
    emb = _emb(tree, table)
    for variant in VARIANTS:
        want = core.dm(tree, table, variant)[0]
        for precision in PRECISIONS[variant]:
            d, _, _ = uf.dm(emb, variant, precision)
            torch.cuda.synchronize()
            _check(d.cpu().numpy(), want, precision, f"n={n} {variant}")


@pytest.mark.parametrize("variant,precision", [(v, p) for v in VARIANTS for p in PRECISIONS[v]])
def test_stripe_ranges_fill_condensed_bitwise(variant, precision):
    import torch
    uf = _uf()
    for n in (97, 300):
        tree = synth.gen_tree(300, 0.1, seed=7)
        table = synth.gen_table_uniform(n, np.arange(300), 25, seed=8)
        emb = _emb(tree, table)
        full, _, _ = uf.dm(emb, variant, precision)
        S = uf.n_stripes(n)
        cuts = [0, 1, S // 3, S // 3 + 129, S]
        cuts = sorted(set(min(max(c, 0), S) for c in cuts))
        buf = torch.full((n * (n - 1) // 2,), -7.0, dtype=torch.float64, device="cuda")
        for a, b in zip(cuts[:-1], cuts[1:]):
            uf.dm_stripes(emb, variant, precision, a, b, layout="condensed", out=buf)
        torch.cuda.synchronize()
        assert torch.equal(buf, full), (n, variant, precision)


@pytest.mark.parametrize("variant", VARIANTS)
def test_stripes_layout_and_row_sums(variant):
    import torch
    uf = _uf()
    for n in (40, 41):
        tree = synth.gen_tree(80, 0.1, seed=3)
        table = synth.gen_table_uniform(n, np.arange(80), 10, seed=4)
        emb = _emb(tree, table)
        want = oracle.dm(tree, table, variant)
        S = uf.n_stripes(n)
        total = np.zeros(n)
        for a, b in ((0, 5), (5, S)):
            st, rs = uf.dm_stripes(emb, variant, "fp64", a, b, layout="stripes", row_sums=True)
            torch.cuda.synchronize()
            _check(st.cpu().numpy().reshape(-1), oracle.to_stripes(want, n, a, b).reshape(-1), "fp64",
                   f"stripes {variant} n={n}")
            total += rs.cpu().numpy()
        r_o, _ = oracle.pcoa_means(want, n)
        assert np.allclose(total / n, r_o, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("variant,precision", [(v, p) for v in VARIANTS for p in PRECISIONS[v]])
def test_chunked_streaming_matches(variant, precision, c1):
    import torch
    uf = _uf()
    tree, table, emb, want = c1
    one, _, _ = uf.dm(emb, variant, precision)
    try:
        uf.set_chunk_nodes(96)
        many, _, _ = uf.dm(emb, variant, precision)
    finally:
        uf.set_chunk_nodes(0)
    torch.cuda.synchronize()
    if precision == "mfma":
        # FP32 partial sums are added in a different order across chunks
        _check(many.cpu().numpy(), want[variant], precision, "chunked")
        assert torch.max(torch.abs(many - one)).item() < 1e-5
    else:
        assert torch.equal(one, many)


def test_repeat_runs_are_bitwise_identical(c1):
    import torch
    uf = _uf()
    tree, table, emb, want = c1
    for variant in VARIANTS:
        for precision in PRECISIONS[variant]:
            a, ra, ga = uf.dm(emb, variant, precision, row_means=True)
            b, rb, gb = uf.dm(emb, variant, precision, row_means=True)
            torch.cuda.synchronize()
            assert torch.equal(a, b) and torch.equal(ra, rb) and torch.equal(ga, gb)


def test_mfma_exact_with_integer_lengths():
    import torch
    uf = _uf()
    tree = synth.gen_tree(400, 1.0, seed=12)
    rng = np.random.default_rng(0)
    tree.length[:] = rng.integers(1, 256, size=tree.n_nodes).astype(float)
    table = synth.gen_table_uniform(150, np.arange(400), 30, seed=13)
    emb = _emb(tree, table)
    want = core.dm(tree, table, "unweighted")[0]
    d, _, _ = uf.dm(emb, "unweighted", "mfma")
    torch.cuda.synchronize()
    err = np.abs(d.cpu().numpy() - want).max()
    print(f"[mfma integer lengths] max|err|={err:.3e}")
    assert err < 1e-12


def test_scalars_match_oracle(c1):
    tree, table, emb, want = c1
    sw, wu = emb.scalars()
    u, a, length, nonroot = oracle.embedding(tree, table)
    assert np.allclose(sw, (u[:, nonroot] * length[nonroot]).sum(1), rtol=1e-13)
    assert np.allclose(wu, (a[:, nonroot] * length[nonroot]).sum(1), rtol=1e-13)


def test_invariants_on_gpu():
    import torch
    uf = _uf()
    t = synth.gen_tree(60, 0.2, seed=4)
    root = t.n_nodes - 1
    kids = np.nonzero(t.parent == root)[0]
    anc = []
    for v in range(t.n_nodes):
        chain, x = set(), v
        while x >= 0:
            chain.add(x)
            x = t.parent[x]
        anc.append(chain)
    tips = _util.tip_ids(t)
    left = [x for x in tips if kids[0] in anc[x]]
    right = [x for x in tips if kids[1] in anc[x]]
    rng = np.random.default_rng(1)
    rows = _util.random_rows(rng, left, 3) + _util.random_rows(rng, right, 3)
    rows.append(dict(rows[0]))
    table = _util.table(rows)
    emb = _emb(t, table)
    for variant in VARIANTS:
        for precision in PRECISIONS[variant]:
            d, _, _ = uf.dm(emb, variant, precision)
            torch.cuda.synchronize()
            sq = _util.squareform(d.cpu().numpy(), 7)
            assert np.allclose(sq[:3, 3:6], 1.0, atol=1e-6 if precision != "fp64" else 1e-15)
            assert abs(sq[0, 6]) <= (1e-6 if precision != "fp64" else 1e-15)
            # the weighted variant is not clamped: its range holds up to rounding
            slack = 1e-12 if precision == "fp64" else 1e-6
            assert np.all(sq >= -slack) and np.all(sq <= 1 + slack)


def test_error_paths_on_gpu(c1):
    import torch
    uf = _uf()
    tree, table, emb, want = c1
    with pytest.raises(uf.UFError) as ei:
        uf.dm(emb, "weighted_normalized", "mfma")
    assert ei.value.name == "UF_ERR_UNSUPPORTED"
    with pytest.raises(uf.UFError) as ei:
        uf.dm_stripes(emb, "unweighted", "fp64", 5, 200)
    assert ei.value.name == "UF_ERR_RANGE"
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(table.n_samples * (table.n_samples - 1) // 2, dtype=torch.float64, device="cuda")
    L = uf.lib()
    import ctypes
    rc = L.uf_dm_unweighted(emb.handle, 0, 0, ctypes.c_void_p(out.data_ptr()), None, None,
                            ctypes.c_void_p(small.data_ptr()), 16, None)
    assert rc == 9
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0   # nothing written on error
