"""The no-allocation entry point uf_dm_weighted_normalized_noalloc against
uf_dm_weighted_normalized (the same kernels with a caller workspace) and the
FP64 oracle.

Its workspace is the library's fixed device array, which keeps the previous
call's contents, so every case makes two calls in a row, the second on a
smaller table: stale values from the first must not leak into the second.
Both calls must equal the workspace entry point bit for bit (same kernels, same
per-pair summation order over the branches) and the oracle within the FP64 /
FP32 tolerances of the parity tests.  Sizes beyond the array are refused on the
host with UF_ERR_RANGE.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _case(n):
    tree, table = synth.config("C1", n_samples=n)
    return tree, table


def _emb(uf, tree, table):
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    return uf.Embedding(t, tb)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_workspace_call_twice(precision):
    import torch
    import paper_2107_05397_amd as uf
    torch.cuda.set_device(0)
    for n in (256, 131):   # the second call on a smaller table
        tree, table = _case(n)
        emb = _emb(uf, tree, table)
        print(f"noalloc {precision} n={n}", flush=True)
        npairs = n * (n - 1) // 2
        # fill the outputs with garbage first: every element must be written
        out = torch.full((npairs,), float("nan"), dtype=torch.float64, device="cuda")
        rm = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        gm = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        uf.dm_weighted_normalized_noalloc(emb, precision, out=out, row_means=rm, grand_mean=gm)
        want, rm_w, gm_w = uf.dm(emb, "weighted_normalized", precision, row_means=True)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want.cpu().numpy()), "differs from the workspace entry point"
        assert np.array_equal(rm.cpu().numpy(), rm_w.cpu().numpy())
        assert np.array_equal(gm.cpu().numpy(), gm_w.cpu().numpy())
        ref = oracle.dm(tree, table, "weighted_normalized")
        err = np.abs(got - ref)
        tol = 1e-6 * np.abs(ref) + 1e-12 if precision == "fp64" else 1e-4
        print(f"  max|err| vs oracle {err.max():.3e}", flush=True)
        assert np.all(err <= tol)
        r_o, g_o = oracle.pcoa_means(ref, n)
        assert np.allclose(rm.cpu().numpy(), r_o, rtol=1e-9 if precision == "fp64" else 1e-4,
                           atol=1e-12 if precision == "fp64" else 1e-4)


def test_noalloc_f32_output_and_no_means():
    import torch
    import paper_2107_05397_amd as uf
    torch.cuda.set_device(0)
    tree, table = _case(200)
    emb = _emb(uf, tree, table)
    n = 200
    out = torch.full((n * (n - 1) // 2,), float("nan"), dtype=torch.float32, device="cuda")
    uf.dm_weighted_normalized_noalloc(emb, "fp32", out=out)
    want, _, _ = uf.dm(emb, "weighted_normalized", "fp32", out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want.cpu().numpy())


def test_noalloc_refuses_what_does_not_fit():
    import torch
    import paper_2107_05397_amd as uf
    torch.cuda.set_device(0)
    # FP64 with row means fits up to N = 2,877; 3,000 samples do not
    n = 3000
    tree, table = synth.config("C1", n_samples=n)
    emb = _emb(uf, tree, table)
    out = torch.zeros(n * (n - 1) // 2, dtype=torch.float64, device="cuda")
    rm = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(uf.UFError) as ei:
        uf.dm_weighted_normalized_noalloc(emb, "fp64", out=out, row_means=rm)
    assert ei.value.status == 5   # UF_ERR_RANGE
    torch.cuda.synchronize()
    assert float(out.abs().max().cpu()) == 0.0   # nothing written
    # the split precisions are not offered
    with pytest.raises(uf.UFError) as ei:
        uf.dm_weighted_normalized_noalloc(emb, "fp32_split", out=out)
    assert ei.value.status == 8   # UF_ERR_UNSUPPORTED
