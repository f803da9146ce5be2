"""Full-size parity: the benchmark workload (200,000-tip tree, 25,000 samples)
in the launch configuration bench.py times, checked on sampled pairs that the
oracle computes one by one, plus properties that hold at any size.

Pairs sampled: random pairs, the first and last samples, and pairs at the
stripe boundary (partner N/2 away, the duplicated last stripe of even N).
Tolerances as in test_gpu_parity.py.

The 50,000-sample workload (same tree laws) is checked on all 1,999,000 pairs
of a 2,000-sample subset spread over the table (every 25th sample), taken from
the full GPU matrix, with the max and mean |d - d_oracle| printed: there
floor(N/2) exceeds one slot workgroup's LDS row, so the sparse part runs in two
segments per sample, and the subset's pairs reach both.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import core
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def c2():
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C2")
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    emb = uf.Embedding(t, tb)
    n = table.n_samples
    rng = np.random.default_rng(2024)
    pairs = [(0, 1), (0, n - 1), (n - 2, n - 1), (0, n // 2), (n // 2 - 1, n - 1), (17, 17 + n // 2)]
    idx = rng.choice(n, size=(30, 2), replace=False)
    pairs += [(int(min(a, b)), int(max(a, b))) for a, b in idx if a != b]
    want = {v: oracle.dm_pairs(tree, table, pairs, v) for v in ("weighted_normalized", "unweighted")}
    return tree, table, emb, pairs, want


def _sampled(d, n, pairs):
    import torch
    import paper_2107_05397_amd as uf
    idx = torch.tensor([uf.condensed_index(n, a, b) for a, b in pairs], device="cuda")
    return d[idx].cpu().numpy()


# the sparse-aware paths run with the automatic dense set, as bench.py times them
@pytest.mark.parametrize("variant,precision,tol", [
    ("weighted_normalized", "fp32_split", 1e-4),
    ("unweighted", "mfma_split", 1e-4),
    ("weighted_normalized", "fp32", 1e-4),
    ("unweighted", "mfma", 1e-4),
    ("unweighted", "fp32", 1e-4),
    ("weighted_normalized", "fp64", None),
    ("unweighted", "fp64", None),
])
def test_c2_sampled_pairs_and_row_means(c2, variant, precision, tol):
    import torch
    import paper_2107_05397_amd as uf
    tree, table, emb, pairs, want = c2
    n = table.n_samples
    d, rm, gm = uf.dm(emb, variant, precision, row_means=True)
    torch.cuda.synchronize()
    got = _sampled(d, n, pairs)
    err = np.abs(got - want[variant])
    print(f"[C2 {variant} {precision}] sampled max|err|={err.max():.3e}", flush=True)
    if tol is None:
        assert np.all(err <= 1e-6 * np.abs(want[variant]) + 1e-12)
    else:
        assert np.all(err <= tol)
    # properties over the whole matrix
    dd = d.cpu().numpy()
    # only the unweighted (Gram form) distances are clamped to [0, 1]; the weighted
    # ones must land there up to rounding by themselves
    slack = 0.0 if variant == "unweighted" else (1e-12 if precision == "fp64" else 1e-6)
    assert np.all(dd >= -slack) and np.all(dd <= 1.0 + slack)
    # row means of -d^2/2 for a few rows, recomputed from the returned matrix
    rows = [0, 1, n // 2, n - 1]
    rmh = rm.cpu().numpy()
    for i in rows:
        js = np.array([j for j in range(n) if j != i])
        a = np.minimum(i, js)
        b = np.maximum(i, js)
        k = n * a - a * (a + 1) // 2 + (b - a - 1)
        r = -0.5 * np.sum(dd[k] ** 2) / n
        assert abs(rmh[i] - r) <= 1e-12 * max(1.0, abs(r))
    assert abs(float(gm.cpu()[0]) - rmh.mean()) <= 1e-12


@pytest.fixture(scope="module")
def c3():
    """The 50,000-sample workload and the FP64 oracle on its 2,000-sample subset:
    every 25th sample (0, 25, ..., 49,975), so that the subset's 1,999,000 pairs
    reach every part of the stripe layout -- both slot segments of a sample,
    wrapped pairs and the stripe of partners N/2 away."""
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C3")
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    emb = uf.Embedding(t, tb)
    ids = np.arange(0, table.n_samples, 25)
    sub = synth.subset_rows(table, ids)
    want = {}
    for v in ("unweighted", "weighted_normalized"):
        print(f"[C3] oracle on {len(ids)} samples, {v}", flush=True)
        want[v] = core.dm(tree, sub, v)[0]
    return table.n_samples, emb, ids, want


@pytest.mark.parametrize("variant,precision", [
    ("unweighted", "mfma_split"),
    ("unweighted", "mfma"),
    ("unweighted", "fp32"),
    ("weighted_normalized", "fp32_split"),
])
def test_c3_subset_all_pairs(c3, variant, precision):
    import torch
    import paper_2107_05397_amd as uf
    n, emb, ids, want = c3
    print(f"[C3 {variant} {precision}] full matrix", flush=True)
    d, _, _ = uf.dm(emb, variant, precision)
    a, b = np.triu_indices(len(ids), 1)
    i, j = ids[a], ids[b]
    idx = torch.from_numpy(n * i - i * (i + 1) // 2 + (j - i - 1)).to("cuda")
    got = d[idx].cpu().numpy()
    err = np.abs(got - want[variant])
    # the subset's pairs reach both slot segments (stripes below and above the
    # first segment boundary, floor(N/2)/2 here), the last stripe, and wrapped pairs
    # (j - i > N/2, held in stripe N - (j - i) - 1 of row j)
    stripe = np.minimum(j - i, n - (j - i)) - 1
    seg = (n // 2 + 1) // 2
    assert np.any(stripe < seg) and np.any(stripe >= seg) and np.any(stripe == n // 2 - 1)
    assert np.any(j - i > n // 2)
    print(f"[C3 {variant} {precision}] 2,000-sample subset: max|err|={err.max():.3e} "
          f"mean|err|={err.mean():.3e} over {err.size} pairs", flush=True)
    assert err.max() <= 1e-4
    slack = 0.0 if variant == "unweighted" else 1e-6
    assert float(d.min()) >= -slack and float(d.max()) <= 1.0 + slack
