"""Full-size parity: the benchmark workload (200,000-tip tree, 25,000 samples)
in the launch configuration bench.py times, checked on sampled pairs that the
oracle computes one by one, plus properties that hold at any size.

Pairs sampled: random pairs, the first and last samples, and pairs at the
stripe boundary (partner N/2 away, the duplicated last stripe of even N).
Tolerances as in test_gpu_parity.py.

The 50,000-sample workload (same tree laws) is checked on all pairs among its
first 300 samples, taken from the full GPU matrix: there floor(N/2) exceeds one
slot workgroup's LDS row, so the sparse part runs in two segments per sample.
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
    ("weighted_normalized", "fp64", None),
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
    assert np.all(dd >= 0.0) and np.all(dd <= 1.0)
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
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C3")
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    emb = uf.Embedding(t, tb)
    m = 300
    sub = synth.subset_rows(table, np.arange(m))
    want = {v: core.dm(tree, sub, v)[0] for v in ("weighted_normalized", "unweighted")}
    return table.n_samples, emb, m, want


@pytest.mark.parametrize("variant,precision", [
    ("weighted_normalized", "fp32_split"),
    ("unweighted", "mfma_split"),
    ("unweighted", "mfma"),
])
def test_c3_leading_samples_all_pairs(c3, variant, precision):
    import torch
    import paper_2107_05397_amd as uf
    n, emb, m, want = c3
    d, _, _ = uf.dm(emb, variant, precision)
    ii, jj = np.triu_indices(m, 1)
    idx = torch.from_numpy(n * ii - ii * (ii + 1) // 2 + (jj - ii - 1)).to("cuda")
    got = d[idx].cpu().numpy()
    err = np.abs(got - want[variant])
    print(f"[C3 {variant} {precision}] first {m} samples max|err|={err.max():.3e}", flush=True)
    assert err.max() <= 1e-4
    assert float(d.min()) >= 0.0 and float(d.max()) <= 1.0
