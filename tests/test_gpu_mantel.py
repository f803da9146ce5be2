"""Mantel test on the GPU (uf_mantel) against the oracle (oracle/mantel.py).

* C1-sized matrices from the distance kernels, Pearson and Spearman, every
  alternative: statistic and each permuted statistic within 1e-12, p-value
  equal (the oracle computes its own matrices);
* inputs with many ties (distances rounded on the host, the same array for
  both sides) exercise the average-tie ranks;
* the identity among the permutations reproduces the statistic exactly;
* constant matrix, out-of-range permutation entries;
* full C2 matrices: the statistic and two permuted statistics against torch's
  own correlation of the (permuted) condensed vectors;
* N = 40,000 random matrices, rows with more partners than one register pass
  holds, three LDS parts per row: the same checks.
"""
import numpy as np
import pytest

import synth
from oracle import core
from oracle import mantel as om
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _emb(tree, table):
    import paper_2107_05397_amd as uf
    t = uf.Tree(tree.parent, tree.length)
    return uf.Embedding(t, uf.Table(t, table.indptr, table.tips, table.counts))


def _perms(n, k, seed):
    rng = np.random.default_rng(seed)
    p = np.stack([rng.permutation(n) for _ in range(k)]).astype(np.int32)
    p[k // 2] = np.arange(n)          # the identity somewhere in the middle
    return p


@pytest.mark.parametrize("method", ["pearson", "spearman"])
@pytest.mark.parametrize("alternative", ["two-sided", "greater", "less"])
@pytest.mark.parametrize("n", [3, 40, 131])
def test_mantel_matches_oracle(method, alternative, n):
    import torch
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C1", n_samples=n)
    emb = _emb(tree, table)
    dw, _, _ = uf.dm(emb, "weighted_normalized", "fp64")
    du, _, _ = uf.dm(emb, "unweighted", "fp64")
    perms = _perms(n, 99, seed=n)
    st, p, ps = uf.mantel(dw, du, n, method, torch.tensor(perms, device="cuda"), alternative)
    xo = core.dm(tree, table, "weighted_normalized")[0]
    yo = core.dm(tree, table, "unweighted")[0]
    st_o, p_o, ps_o = om.mantel(xo, yo, n, method, perms, alternative)
    print(f"[mantel {method} {alternative} n={n}] r={st:.6f} (oracle {st_o:.6f}) p={p:.3f} ({p_o:.3f})")
    assert st == pytest.approx(st_o, abs=1e-12)
    assert np.allclose(ps, ps_o, atol=1e-12)
    assert p == p_o
    assert ps[len(ps) // 2] == st


@pytest.mark.parametrize("method", ["pearson", "spearman"])
def test_mantel_ties(method):
    import torch
    import paper_2107_05397_amd as uf
    n = 120
    tree, table = synth.config("C1", n_samples=n)
    x = np.round(core.dm(tree, table, "weighted_normalized")[0], 2)
    y = np.round(core.dm(tree, table, "unweighted")[0], 1)
    perms = _perms(n, 50, seed=3)
    st, p, ps = uf.mantel(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"), n, method,
                          torch.tensor(perms, device="cuda"))
    st_o, p_o, ps_o = om.mantel(x, y, n, method, perms)
    print(f"[mantel ties {method}] distinct x {np.unique(x).size}, y {np.unique(y).size}: r={st:.6f}")
    assert st == pytest.approx(st_o, abs=1e-12)
    assert np.allclose(ps, ps_o, atol=1e-12)
    assert p == p_o


def test_mantel_edge_cases():
    import torch
    import paper_2107_05397_amd as uf
    n = 10
    m = n * (n - 1) // 2
    x = torch.ones(m, dtype=torch.float64, device="cuda")
    y = torch.arange(m, dtype=torch.float64, device="cuda")
    st, p, ps = uf.mantel(x, y, n, "pearson", torch.tensor(_perms(n, 5, 1), device="cuda"))
    assert st == 0.0 and p == 1.0
    bad = _perms(n, 3, 2)
    bad[1, 4] = n
    with pytest.raises(uf.UFError):
        uf.mantel(y, y, n, "pearson", torch.tensor(bad, device="cuda"))
    st, p, ps = uf.mantel(y, y, n, "pearson")
    assert st == pytest.approx(1.0, abs=1e-14) and p == 1.0 and ps.size == 0


def test_mantel_full_size():
    import torch
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C2")
    n = table.n_samples
    emb = _emb(tree, table)
    dw, _, _ = uf.dm(emb, "weighted_normalized", "fp32_split")
    du, _, _ = uf.dm(emb, "unweighted", "mfma_split")
    perms = _perms(n, 9, seed=7)
    st, p, ps = uf.mantel(dw, du, n, "pearson", torch.tensor(perms, device="cuda"))
    torch.cuda.synchronize()
    want = torch.corrcoef(torch.stack([dw, du]))[0, 1].item()
    iu = torch.triu_indices(n, n, 1, device="cuda")
    full = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    full[iu[0], iu[1]] = dw
    full = full + full.T
    checks = []
    for b in (0, 1):
        pm = torch.tensor(perms[b], dtype=torch.int64, device="cuda")
        xp = full[pm[iu[0]], pm[iu[1]]]
        checks.append(torch.corrcoef(torch.stack([xp, du]))[0, 1].item())
    print(f"[mantel C2] r={st:.9f} torch {want:.9f}; perm {ps[:2]} torch {checks}; p={p:.3f}")
    assert st == pytest.approx(want, abs=1e-9)
    assert np.allclose(ps[:2], checks, atol=1e-9)
    assert ps[len(ps) // 2] == st
    assert 1 / 10 <= p <= 1


def test_mantel_rows_longer_than_one_register_pass():
    """N = 40,000: a block holds 32,768 partners in registers, so the first 7,231
    rows take a second pass over S's row, and each row streams in three LDS parts.
    Statistic and two permuted statistics against torch's correlation of the
    (permuted) condensed vectors."""
    import torch
    import paper_2107_05397_amd as uf
    n = 40_000
    m = n * (n - 1) // 2
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    x = torch.rand(m, dtype=torch.float64, device="cuda", generator=g)
    y = x + 0.5 * torch.rand(m, dtype=torch.float64, device="cuda", generator=g)
    perms = _perms(n, 5, seed=12)
    st, p, ps = uf.mantel(x, y, n, "pearson", torch.tensor(perms, device="cuda"))
    torch.cuda.synchronize()
    want = torch.corrcoef(torch.stack([x, y]))[0, 1].item()
    iu = torch.triu_indices(n, n, 1, device="cuda")
    full = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    full[iu[0], iu[1]] = x
    full = full + full.T
    checks = []
    for b in (0, 1):
        pm = torch.tensor(perms[b], dtype=torch.int64, device="cuda")
        xp = full[pm[iu[0]], pm[iu[1]]]
        checks.append(torch.corrcoef(torch.stack([xp, y]))[0, 1].item())
        del xp
    print(f"[mantel n=40000] r={st:.12f} torch {want:.12f}; perm {ps[:2]} torch {checks}")
    assert st == pytest.approx(want, abs=1e-9)
    assert np.allclose(ps[:2], checks, atol=1e-9)
    assert ps[len(ps) // 2] == st
    assert p == pytest.approx(2 / 6)   # the identity and r itself are as extreme as r
