"""PCoA on the GPU (uf_pcoa) against the oracle (oracle/pcoa.py).

* C1-sized matrices, both variants: the GPU result and the oracle's randomized
  subspace iteration run on the same test matrix Omega, so they span the same
  subspace and must agree to rounding (eigenvalues 1e-9 relative, coordinates
  1e-7 of their scale);
* row means computed inside the call equal the ones the distance call returns;
* a Euclidean point set (rank 3): eigenvalues equal those of Xc^T Xc and the
  coordinates reproduce every distance (closed form);
* the full C2 weighted matrix in the benchmark's configuration, by properties
  that hold at any size: v_k^T B v_k = lambda_k (Rayleigh-Ritz identity, with B
  applied independently in torch FP64), orthogonal coordinates with squared
  norms lambda_k, decreasing eigenvalues summing to at most trace(B), and small
  residuals for the leading pairs.
"""
import numpy as np
import pytest

import synth
from oracle import core
from oracle import pcoa as opcoa
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _emb(tree, table):
    import paper_2107_05397_amd as uf
    t = uf.Tree(tree.parent, tree.length)
    return uf.Embedding(t, uf.Table(t, table.indptr, table.tips, table.counts))


@pytest.mark.parametrize("variant", ["weighted_normalized", "unweighted"])
@pytest.mark.parametrize("n,dims,cols,q", [(256, 5, 16, 3), (97, 3, 10, 0), (40, 8, 40, 2)])
def test_pcoa_matches_oracle(variant, n, dims, cols, q):
    import torch
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C1", n_samples=n)
    emb = _emb(tree, table)
    d, rm, gm = uf.dm(emb, variant, "fp64", row_means=True)
    omega_h = synth.gaussian_matrix(n, cols, seed=17)
    omega = torch.tensor(omega_h, dtype=torch.float64, device="cuda")
    coords, vals, tr = uf.pcoa(d, n, dims, omega, power_iters=q, row_means=rm, grand_mean=gm)
    torch.cuda.synchronize()
    d_o = core.dm(tree, table, variant)[0]
    v_o, c_o, tr_o = opcoa.pcoa_randomized(d_o, n, dims, omega_h, q)
    print(f"[pcoa {variant} n={n}] eig {vals[:3]} vs {v_o[:3]}")
    assert np.allclose(vals, v_o, rtol=1e-9, atol=1e-12 * abs(v_o[0]))
    assert tr == pytest.approx(tr_o, rel=1e-12)
    scale = np.sqrt(max(v_o[0], 1e-300))
    got = coords.cpu().numpy()
    # eigenvalues closer than 1e-6 relative may rotate inside their eigenspace
    sep = [k for k in range(dims)
           if all(abs(v_o[k] - v_o[m]) > 1e-6 * abs(v_o[0]) for m in range(dims) if m != k)]
    assert np.allclose(got[:, sep], c_o[:, sep], atol=1e-7 * scale)
    # row means computed internally
    coords2, vals2, tr2 = uf.pcoa(d, n, dims, omega, power_iters=q)
    assert np.allclose(vals2, vals, rtol=1e-12, atol=1e-14 * abs(vals[0]))
    assert tr2 == pytest.approx(tr, rel=1e-12)


def test_pcoa_euclidean_closed_form():
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(11)
    n = 300
    x = rng.normal(size=(n, 3)) * np.array([4.0, 2.0, 1.0]) + 7.0
    iu = np.triu_indices(n, 1)
    diff = x[:, None, :] - x[None, :, :]
    dmat = np.sqrt((diff ** 2).sum(-1))[iu]
    d = torch.tensor(dmat, dtype=torch.float64, device="cuda")
    omega = torch.tensor(synth.gaussian_matrix(n, 12, seed=5), dtype=torch.float64, device="cuda")
    coords, vals, tr = uf.pcoa(d, n, 6, omega, power_iters=1)
    xc = x - x.mean(axis=0)
    want = np.sort(np.linalg.eigvalsh(xc.T @ xc))[::-1]
    print("[pcoa euclidean]", vals, want)
    assert np.allclose(vals[:3], want, rtol=1e-10)
    assert np.all(np.abs(vals[3:]) <= 1e-8 * want[0])
    c = coords.cpu().numpy()[:, :3]
    rec = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))[iu]
    assert np.allclose(rec, dmat, atol=1e-8 * dmat.max())
    assert tr == pytest.approx(want.sum(), rel=1e-10)


def test_pcoa_rejects_bad_sizes():
    import torch
    import paper_2107_05397_amd as uf
    d = torch.zeros(3, dtype=torch.float64, device="cuda")
    omega = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(uf.UFError):
        uf.pcoa(d, 3, 4, omega)          # dims > n_cols
    with pytest.raises(uf.UFError):
        uf.pcoa(d, 3, 1, torch.zeros((3, 49), dtype=torch.float64, device="cuda"))


def test_pcoa_full_size_properties():
    import torch
    import paper_2107_05397_amd as uf
    tree, table = synth.config("C2")
    n = table.n_samples
    emb = _emb(tree, table)
    d, rm, gm = uf.dm(emb, "weighted_normalized", "fp32_split", row_means=True)
    dims, cols, q = 10, 20, 3
    omega = torch.tensor(synth.gaussian_matrix(n, cols, seed=17), dtype=torch.float64, device="cuda")
    coords, vals, tr = uf.pcoa(d, n, dims, omega, power_iters=q, row_means=rm, grand_mean=gm)
    torch.cuda.synchronize()
    print(f"[pcoa C2] eig {vals} trace {tr:.4f}", flush=True)
    assert np.all(np.diff(vals) <= 1e-12 * vals[0]) and vals[-1] > 0
    assert vals.sum() <= tr * (1 + 1e-12)
    # B V with B applied independently: square matrix in torch FP64
    iu = torch.triu_indices(n, n, 1, device="cuda")
    a = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    a[iu[0], iu[1]] = -0.5 * d * d
    a = a + a.T
    del iu
    r = a.mean(dim=1)
    g = r.mean()
    lam = torch.tensor(vals, dtype=torch.float64, device="cuda")
    v = coords / torch.sqrt(lam)                      # unit eigenvectors
    bv = a @ v - r[:, None] * v.sum(0)[None, :] - (r @ v)[None, :] + g * v.sum(0)[None, :]
    ray = (v * bv).sum(0)
    gram = coords.T @ coords
    res = torch.linalg.norm(bv - v * lam[None, :], dim=0) / lam[0]
    print("[pcoa C2] rayleigh rel err", ((ray - lam).abs() / lam).max().item(),
          "residuals", res[:4].cpu().numpy(), flush=True)
    assert torch.allclose(ray, lam, rtol=1e-9)
    assert torch.allclose(gram, torch.diag(lam), atol=1e-9 * vals[0])
    assert torch.all(res[:3] < 0.05)
    assert abs(float(g.item()) - float(gm.item())) < 1e-12
