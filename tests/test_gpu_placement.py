"""GPU parity of the placement-encoder kernels through the C ABI.

Tolerances:
* GEMM layouts: FP32 accumulation of K bf16 products vs an FP64 numpy matmul
  of the same bf16 operands: |err| <= 1e-5 * sum_k |a||b| (+1 bf16 ulp of the
  result for bf16-stored epilogues).
* MLP loss / gradients vs the FP64 oracle with the kernels' bf16 storage
  points: 2e-2 of the largest gradient entry per tensor (bf16 has an 8-bit
  significand; a stored activation that rounds the other way moves a gradient
  entry by ~2^-8 of its scale), loss 1e-3 relative.
* Adam: one step from the oracle's own gradients in FP64 vs the kernel chain.
* top-k: indices bit-exact (ties to the smaller column).
* projection: within one bf16 rounding of the FP64 oracle.
* exact re-rank across two tables: 1e-12 (FP64 min-form).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import placement as op
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _bf(rng, shape, scale=1.0):
    return synth.bf16_grid(rng.normal(size=shape) * scale)


def _t(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("M,N,K", [(128, 128, 64), (200, 96, 160), (37, 300, 32)])
def test_gemm_layouts_against_numpy(M, N, K):
    import ctypes
    import torch
    import paper_2107_05397_amd as uf
    L = uf.lib()
    rng = np.random.default_rng(M + N + K)
    a = _bf(rng, (M, K))
    b = _bf(rng, (N, K))
    want = a.astype(np.float64) @ b.astype(np.float64).T
    bound = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64).T
    # the three operand layouts through the MLP entry points are exercised by
    # the gradient test; here: forward layout (row, row) via a 1-layer MLP
    if M >= 2 and K % 32 == 0 and N % 32 == 0:
        mlp = uf.MLP([K, N], max_rows=max(M, 2), params=[(b, np.zeros(N, np.float32))])
        x = _t(a, torch.bfloat16)
        z = mlp.forward(x).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(z - want) <= 1e-5 * bound + 1e-30)


def _mlp_problem(seed=0, dims=(64, 32, 32, 32), n=50, p=40):
    rng = np.random.default_rng(seed)
    x = _bf(rng, (n, dims[0]))
    params = synth.mlp_init(dims, seed=seed)
    params = [(w, synth.bf16_grid(rng.normal(size=w.shape[0]) * 0.05)) for w, _ in params]
    pa = rng.integers(0, n, size=p).astype(np.int32)
    pb = ((pa + rng.integers(1, n, size=p)) % n).astype(np.int32)
    target = (rng.random(p) * 2.0).astype(np.float32)
    return x, params, pa, pb, target


def test_mlp_loss_and_gradients_vs_oracle():
    import torch
    import paper_2107_05397_amd as uf
    dims = (64, 32, 32, 32)
    x, params, pa, pb, t = _mlp_problem(dims=dims)
    mlp = uf.MLP(dims, max_rows=128, params=params)
    loss = mlp.loss_grad(_t(x, torch.bfloat16), _t(pa, torch.int32), _t(pb, torch.int32),
                         _t(t, torch.float32))
    torch.cuda.synchronize()
    w_loss, w_grads = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=True)
    f_loss, f_grads = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=False)
    assert float(loss.cpu()[0]) == pytest.approx(w_loss, rel=1e-3)
    assert float(loss.cpu()[0]) == pytest.approx(f_loss, rel=2e-2)
    for l in range(3):
        gw, gb = mlp.get(l, "grads")
        for got, want in ((gw, w_grads[l][0]), (gb, w_grads[l][1])):
            scale = np.abs(want).max()
            err = np.abs(got - want).max()
            print(f"[layer {l}] grad max|err|={err:.3e} scale={scale:.3e}")
            assert err <= 2e-2 * scale + 1e-7
        corr = np.corrcoef(gw.ravel(), f_grads[l][0].ravel())[0, 1]
        assert corr > 0.99


def test_adam_step_vs_oracle():
    import torch
    import paper_2107_05397_amd as uf
    dims = (64, 32, 32, 32)
    x, params, pa, pb, t = _mlp_problem(seed=4, dims=dims)
    mlp = uf.MLP(dims, max_rows=128, params=params)
    mlp.loss_grad(_t(x, torch.bfloat16), _t(pa, torch.int32), _t(pb, torch.int32), _t(t, torch.float32))
    mlp.adam(1e-3, 1)
    torch.cuda.synchronize()
    _, g = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=True)
    for l in range(3):
        w_new, b_new = mlp.get(l, "params")
        want_w, _, _ = op.adam(params[l][0].astype(np.float64), g[l][0], 0.0, 0.0, 1e-3, 0.9, 0.999, 1e-8, 1)
        # the first Adam step moves each weight by ~lr * sign(g); compare the step
        step_got = w_new - params[l][0]
        step_want = want_w - params[l][0]
        agree = np.mean(np.sign(step_got) == np.sign(step_want))
        assert agree > 0.97
        assert np.allclose(np.abs(step_got), np.abs(step_want), atol=2e-4)


def test_training_reduces_loss():
    import torch
    import paper_2107_05397_amd as uf
    from paper_2107_05397_amd import placement
    dims = (64, 64, 64, 32)
    rng = np.random.default_rng(9)
    n = 300
    x = _bf(rng, (n, dims[0]))
    pa = rng.integers(0, n, size=4096).astype(np.int32)
    pb = ((pa + rng.integers(1, n, size=4096)) % n).astype(np.int32)
    # a learnable target: a fixed random linear map's distances
    proj = rng.normal(size=(dims[0], 8)) / 8.0
    e = x.astype(np.float64) @ proj
    target = np.linalg.norm(e[pa] - e[pb], axis=1).astype(np.float32)
    mlp, losses = placement.train(_t(x, torch.bfloat16), pa, pb, _t(target, torch.float32), dims,
                                  synth.mlp_init(dims, seed=1), epochs=30, batch_pairs=512, lr=2e-3)
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.2 * losses[0]


def test_topk_rows_exact_with_ties():
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(2)
    for rows, cols, k in ((7, 300, 10), (3, 129, 128), (5, 2000, 50), (2, 10, 1)):
        v = rng.integers(0, 20, size=(rows, cols)).astype(np.float32) * 0.25   # many ties
        idx, vals = uf.topk_rows(_t(v, torch.float32), k)
        want_i, want_v = op.topk_rows(v, k)
        assert np.array_equal(idx.cpu().numpy(), want_i)
        assert np.array_equal(vals.cpu().numpy(), want_v.astype(np.float32))


def test_sqdist_against_cdist():
    import torch
    import paper_2107_05397_amd as uf
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(3)
    a = rng.normal(size=(70, 128)).astype(np.float32)
    b = rng.normal(size=(130, 128)).astype(np.float32)
    got = uf.sqdist(_t(a, torch.float32), _t(b, torch.float32)).cpu().numpy()
    want = cdist(a.astype(np.float64), b.astype(np.float64), "sqeuclidean")
    assert np.allclose(got, want, rtol=1e-5, atol=1e-4)


def _two_tables(n_tips=400, n_ref=60, n_q=15):
    tree = synth.gen_tree(n_tips, 0.1, seed=21)
    ref = synth.gen_table_zipf(n_ref, np.arange(n_tips), 40, seed=22)
    qry = synth.gen_table_zipf(n_q, np.arange(n_tips), 40, seed=23)
    return tree, ref, qry


def test_projection_vs_oracle():
    import torch
    import paper_2107_05397_amd as uf
    tree, ref, _ = _two_tables()
    dims, signs = synth.sparse_projection(tree.n_nodes, out_dim=256, per_node=4, seed=5)
    t = uf.Tree(tree.parent, tree.length)
    emb = uf.Embedding(t, uf.Table(t, ref.indptr, ref.tips, ref.counts))
    got = uf.project(t, emb, dims, signs, out_dim=256).float().cpu().numpy().astype(np.float64)
    want = op.project(tree, ref, dims, signs, 256)
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -8 + 1e-9)


def test_sparse_rerank_vs_oracle():
    import torch
    import paper_2107_05397_amd as uf
    tree, ref, qry = _two_tables()
    t = uf.Tree(tree.parent, tree.length)
    er = uf.Embedding(t, uf.Table(t, ref.indptr, ref.tips, ref.counts))
    eq = uf.Embedding(t, uf.Table(t, qry.indptr, qry.tips, qry.counts))
    sr, sq = uf.Sparse(er), uf.Sparse(eq)
    nq, nr = qry.n_samples, ref.n_samples
    cand = np.tile(np.arange(nr, dtype=np.int32), (nq, 1))
    got = uf.rerank(sq, sr, _t(np.arange(nq, dtype=np.int32), torch.int32), _t(cand, torch.int32))
    torch.cuda.synchronize()
    both = synth.Table(indptr=np.concatenate([ref.indptr, ref.indptr[-1] + qry.indptr[1:]]),
                       tips=np.concatenate([ref.tips, qry.tips]),
                       counts=np.concatenate([ref.counts, qry.counts]))
    pairs = [(nr + q, r) for q in range(nq) for r in range(nr)]
    want = oracle.dm_pairs(tree, both, pairs, "weighted_normalized").reshape(nq, nr)
    assert np.max(np.abs(got.cpu().numpy() - want)) <= 1e-12


def test_condensed_reads():
    import torch
    import paper_2107_05397_amd as uf
    n = 23
    cond = np.arange(n * (n - 1) // 2, dtype=np.float64) / 7.0
    c = _t(cond, torch.float64)
    blk = uf.condensed_block(c, n, 3, 5, 10, 13).cpu().numpy()
    for r in range(5):
        for q in range(13):
            i, j = 3 + r, 10 + q
            want = np.inf if i == j else cond[oracle.condensed_index(n, i, j)]
            assert blk[r, q] == np.float32(want)
    a = np.array([0, 5, 22, 7], np.int32)
    b = np.array([1, 2, 3, 7], np.int32)
    g = uf.gather_pairs(c, n, _t(a, torch.int32), _t(b, torch.int32)).cpu().numpy()
    want = [cond[oracle.condensed_index(n, x, y)] if x != y else 0.0 for x, y in zip(a, b)]
    assert np.allclose(g, np.float32(want))
