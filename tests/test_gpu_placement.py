"""GPU parity of the placement-encoder kernels through the C ABI.

Tolerances:
* GEMM layouts: FP32 accumulation of K bf16 products vs an FP64 numpy matmul
  of the same bf16 operands: |err| <= 1e-5 * sum_k |a||b| (+1 bf16 ulp of the
  result for bf16-stored epilogues).
* MLP loss / gradients vs the FP64 oracle with the kernels' bf16 storage
  points: 2e-2 of the largest gradient entry per tensor (bf16 has an 8-bit
  significand; a stored activation that rounds the other way moves a gradient
  entry by ~2^-8 of its scale), loss 1e-3 relative.
* GEMM layouts, exact: with small integer operands every product, FP32 sum and
  BF16-stored activation is exact, so forward, backward-data and weight-gradient
  results must equal int64 numpy bit for bit.
* Adam / AdamW: three steps; parameters and both moments vs the FP64 oracle fed
  with the kernel's own gradients, to FP32 rounding (1e-5 relative).
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


@pytest.mark.parametrize("M,N,K", [(128, 128, 64), (200, 96, 160), (37, 288, 32)])
def test_gemm_forward_layout_against_numpy(M, N, K):
    # forward layout (row, row) via a 1-layer MLP on random bf16 operands; every
    # case runs (widths are multiples of 32, M ragged)
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(M + N + K)
    a = _bf(rng, (M, K))
    b = _bf(rng, (N, K))
    want = a.astype(np.float64) @ b.astype(np.float64).T
    bound = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64).T
    mlp = uf.MLP([K, N], max_rows=max(M, 2), params=[(b, np.zeros(N, np.float32))])
    z = mlp.forward(_t(a, torch.bfloat16)).cpu().numpy().astype(np.float64)
    assert z.shape == (M, N)
    assert np.all(np.abs(z - want) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("d0,d1,d2,n_src,n", [(288, 160, 64, 250, 300),
                                             (608, 544, 288, 500, 777)])
def test_all_gemm_layouts_exact_on_integers(d0, d1, d2, n_src, n):
    """Forward (row x row, gathered rows, bias + ReLU, linear path), backward-data
    ((dz W) masked by the ReLU) and weight-gradient (column x column, gathered
    rows) layouts, each checked bit for bit: small integer operands keep every
    product, every FP32 sum and every BF16-stored activation exact, so the result
    must equal an int64 numpy computation.  Sizes span several tiles in every
    dimension with ragged edges; the second case puts every layout on 256 x 256
    tiles (both sides >= 256) with a K tail of 9 rows in the weight gradients."""
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(77)
    x = rng.integers(-1, 2, size=(n_src, d0))
    w1 = np.zeros((d1, d0), dtype=np.int64)            # 100 entries of +-1 per row: |h1| <= 103
    for r in range(d1):
        w1[r, rng.choice(d0, size=100, replace=False)] = rng.choice([-1, 1], size=100)
    b1 = rng.integers(-3, 4, size=d1)
    w2 = np.zeros((d2, d1), dtype=np.int64)            # at most 60 entries of +-1 per column
    for c in range(d1):
        w2[rng.choice(d2, size=min(60, d2), replace=False), c] = rng.choice([-1, 1], size=min(60, d2))
    b2 = rng.integers(-3, 4, size=d2)
    sk = rng.integers(-1, 2, size=(d2, d0))
    rows = rng.integers(0, n_src, size=n).astype(np.int32)   # a gather with repeats
    dz = rng.integers(-2, 3, size=(n, d2))             # |dz w2| <= 120: exact in bf16
    mlp = uf.MLP([d0, d1, d2], max_rows=n, params=[(w1, b1), (w2, b2)], skip=sk)
    xt = _t(x, torch.bfloat16)
    rt = _t(rows, torch.int32)
    z = mlp.forward(xt, rows=rt).cpu().numpy()
    xr = x[rows]
    h1 = np.maximum(xr @ w1.T + b1, 0)
    assert np.abs(h1).max() <= 256                       # exact in bf16
    want_z = h1 @ w2.T + b2 + xr @ sk.T
    assert np.array_equal(z.astype(np.int64), want_z) and np.array_equal(z, want_z.astype(np.float32))
    mlp.backward(xt, _t(dz, torch.bfloat16), rows=rt)
    g1 = (dz @ w2) * (h1 > 0)
    assert np.abs(g1).max() <= 256
    want = {0: (g1.T @ xr, g1.sum(0)), 1: (dz.T @ h1, dz.sum(0))}
    for l in (0, 1):
        gw, gb = mlp.get(l, "grads")
        assert np.array_equal(gw, want[l][0].astype(np.float32)), l
        assert np.array_equal(gb, want[l][1].astype(np.float32)), l
    gs, _ = mlp.get(2, "grads")
    assert np.array_equal(gs, (dz.T @ xr).astype(np.float32))


def test_gemm_paths_exact_at_encoder_shapes():
    """The encoder's own shapes (4096 -> 1024 -> 1024 -> 128 with the linear path,
    8,192 gathered rows, as one training batch of 4,096 pairs): these take the
    256-row tiles and every split-K path (the narrow layers and the weight
    gradients over 8,192 rows).  Integer operands chosen so that every FP32 sum
    and every BF16-stored activation or gradient is exact: forward, backward-data
    and weight gradients must equal a float64 numpy computation bit for bit."""
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(2107)
    d0, d1, d2, d3, n_src, n = 4096, 1024, 1024, 128, 9000, 8192
    x = rng.integers(-1, 2, size=(n_src, d0)).astype(np.float64)
    w1 = np.zeros((d1, d0))                       # 32 entries +-1 per row: |h1| <= 35
    for r in range(d1):
        w1[r, rng.choice(d0, size=32, replace=False)] = rng.choice([-1.0, 1.0], size=32)
    b1 = rng.integers(-3, 4, size=d1).astype(np.float64)
    w2 = np.zeros((d2, d1))                       # 4 signed permutations: 4 per row and column
    for _ in range(4):
        w2[np.arange(d2), rng.permutation(d1)] += rng.choice([-1.0, 1.0], size=d2)
    b2 = rng.integers(-3, 4, size=d2).astype(np.float64)
    w3 = np.zeros((d3, d2))                       # 2 entries per column: |dz W3| <= 2
    for c in range(d2):
        w3[rng.choice(d3, size=2, replace=False), c] = rng.choice([-1.0, 1.0], size=2)
    b3 = rng.integers(-3, 4, size=d3).astype(np.float64)
    sk = rng.integers(-1, 2, size=(d3, d0)).astype(np.float64)
    rows = rng.integers(0, n_src, size=n).astype(np.int32)
    dz = rng.integers(-1, 2, size=(n, d3)).astype(np.float64)
    mlp = uf.MLP([d0, d1, d2, d3], max_rows=n, params=[(w1, b1), (w2, b2), (w3, b3)], skip=sk)
    xt = _t(x, torch.bfloat16)
    rt = _t(rows, torch.int32)
    z = mlp.forward(xt, rows=rt).cpu().numpy().astype(np.float64)
    xr = x[rows]
    h1 = np.maximum(xr @ w1.T + b1, 0)
    h2 = np.maximum(h1 @ w2.T + b2, 0)
    assert np.abs(h1).max() <= 256 and np.abs(h2).max() <= 256   # exact in bf16
    want_z = h2 @ w3.T + b3 + xr @ sk.T
    assert np.abs(want_z).max() < 2 ** 24
    assert np.array_equal(z, want_z)
    mlp.backward(xt, _t(dz, torch.bfloat16), rows=rt)
    g2 = (dz @ w3) * (h2 > 0)
    g1 = (g2 @ w2) * (h1 > 0)
    assert np.abs(g2).max() <= 256 and np.abs(g1).max() <= 256
    want = {0: (g1.T @ xr, g1.sum(0)), 1: (g2.T @ h1, g2.sum(0)), 2: (dz.T @ h2, dz.sum(0))}
    for l in (0, 1, 2):
        gw, gb = mlp.get(l, "grads")
        assert np.array_equal(gw.astype(np.float64), want[l][0]), l
        assert np.array_equal(gb.astype(np.float64), want[l][1]), l
    gs, _ = mlp.get(3, "grads")
    assert np.array_equal(gs.astype(np.float64), dz.T @ xr)


@pytest.mark.parametrize("d1,n", [(32, 1), (96, 33), (2080, 17), (1024, 3000), (128, 6144)])
def test_bias_gradients_and_weight_gradients_exact(d1, n):
    """One layer: its bias gradient is the column sum of dZ (16-byte column
    groups, up to 128 row chunks, a second column block above 2,048 columns)
    and its weight gradient dZ^T x; with small integer operands both are exact
    and must equal int64 numpy.  Covers a single row, ragged row counts and the
    column-group layouts of every branch of the column-sum kernel."""
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(d1 + n)
    d0 = 64
    x = rng.integers(-2, 3, size=(n, d0))
    dz = rng.integers(-3, 4, size=(n, d1))
    w = rng.integers(-1, 2, size=(d1, d0)).astype(np.float64)
    mlp = uf.MLP([d0, d1], max_rows=max(n, 2), params=[(w, np.zeros(d1))])
    mlp.backward(_t(x, torch.bfloat16), _t(dz, torch.bfloat16))
    gw, gb = mlp.get(0, "grads")
    assert np.array_equal(gb.astype(np.int64), dz.sum(0))
    assert np.array_equal(gw.astype(np.int64), dz.T @ x)


def _mlp_problem(seed=0, dims=(64, 32, 32, 32), n=50, p=40):
    rng = np.random.default_rng(seed)
    x = _bf(rng, (n, dims[0]))
    params = synth.mlp_init(dims, seed=seed)
    params = [(w, synth.bf16_grid(rng.normal(size=w.shape[0]) * 0.05)) for w, _ in params]
    pa = rng.integers(0, n, size=p).astype(np.int32)
    pb = ((pa + rng.integers(1, n, size=p)) % n).astype(np.int32)
    target = (rng.random(p) * 2.0).astype(np.float32)
    return x, params, pa, pb, target


@pytest.mark.parametrize("rel_floor", [0.0, 0.3])
@pytest.mark.parametrize("with_skip", [False, True])
def test_mlp_loss_and_gradients_vs_oracle(with_skip, rel_floor):
    # rel_floor 0.3 with targets in [0, 2): both branches of max(d, floor) occur
    import torch
    import paper_2107_05397_amd as uf
    dims = (64, 32, 32, 32)
    x, params, pa, pb, t = _mlp_problem(dims=dims)
    skip = synth.bf16_grid(np.random.default_rng(8).normal(size=(dims[-1], dims[0])) * 0.05) \
        if with_skip else None
    mlp = uf.MLP(dims, max_rows=128, params=params, skip=skip)
    loss = mlp.loss_grad(_t(x, torch.bfloat16), _t(pa, torch.int32), _t(pb, torch.int32),
                         _t(t, torch.float32), rel_floor=rel_floor)
    torch.cuda.synchronize()
    w_loss, w_grads = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=True, rel_floor=rel_floor,
                                        skip=skip)
    f_loss, f_grads = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=False,
                                        rel_floor=rel_floor, skip=skip)
    assert float(loss.cpu()[0]) == pytest.approx(w_loss, rel=1e-3)
    assert float(loss.cpu()[0]) == pytest.approx(f_loss, rel=2e-2)
    layers = list(range(3)) + ([3] if with_skip else [])
    for l in layers:
        gw, gb = mlp.get(l, "grads")
        pairs = [(gw, w_grads[l][0])] + ([(gb, w_grads[l][1])] if gb is not None else [])
        for got, want in pairs:
            scale = np.abs(want).max()
            err = np.abs(got - want).max()
            print(f"[layer {l} skip={with_skip} floor={rel_floor}] grad max|err|={err:.3e} "
                  f"scale={scale:.3e}")
            assert err <= 2e-2 * scale + 1e-7
        corr = np.corrcoef(gw.ravel(), f_grads[l][0].ravel())[0, 1]
        assert corr > 0.99


@pytest.mark.parametrize("dist_weight,rank_weight,tau", [(1.0, 0.0, 0.05), (1.0, 2.0, 0.05),
                                                         (1.0, 5.0, 0.01), (0.0, 1.0, 0.05),
                                                         (0.1, 1.0, 0.01)])
@pytest.mark.parametrize("with_skip", [False, True])
def test_triplet_loss_and_gradients_vs_oracle(with_skip, dist_weight, rank_weight, tau):
    """The ranking loss: loss and every gradient vs the FP64 oracle at the
    kernels' BF16 storage points (tolerances as for the pair loss).  With tau =
    0.05 the ranking term's slope sigmoid((e_p - e_n) / tau) takes values across
    (0, 1); with rank_weight 0 only the two regression terms remain, with
    dist_weight 0 only the ranking term."""
    import torch
    import paper_2107_05397_amd as uf
    dims = (64, 32, 32, 32)
    x, params, _, _, _ = _mlp_problem(seed=21, dims=dims)
    rng = np.random.default_rng(22)
    n, T = x.shape[0], 40
    a = rng.integers(0, n, size=T).astype(np.int32)
    p = ((a + rng.integers(1, n, size=T)) % n).astype(np.int32)
    q = ((a + rng.integers(1, n, size=T)) % n).astype(np.int32)
    dp = (rng.random(T) * 2.0).astype(np.float32)
    dq = (rng.random(T) * 2.0).astype(np.float32)
    skip = synth.bf16_grid(rng.normal(size=(dims[-1], dims[0])) * 0.05) if with_skip else None
    mlp = uf.MLP(dims, max_rows=3 * T, params=params, skip=skip)
    loss = mlp.triplet_loss_grad(_t(x, torch.bfloat16), _t(a, torch.int32), _t(p, torch.int32),
                                 _t(q, torch.int32), _t(dp, torch.float32), _t(dq, torch.float32),
                                 rank_weight=rank_weight, tau=tau, dist_weight=dist_weight)
    torch.cuda.synchronize()
    w_loss, w_grads = op.triplet_loss_and_grads(x, params, a, p, q, dp, dq, rank_weight, tau,
                                                bf16_storage=True, skip=skip,
                                                dist_weight=dist_weight)
    f_loss, f_grads = op.triplet_loss_and_grads(x, params, a, p, q, dp, dq, rank_weight, tau,
                                                skip=skip, dist_weight=dist_weight)
    assert float(loss.cpu()[0]) == pytest.approx(w_loss, rel=1e-3)
    assert float(loss.cpu()[0]) == pytest.approx(f_loss, rel=2e-2)
    layers = list(range(3)) + ([3] if with_skip else [])
    for l in layers:
        gw, gb = mlp.get(l, "grads")
        pairs = [(gw, w_grads[l][0])] + ([(gb, w_grads[l][1])] if gb is not None else [])
        for got, want in pairs:
            scale = np.abs(want).max()
            err = np.abs(got - want).max()
            print(f"[triplet layer {l} skip={with_skip} lam={rank_weight}] grad max|err|={err:.3e} "
                  f"scale={scale:.3e}")
            assert err <= 2e-2 * scale + 1e-7
        assert np.corrcoef(gw.ravel(), f_grads[l][0].ravel())[0, 1] > 0.99
    with pytest.raises(uf.UFError):   # 3 * 41 rows do not fit max_rows = 120
        mlp.triplet_loss_grad(_t(x, torch.bfloat16), *(_t(np.resize(v, 41), torch.int32)
                                                       for v in (a, p, q)),
                              *(_t(np.resize(v, 41), torch.float32) for v in (dp, dq)))


@pytest.mark.parametrize("weight_decay", [0.0, 0.01])
def test_adam_three_steps_vs_oracle(weight_decay):
    """Three Adam steps on every parameter (weights, biases, linear path): after each
    step the parameters and both moment buffers equal the FP64 oracle's update fed
    with the same gradients (read back from the kernel), to FP32 rounding.  Decay
    applies to weight matrices and the linear path, not to biases.  The C ABI takes
    the hyperparameters as FP32, so the oracle is given their FP32 roundings (with
    b2 = 0.999 the rounding alone moves 1 - b2 by 1.3e-5 relative)."""
    import torch
    import paper_2107_05397_amd as uf
    dims = (64, 32, 32, 32)
    x, params, pa, pb, t = _mlp_problem(seed=4, dims=dims)
    skip = synth.bf16_grid(np.random.default_rng(3).normal(size=(dims[-1], dims[0])) * 0.05)
    mlp = uf.MLP(dims, max_rows=128, params=params, skip=skip)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    n_l = len(dims) - 1
    state = {}
    for l in range(n_l + 1):
        w, b = mlp.get(l, "params")
        state[l] = [(w.astype(np.float64), np.zeros(w.shape), np.zeros(w.shape))] + \
                   ([(b.astype(np.float64), np.zeros(b.shape), np.zeros(b.shape))] if b is not None else [])
    xt, at, bt, tt = _t(x, torch.bfloat16), _t(pa, torch.int32), _t(pb, torch.int32), _t(t, torch.float32)
    for step in (1, 2, 3):
        mlp.loss_grad(xt, at, bt, tt)
        grads = {l: mlp.get(l, "grads") for l in range(n_l + 1)}
        mlp.adam(lr, step, weight_decay=weight_decay)
        for l in range(n_l + 1):
            got = mlp.get(l, "params"), mlp.get(l, "adam_m"), mlp.get(l, "adam_v")
            for k, (p, m, v) in enumerate(state[l]):
                g = grads[l][k].astype(np.float64)
                wd = weight_decay if k == 0 else 0.0
                # m = b1 m' + (1 - b1) g can cancel: its FP32 error is relative to
                # the magnitudes that enter it (products and sum each rounded once,
                # m' already FP32-rounded), not to the result
                m_scale = float(np.float32(b1)) * np.abs(m) + (1 - float(np.float32(b1))) * np.abs(g)
                p, m, v = op.adam(p, g, m, v, *(float(np.float32(h)) for h in (lr, b1, b2, eps)),
                                  step, weight_decay=float(np.float32(wd)))
                state[l][k] = (p, m, v)
                gp, gm, gv = got[0][k], got[1][k], got[2][k]
                assert np.all(np.abs(gm - m) <= 1e-6 * m_scale + 1e-30), (step, l, k)
                assert np.allclose(gv, v, rtol=1e-5, atol=1e-16), (step, l, k)
                assert np.all(np.abs(gp - p) <= 1e-6 * np.abs(p) + 1e-8), (step, l, k)
            # the moments are the ones after `step` updates, not a first step again
            if step > 1:
                assert not np.allclose(got[1][0], (1 - b1) * grads[l][0], rtol=1e-3)


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


def test_rerank_long_lists_vs_oracle():
    """Samples of 6,000 tips on a 300,000-node tree (about 40,000 branches
    each): the re-rank against the FP64 oracle on long lists."""
    import torch
    import paper_2107_05397_amd as uf
    tree = synth.gen_tree(150000, 0.05, seed=61)
    ref = synth.gen_table_zipf(5, np.arange(150000), 6000, seed=62)
    qry = synth.gen_table_zipf(3, np.arange(150000), 6000, seed=63)
    t = uf.Tree(tree.parent, tree.length)
    er = uf.Embedding(t, uf.Table(t, ref.indptr, ref.tips, ref.counts))
    eq = uf.Embedding(t, uf.Table(t, qry.indptr, qry.tips, qry.counts))
    sr, sq = uf.Sparse(er), uf.Sparse(eq)
    assert sq.nnz > 100000
    nq, nr = qry.n_samples, ref.n_samples
    cand = np.tile(np.arange(nr, dtype=np.int32), (nq, 1))
    got = uf.rerank(sq, sr, _t(np.arange(nq, dtype=np.int32), torch.int32), _t(cand, torch.int32))
    both = synth.Table(indptr=np.concatenate([ref.indptr, ref.indptr[-1] + qry.indptr[1:]]),
                       tips=np.concatenate([ref.tips, qry.tips]),
                       counts=np.concatenate([ref.counts, qry.counts]))
    want = oracle.dm_pairs(tree, both, [(nr + q, r) for q in range(nq) for r in range(nr)],
                           "weighted_normalized").reshape(nq, nr)
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


def test_dm_pairs_across_tables_vs_oracle():
    import torch
    import paper_2107_05397_amd as uf
    tree, ref, qry = _two_tables()
    t = uf.Tree(tree.parent, tree.length)
    er = uf.Embedding(t, uf.Table(t, ref.indptr, ref.tips, ref.counts))
    eq = uf.Embedding(t, uf.Table(t, qry.indptr, qry.tips, qry.counts))
    sr, sq = uf.Sparse(er), uf.Sparse(eq)
    rng = np.random.default_rng(5)
    qa = rng.integers(0, qry.n_samples, size=137).astype(np.int32)
    rb = rng.integers(0, ref.n_samples, size=137).astype(np.int32)
    got = uf.dm_pairs(sq, sr, _t(np.stack([qa, rb]), torch.int32)).cpu().numpy()
    nr = ref.n_samples
    both = synth.Table(indptr=np.concatenate([ref.indptr, ref.indptr[-1] + qry.indptr[1:]]),
                       tips=np.concatenate([ref.tips, qry.tips]),
                       counts=np.concatenate([ref.counts, qry.counts]))
    want = oracle.dm_pairs(tree, both, [(int(r), nr + int(q)) for q, r in zip(qa, rb)],
                           "weighted_normalized")
    assert np.max(np.abs(got - want)) <= 1e-12


def test_pca_basis_vs_oracle():
    """Principal directions of a BF16 data matrix with 12 planted directions
    (standard deviations 3 down to 1.5) over small noise, plus a mean: the
    library's subspace equals the oracle's (eigenvectors of the FP64 covariance
    of the same BF16 values): each returned row lies in the oracle's span up to a
    residual of 1e-5 (the rows are FP32: 6e-8 per entry over 256 entries), its
    rows are orthonormal to 1e-6 and its eigenvalues agree to 1e-6 relative."""
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(41)
    n, d, k, c = 3000, 256, 12, 24
    u = rng.normal(size=(n, k)) * np.linspace(3.0, 1.5, k)
    v = np.linalg.qr(rng.normal(size=(d, k)))[0].T
    x = synth.bf16_grid(u @ v + 0.05 * rng.normal(size=(n, d)) + 1.0)
    omega = torch.tensor(synth.gaussian_matrix(d, c, seed=5), dtype=torch.float64, device="cuda")
    basis, vals = uf.pca_basis(_t(x, torch.bfloat16), k, omega, power_iters=3)
    torch.cuda.synchronize()
    got = basis.double().cpu().numpy()
    want, wv = op.pca_basis(x, k)
    resid = np.linalg.norm(got - (got @ want.T) @ want, axis=1)
    print("max residual", resid.max(), "eig rel err", np.abs(vals / wv - 1).max())
    assert resid.max() <= 1e-5
    assert np.allclose(got @ got.T, np.eye(k), atol=1e-6)
    assert np.allclose(vals, wv, rtol=1e-6)


def test_pca_basis_rank_deficient():
    """Fewer samples than directions: Xc has rank n - 1, so rows past it are zero
    and their eigenvalues 0; the others still match the oracle."""
    import torch
    import paper_2107_05397_amd as uf
    rng = np.random.default_rng(43)
    n, d, k, c = 6, 32, 8, 10
    x = synth.bf16_grid(rng.normal(size=(n, d)))
    omega = torch.tensor(synth.gaussian_matrix(d, c, seed=6), dtype=torch.float64, device="cuda")
    basis, vals = uf.pca_basis(_t(x, torch.bfloat16), k, omega, power_iters=2)
    torch.cuda.synchronize()
    got = basis.double().cpu().numpy()
    want, wv = op.pca_basis(x, n - 1)
    assert np.all(vals[n - 1:] == 0.0) and np.all(got[n - 1:] == 0.0)
    assert np.allclose(vals[:n - 1], wv, rtol=1e-6)
    resid = np.linalg.norm(got[:n - 1] - (got[:n - 1] @ want.T) @ want, axis=1)
    assert resid.max() <= 1e-5
    with pytest.raises(uf.UFError):   # more directions than test-matrix columns
        uf.pca_basis(_t(x, torch.bfloat16), 12, omega)
