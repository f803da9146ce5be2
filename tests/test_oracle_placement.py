"""Pins of the placement-encoder oracle (oracle/placement.py) on the CPU.

* analytic FP64 gradients vs central finite differences of the loss
* the same loss and gradients through torch's CPU autograd (FP64) -- an
  independent library implementation of the same definition
* Adam vs torch.optim.Adam (FP64)
* kNN / top-k vs scipy.spatial.distance.cdist + a stable sort
* projection: a one-dim-per-node projection of a star tree is l*u/2 exactly;
  linearity in the counts' proportions
"""
import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

import synth
from oracle import placement as op
from oracle import unifrac
from tests import _util


def _problem(seed=0, dims=(16, 12, 8, 4), n=10, p=7):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, dims[0]))
    params = [(rng.normal(size=(b, a)) / np.sqrt(a), rng.normal(size=b) * 0.1)
              for a, b in zip(dims[:-1], dims[1:])]
    pa = rng.integers(0, n, size=p)
    pb = (pa + rng.integers(1, n, size=p)) % n
    target = rng.random(p)
    return x, params, pa, pb, target


def test_gradients_match_finite_differences():
    x, params, pa, pb, t = _problem()
    loss, grads = op.loss_and_grads(x, params, pa, pb, t)
    h = 1e-6
    rng = np.random.default_rng(1)
    for l, (w, b) in enumerate(params):
        for _ in range(6):
            i, j = rng.integers(w.shape[0]), rng.integers(w.shape[1])
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[l][0][i, j] += h
            wm[l][0][i, j] -= h
            fd = (op.loss_only(x, wp, pa, pb, t) - op.loss_only(x, wm, pa, pb, t)) / (2 * h)
            assert grads[l][0][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)
        i = rng.integers(b.shape[0])
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[l][1][i] += h
        bm[l][1][i] -= h
        fd = (op.loss_only(x, bp, pa, pb, t) - op.loss_only(x, bm, pa, pb, t)) / (2 * h)
        assert grads[l][1][i] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_loss_and_gradients_match_torch_autograd():
    x, params, pa, pb, t = _problem(seed=3)
    loss, grads = op.loss_and_grads(x, params, pa, pb, t)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    h = torch.tensor(x)
    rows = np.concatenate([pa, pb])
    h = h[rows]
    for l, (w, b) in enumerate(tp):
        h = h @ w.T + b
        if l < len(tp) - 1:
            h = torch.relu(h)
    p = len(pa)
    dist = torch.sqrt(((h[:p] - h[p:]) ** 2).sum(1))
    tl = ((dist - torch.tensor(t)) ** 2).mean()
    tl.backward()
    assert float(tl) == pytest.approx(loss, rel=1e-12)
    for (w, b), (gw, gb) in zip(tp, grads):
        assert np.allclose(w.grad.numpy(), gw, rtol=1e-10, atol=1e-12)
        assert np.allclose(b.grad.numpy(), gb, rtol=1e-10, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=20)
    grads = [rng.normal(size=20) for _ in range(3)]
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for step, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = op.adam(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, step)
        assert np.allclose(tp.detach().numpy(), p, rtol=1e-12, atol=1e-14)


def test_knn_and_topk_match_cdist():
    rng = np.random.default_rng(7)
    zq = rng.integers(0, 4, size=(9, 3)).astype(float)     # many ties
    zr = rng.integers(0, 4, size=(40, 3)).astype(float)
    idx, d = op.knn(zq, zr, 7)
    full = cdist(zq, zr, "sqeuclidean")
    for q in range(9):
        order = sorted(range(40), key=lambda r: (full[q, r], r))[:7]
        assert list(idx[q]) == order
        assert np.allclose(d[q], full[q, order])
    idx2, v2 = op.topk_rows(full, 7)
    assert np.array_equal(idx2, idx)


def test_projection_of_a_star_tree_is_half_l_u():
    n_tips = 12
    t = _util.tree([n_tips] * n_tips + [-1], list(np.arange(1, n_tips + 1) * 0.5) + [0.0])
    rows = [{0: 3, 5: 1}, {2: 4, 11: 4, 7: 2}]
    tab = _util.table(rows)
    dims = np.arange(n_tips + 1, dtype=np.int32).reshape(-1, 1)   # node v -> dim v
    signs = np.ones((n_tips + 1, 1), dtype=np.int8)
    signs[3, 0] = -1
    x = op.project(t, tab, dims, signs, n_tips + 1)
    u, a, length, nonroot = unifrac.embedding(t, tab)
    want = (u * length) / 2.0
    want[:, 3] *= -1
    want[:, n_tips] = 0.0                    # the root contributes nothing
    assert np.allclose(x, want, atol=1e-15)


def test_projection_is_linear_in_embedding():
    tr = synth.gen_tree(50, 0.2, seed=2)
    tab = synth.gen_table_uniform(5, np.arange(50), 8, seed=3)
    dims, signs = synth.sparse_projection(tr.n_nodes, out_dim=32, per_node=4, seed=1)
    x = op.project(tr, tab, dims, signs, 32)
    u, a, length, nonroot = unifrac.embedding(tr, tab)
    R = np.zeros((32, tr.n_nodes))
    for j in range(4):
        np.add.at(R, (dims[:, j], np.arange(tr.n_nodes)), np.where(nonroot, signs[:, j] / 2.0, 0))
    assert np.allclose(x, (u * length) @ R.T, atol=1e-14)


def test_recall_helper():
    exact = np.array([[0.1, 0.2, 0.3, 0.4], [0.5, 0.1, 0.1, 0.9]])
    assert op.recall_at_k(np.array([[0, 1], [1, 2]]), exact, 2) == 1.0
    assert op.recall_at_k(np.array([[0, 3], [1, 0]]), exact, 2) == 0.5


# ---------------------------------------------------------------- loss options, skip path, AdamW
def _fd_check(loss_fn, params, grads, skip=None, dskip=None, n_probe=5, seed=11):
    """Central differences of loss_fn(params, skip) against the analytic gradients."""
    h = 1e-6
    rng = np.random.default_rng(seed)
    for l, (w, b) in enumerate(params):
        for _ in range(n_probe):
            i, j = rng.integers(w.shape[0]), rng.integers(w.shape[1])
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[l][0][i, j] += h
            wm[l][0][i, j] -= h
            fd = (loss_fn(wp, skip) - loss_fn(wm, skip)) / (2 * h)
            assert grads[l][0][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)
        i = rng.integers(b.shape[0])
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[l][1][i] += h
        bm[l][1][i] -= h
        fd = (loss_fn(bp, skip) - loss_fn(bm, skip)) / (2 * h)
        assert grads[l][1][i] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    if skip is not None:
        for _ in range(2 * n_probe):
            i, j = rng.integers(skip.shape[0]), rng.integers(skip.shape[1])
            sp_, sm_ = skip.copy(), skip.copy()
            sp_[i, j] += h
            sm_[i, j] -= h
            fd = (loss_fn(params, sp_) - loss_fn(params, sm_)) / (2 * h)
            assert dskip[i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("rel_floor", [0.0, 0.3])
@pytest.mark.parametrize("with_skip", [False, True])
def test_loss_options_match_finite_differences(rel_floor, with_skip):
    # targets straddle the floor so both branches of max(d, floor) are exercised
    x, params, pa, pb, t = _problem(seed=21)
    t = np.linspace(0.05, 0.9, t.shape[0])
    rng = np.random.default_rng(4)
    skip = rng.normal(size=(params[-1][0].shape[0], x.shape[1])) * 0.2 if with_skip else None
    loss, grads = op.loss_and_grads(x, params, pa, pb, t, rel_floor=rel_floor, skip=skip)
    assert len(grads) == len(params) + (1 if with_skip else 0)
    lf = lambda ps, sk: op.loss_and_grads(x, ps, pa, pb, t, rel_floor=rel_floor, skip=sk)[0]  # noqa: E731
    _fd_check(lf, params, grads, skip, grads[-1][0] if with_skip else None)


@pytest.mark.parametrize("rel_floor", [0.0, 0.3])
@pytest.mark.parametrize("with_skip", [False, True])
def test_loss_options_match_torch_autograd(rel_floor, with_skip):
    x, params, pa, pb, t = _problem(seed=23)
    t = np.linspace(0.05, 0.9, t.shape[0])
    rng = np.random.default_rng(6)
    skip = rng.normal(size=(params[-1][0].shape[0], x.shape[1])) * 0.2 if with_skip else None
    loss, grads = op.loss_and_grads(x, params, pa, pb, t, rel_floor=rel_floor, skip=skip)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    ts = torch.tensor(skip, requires_grad=True) if with_skip else None
    rows = np.concatenate([pa, pb])
    x0 = torch.tensor(x)[rows]
    h = x0
    for l, (w, b) in enumerate(tp):
        h = h @ w.T + b
        if l < len(tp) - 1:
            h = torch.relu(h)
    if ts is not None:
        h = h + x0 @ ts.T
    p = len(pa)
    dist = torch.sqrt(((h[:p] - h[p:]) ** 2).sum(1))
    tt = torch.tensor(t)
    wgt = 1.0 / torch.clamp(tt, min=rel_floor) if rel_floor > 0 else torch.ones_like(tt)
    tl = (((dist - tt) * wgt) ** 2).mean()
    tl.backward()
    assert float(tl) == pytest.approx(loss, rel=1e-12)
    for (w, b), (gw, gb) in zip(tp, grads):
        assert np.allclose(w.grad.numpy(), gw, rtol=1e-10, atol=1e-12)
        assert np.allclose(b.grad.numpy(), gb, rtol=1e-10, atol=1e-12)
    if ts is not None:
        assert grads[-1][1] is None
        assert np.allclose(ts.grad.numpy(), grads[-1][0], rtol=1e-10, atol=1e-12)


def test_adamw_matches_torch():
    # decoupled weight decay (Loshchilov and Hutter): torch.optim.AdamW is an
    # independent implementation of the same update
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=30)
    grads = [rng.normal(size=30) for _ in range(4)]
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=3e-3, betas=(0.9, 0.99), eps=1e-8, weight_decay=0.05)
    p, m, v = p0.copy(), np.zeros(30), np.zeros(30)
    for step, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = op.adam(p, g, m, v, 3e-3, 0.9, 0.99, 1e-8, step, weight_decay=0.05)
        st = opt.state[tp]
        assert np.allclose(tp.detach().numpy(), p, rtol=1e-12, atol=1e-14)
        assert np.allclose(st["exp_avg"].numpy(), m, rtol=1e-12, atol=1e-15)
        assert np.allclose(st["exp_avg_sq"].numpy(), v, rtol=1e-12, atol=1e-15)


def test_bf16_storage_matches_an_independent_cast_chain():
    # the kernel's precision model: inputs, hidden activations, dZ and the hidden
    # gradients are stored in bfloat16, everything else in FP64.  Rebuilt here with
    # torch's own bfloat16 casts at those points.
    x, params, pa, pb, t = _problem(seed=31, dims=(32, 24, 16, 8), n=12, p=9)
    rng = np.random.default_rng(9)
    skip = rng.normal(size=(8, 32)) * 0.1
    for sk in (None, skip):
        loss, grads = op.loss_and_grads(x, params, pa, pb, t, bf16_storage=True, rel_floor=0.2,
                                        skip=sk)
        rb = lambda a: a.to(torch.bfloat16).to(torch.float64)  # noqa: E731
        rows = np.concatenate([pa, pb])
        h0 = rb(torch.tensor(x)[rows])
        hs, h = [h0], h0
        for l, (w, b) in enumerate(params):
            a = h @ torch.tensor(w).T + torch.tensor(b)
            if l < len(params) - 1:
                h = rb(torch.relu(a))
                hs.append(h)
            else:
                z = a
        if sk is not None:
            z = z + h0 @ torch.tensor(sk).T
        p = len(pa)
        diff = z[:p] - z[p:]
        dist = torch.sqrt((diff ** 2).sum(1))
        tt = torch.tensor(t)
        wgt = 1.0 / torch.clamp(tt, min=0.2)
        r = (dist - tt) * wgt
        assert float((r ** 2).mean()) == pytest.approx(loss, rel=1e-12)
        coef = 2.0 * r * wgt / dist / p
        dz = rb(torch.cat([coef[:, None] * diff, -coef[:, None] * diff]))
        g = dz
        for l in range(len(params) - 1, -1, -1):
            assert np.allclose((g.T @ hs[l]).numpy(), grads[l][0], rtol=1e-10, atol=1e-13)
            assert np.allclose(g.sum(0).numpy(), grads[l][1], rtol=1e-10, atol=1e-13)
            if l > 0:
                g = rb((g @ torch.tensor(params[l][0])) * (hs[l] > 0))
        if sk is not None:
            assert np.allclose((dz.T @ h0).numpy(), grads[-1][0], rtol=1e-10, atol=1e-13)


def _triplets(seed=5, n=10, t=6):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, size=t)
    p = (a + rng.integers(1, n, size=t)) % n
    q = (a + rng.integers(1, n, size=t)) % n
    return a, p, q, rng.random(t), rng.random(t)


def test_softplus_and_sigmoid_match_scipy():
    from scipy.special import expit
    x = np.array([-800.0, -40.0, -1.5, -1e-9, 0.0, 1e-9, 2.0, 40.0, 800.0])
    assert np.allclose(op.sigmoid(x), expit(x), rtol=1e-15, atol=0)
    assert np.allclose(op.softplus(x), np.logaddexp(0.0, x), rtol=1e-15, atol=0)


@pytest.mark.parametrize("with_skip,alpha", [(False, 1.0), (True, 1.0), (True, 0.0), (False, 0.3)])
def test_triplet_gradients_match_finite_differences(with_skip, alpha):
    x, params, _, _, _ = _problem(seed=11)
    a, p, q, dp, dq = _triplets()
    skip = np.random.default_rng(2).normal(size=(4, 16)) * 0.1 if with_skip else None
    lam, tau = 2.0, 0.05
    loss, grads = op.triplet_loss_and_grads(x, params, a, p, q, dp, dq, lam, tau, skip=skip,
                                            dist_weight=alpha)
    h = 1e-6
    rng = np.random.default_rng(4)

    def f(ps, sk):
        return op.triplet_loss_only(x, ps, a, p, q, dp, dq, lam, tau, skip=sk, dist_weight=alpha)

    for l, (w, b) in enumerate(params):
        for _ in range(5):
            i, j = rng.integers(w.shape[0]), rng.integers(w.shape[1])
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[l][0][i, j] += h
            wm[l][0][i, j] -= h
            fd = (f(wp, skip) - f(wm, skip)) / (2 * h)
            assert grads[l][0][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)
        i = rng.integers(b.shape[0])
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[l][1][i] += h
        bm[l][1][i] -= h
        fd = (f(bp, skip) - f(bm, skip)) / (2 * h)
        assert grads[l][1][i] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    if with_skip:
        for _ in range(5):
            i, j = rng.integers(skip.shape[0]), rng.integers(skip.shape[1])
            sp, sm = skip.copy(), skip.copy()
            sp[i, j] += h
            sm[i, j] -= h
            fd = (f(params, sp) - f(params, sm)) / (2 * h)
            assert grads[-1][0][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("alpha", [1.0, 0.25])
def test_triplet_loss_matches_torch_autograd(alpha):
    x, params, _, _, _ = _problem(seed=13)
    a, p, q, dp, dq = _triplets(seed=6)
    skip = np.random.default_rng(8).normal(size=(4, 16)) * 0.1
    lam, tau = 3.0, 0.02
    loss, grads = op.triplet_loss_and_grads(x, params, a, p, q, dp, dq, lam, tau, skip=skip,
                                            dist_weight=alpha)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    ts = torch.tensor(skip, requires_grad=True)

    def enc(rows):
        h0 = torch.tensor(x[rows])
        h = h0
        for l, (w, b) in enumerate(tp):
            h = h @ w.T + b
            if l < len(tp) - 1:
                h = torch.relu(h)
        return h + h0 @ ts.T

    za, zp, zq = enc(a), enc(p), enc(q)
    ep = torch.linalg.vector_norm(za - zp, dim=1)
    eq = torch.linalg.vector_norm(za - zq, dim=1)
    tl = (alpha * ((ep - torch.tensor(dp)) ** 2 + (eq - torch.tensor(dq)) ** 2) +
          lam * tau * torch.nn.functional.softplus((ep - eq) / tau)).mean()
    tl.backward()
    assert float(tl) == pytest.approx(loss, rel=1e-12)
    for l, (w, b) in enumerate(tp):
        assert np.allclose(grads[l][0], w.grad.numpy(), rtol=1e-9, atol=1e-12)
        assert np.allclose(grads[l][1], b.grad.numpy(), rtol=1e-9, atol=1e-12)
    assert np.allclose(grads[-1][0], ts.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_triplet_without_ranking_is_twice_the_pair_loss():
    """lam = 0 leaves the two regression terms: the pair loss over the 2T pairs
    (a, p) and (a, n), times 2 (a mean over T triples of two terms each)."""
    x, params, _, _, _ = _problem(seed=17)
    a, p, q, dp, dq = _triplets(seed=9)
    loss, grads = op.triplet_loss_and_grads(x, params, a, p, q, dp, dq, 0.0, 0.1)
    l2, g2 = op.loss_and_grads(x, params, np.concatenate([a, a]), np.concatenate([p, q]),
                               np.concatenate([dp, dq]))
    assert loss == pytest.approx(2 * l2, rel=1e-12)
    for (w, b), (w2, b2) in zip(grads, g2):
        assert np.allclose(w, 2 * w2, rtol=1e-10, atol=1e-14)
        assert np.allclose(b, 2 * b2, rtol=1e-10, atol=1e-14)


def test_triplet_ranking_term_tends_to_the_hinge():
    """tau softplus(s / tau) -> max(s, 0) as tau -> 0: the ranking term becomes
    lam * max(e_p - e_n, 0)."""
    x, params, _, _, _ = _problem(seed=19)
    a, p, q, dp, dq = _triplets(seed=10)
    base = op.triplet_loss_only(x, params, a, p, q, dp, dq, 0.0, 1.0)
    _, z = op.forward(x, params)
    ep = np.linalg.norm(z[a] - z[p], axis=1)
    eq = np.linalg.norm(z[a] - z[q], axis=1)
    hinge = np.mean(np.maximum(ep - eq, 0.0))
    got = op.triplet_loss_only(x, params, a, p, q, dp, dq, 1.0, 1e-6) - base
    assert got == pytest.approx(hinge, abs=1e-6)


def test_pca_basis_of_orthogonal_columns():
    """Columns that are centred and mutually orthogonal make the covariance
    diagonal: the principal directions are the coordinate axes, ordered by the
    columns' mean squares, and the eigenvalues are those mean squares."""
    rng = np.random.default_rng(31)
    n, d = 64, 6
    q, _ = np.linalg.qr(rng.normal(size=(n, d)) - 0.0)
    q -= q.mean(axis=0, keepdims=True)              # centre, then re-orthogonalise
    q, _ = np.linalg.qr(q)
    q -= q.mean(axis=0, keepdims=True)
    # exact orthogonality after centring: Gram-Schmidt on centred columns
    cols = []
    for j in range(d):
        c = q[:, j].copy()
        for b in cols:
            c -= (c @ b) / (b @ b) * b
        cols.append(c)
    scales = np.array([3.0, 0.5, 2.0, 1.0, 4.0, 0.25])
    x = np.stack([c / np.linalg.norm(c) * s * np.sqrt(n) for c, s in zip(cols, scales)], axis=1)
    x += np.array([5.0, -1.0, 0.0, 2.0, 0.0, 7.0])  # a mean, which the covariance removes
    basis, w = op.pca_basis(x, 3)
    assert np.allclose(w, [16.0, 9.0, 4.0], rtol=1e-12)
    want = np.zeros((3, d))
    want[0, 4] = want[1, 0] = want[2, 2] = 1.0
    assert np.allclose(np.abs(basis), want, atol=1e-12)
