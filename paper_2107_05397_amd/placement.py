"""Learned placement of new samples against a reference set.

The paper's introduction motivates data reuse: new sample collections are
placed into the context of existing data.  Here an encoder maps a sample's
embedded proportions to a space whose Euclidean distances approximate
weighted-normalized UniFrac:

    x = R (l * u)                       sparse random projection (uf_project)
    z = MLP(x)                          BF16 MFMA forward kernels
    loss = mean (||z_a - z_b|| - d_ab)^2 over pairs with exact targets d

Placement of a query: its k' nearest references in z-space are candidates;
the exact distance (uf_dm_rerank_weighted_normalized) re-ranks them and the
best k are returned.  The exact method is both the fallback (k' = all) and
the reference for the encoder's error.

This module only orchestrates library calls (argument marshalling, pair
sampling on the host, the epoch loop); every numerical step runs in the HIP
kernels behind include/uf.h.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import (MLP, Sparse, gather_pairs, pca_basis, profile_enable, profile_read, profile_reset,
               rerank, sqdist, topk_rows)


def train(x, pair_a: np.ndarray, pair_b: np.ndarray, target, dims: Sequence[int],
          init_params, epochs: int = 5, batch_pairs: int = 4096, lr: float = 1e-3,
          seed: int = 0, rel_floor: float = 0.0, skip=None, weight_decay: float = 0.0,
          log=None) -> Tuple[MLP, List[float]]:
    """Train the encoder on (pair_a, pair_b, target) with Adam.

    x: device bfloat16 [N][d0] inputs; target: device FP32 [P] exact distances.
    Returns the MLP and the mean loss of every epoch.
    """
    import torch
    mlp = MLP(dims, max_rows=2 * batch_pairs, params=init_params, skip=skip)
    P = len(pair_a)
    pa_all = torch.as_tensor(np.asarray(pair_a, np.int32), device="cuda")
    pb_all = torch.as_tensor(np.asarray(pair_b, np.int32), device="cuda")
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses: List[float] = []
    step = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(P).astype(np.int64), device="cuda")
        # the epoch's order applied once; every batch is then a contiguous slice
        pa_e, pb_e, tg_e = pa_all[perm], pb_all[perm], target[perm]
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = 0
        for b0 in range(0, P - batch_pairs + 1 if P >= batch_pairs else 1, batch_pairs):
            s_ = slice(b0, b0 + batch_pairs)
            mlp.loss_grad(x, pa_e[s_], pb_e[s_], tg_e[s_], loss=loss, rel_floor=rel_floor)
            step += 1
            mlp.adam(lr, step, weight_decay=weight_decay)
            acc += loss
            nb += 1
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {losses[-1]:.3e}")
    return mlp, losses


def train_triplets(x, anchor: np.ndarray, near: np.ndarray, far: np.ndarray, d_near, d_far,
                   dims: Sequence[int], init_params, epochs: int = 5, batch_triples: int = 4096,
                   lr: float = 1e-3, rank_weight: float = 1.0, tau: float = 0.01,
                   dist_weight: float = 0.0, seed: int = 0, skip=None, weight_decay: float = 0.0,
                   log=None) -> Tuple[MLP, List[float]]:
    """Train the encoder on (anchor, near, far) triples with the ranking loss
    (uf_mlp_triplet_loss_grad) and Adam.  d_near, d_far: device FP32 exact
    distances d(anchor, near), d(anchor, far).  Returns the MLP and the mean loss
    of every epoch."""
    import torch
    mlp = MLP(dims, max_rows=3 * batch_triples, params=init_params, skip=skip)
    T = len(anchor)
    dev = [torch.as_tensor(np.asarray(v, np.int32), device="cuda") for v in (anchor, near, far)]
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses: List[float] = []
    step = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(T).astype(np.int64), device="cuda")
        # the epoch's order applied once; every batch is then a contiguous slice
        a_e, p_e, q_e = (v[perm] for v in dev)
        dn_e, df_e = d_near[perm], d_far[perm]
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = 0
        for b0 in range(0, T - batch_triples + 1 if T >= batch_triples else 1, batch_triples):
            s_ = slice(b0, b0 + batch_triples)
            mlp.triplet_loss_grad(x, a_e[s_], p_e[s_], q_e[s_], dn_e[s_], df_e[s_],
                                  rank_weight=rank_weight, tau=tau, dist_weight=dist_weight,
                                  loss=loss)
            step += 1
            mlp.adam(lr, step, weight_decay=weight_decay)
            acc += loss
            nb += 1
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {losses[-1]:.3e}")
    return mlp, losses


def train_step_flops(dims: Sequence[int], rows: int, skip: bool) -> int:
    """Multiply-add flops of one training step's GEMMs over `rows` rows: the
    forward product of every layer, every weight gradient, and the data gradient
    of every layer but the first (the input needs none); the linear path adds a
    forward product and a weight gradient."""
    mac = sum(dims[l] * dims[l + 1] for l in range(len(dims) - 1))
    mac_data = sum(dims[l] * dims[l + 1] for l in range(1, len(dims) - 1))
    total = 2 * mac + mac_data
    if skip:
        total += 2 * dims[0] * dims[-1]
    return 2 * rows * total


def place(z_ref, z_q, q_sparse: Sparse, r_sparse: Sparse, k_candidates: int, k: int = 10,
          d=None):
    """k nearest references of every query: candidates in z-space, exact re-rank.
    d: the squared z-space distances [nq][n_ref] if already computed (sqdist).

    Returns (idx int32 [nq][k], exact FP64 distances [nq][k], candidate idx).
    """
    import torch
    if d is None:
        d = sqdist(z_q, z_ref)
    cand, _ = topk_rows(d, k_candidates)
    del d
    nq = z_q.shape[0]
    qids = torch.arange(nq, dtype=torch.int32, device="cuda")
    exact = rerank(q_sparse, r_sparse, qids, cand)
    best, _ = topk_rows(exact.float(), k)
    idx = torch.gather(cand, 1, best.long())
    ex = torch.gather(exact, 1, best.long())
    return idx, ex, cand


def recall_at_k(found_idx, exact_cross, k: int = 10) -> float:
    """Tie-tolerant recall: a returned reference counts when its exact distance
    is <= the exact k-th smallest distance of that query.  exact_cross: device
    FP32 [nq][n_ref] exact distances."""
    import torch
    _, truth = topk_rows(exact_cross, k)
    kth = truth[:, k - 1:k]
    got = torch.gather(exact_cross, 1, found_idx.long())
    return float((got <= kth).float().mean().item())


def distance_error(z_q, z_ref, idx, exact_cross) -> float:
    """Mean |encoder distance - exact distance| over the returned neighbours."""
    import torch
    zq = z_q.unsqueeze(1)
    zr = z_ref[idx.long()]
    approx = torch.sqrt(((zq - zr) ** 2).sum(-1))
    ex = torch.gather(exact_cross, 1, idx.long())
    return float((approx - ex).abs().mean().item())


def experiment(tree, ref_table, q_table, dims=(4096, 1024, 1024, 128), epochs: int = 5,
               n_uniform: int = 1_000_000, n_near: int = 1_000_000, near_k: int = 50,
               batch_pairs: int = 4096, lr: float = 1e-3, k: int = 10,
               k_candidates=(10, 100), proj_seed: int = 7, init_seed: int = 11,
               pair_seed: int = 13, rel_floor: float = 0.02, input_scale: float = 1.0,
               skip: bool = True, weight_decay: float = 0.0, objective: str = "pairs",
               n_triplets: int = 1_000_000, rank_weight: float = 1.0, tau: float = 0.01,
               dist_weight: float = 0.0, far_k: int = 100, skip_init: str = "pca",
               log=None) -> Dict:
    """Train the encoder on a reference table and place a query table.

    Exact distances (training targets and ground truth) come from the
    weighted-normalized matrix of the union of both tables (reference rows
    first), computed by the FP32 stripe kernels.  objective "pairs": the
    distance regression over n_uniform uniform + n_near neighbour pairs;
    "triplets": the ranking loss over n_triplets (anchor, near, far) triples
    (near among the anchor's near_k nearest, far among its ranks near_k..far_k-1
    or uniform).  Returns metrics and timings.
    """
    if objective not in ("pairs", "triplets"):
        raise ValueError("objective is 'pairs' or 'triplets'")
    if skip_init not in ("pca", "gaussian"):
        raise ValueError("skip_init is 'pca' or 'gaussian'")
    import torch
    import synth
    from . import Embedding, Table, Tree, condensed_block, dm, project
    log = log or (lambda m: None)
    sync = torch.cuda.synchronize
    nr, nq = ref_table.n_samples, q_table.n_samples
    t_tree = Tree(tree.parent, tree.length)
    union = synth.Table(indptr=np.concatenate([ref_table.indptr, ref_table.indptr[-1] + q_table.indptr[1:]]),
                        tips=np.concatenate([ref_table.tips, q_table.tips]),
                        counts=np.concatenate([ref_table.counts, q_table.counts]))
    e_ref = Embedding(t_tree, Table(t_tree, ref_table.indptr, ref_table.tips, ref_table.counts))
    e_q = Embedding(t_tree, Table(t_tree, q_table.indptr, q_table.tips, q_table.counts))
    e_u = Embedding(t_tree, Table(t_tree, union.indptr, union.tips, union.counts))
    out: Dict = {"n_ref": nr, "n_query": nq, "dims": list(dims)}

    sync()
    t0 = time.perf_counter()
    d_union, _, _ = dm(e_u, "weighted_normalized", "fp32")
    sync()
    out["exact_union_dm_s"] = time.perf_counter() - t0
    n_all = nr + nq
    pairs_union = n_all * (n_all - 1) // 2
    out["exact_cross_pairs_s_estimate"] = out["exact_union_dm_s"] * (nr * nq) / pairs_union
    log(f"exact union matrix: {out['exact_union_dm_s']:.2f}s")
    cross = condensed_block(d_union, n_all, nr, nq, 0, nr)              # [nq][nr] exact
    # training data: uniform pairs + pairs from each reference's exact neighbours
    kn = near_k if objective == "pairs" else max(far_k, near_k + 1)
    neigh = np.empty((nr, kn), dtype=np.int32)
    step_rows = 4096
    for r0 in range(0, nr, step_rows):
        rr = min(step_rows, nr - r0)
        blk = condensed_block(d_union, n_all, r0, rr, 0, nr)
        idx, _ = topk_rows(blk, kn)
        neigh[r0:r0 + rr] = idx.cpu().numpy()
        del blk
    # the pairs also give the skip path's scale and the projection-only fit below
    pa, pb = synth.placement_pairs(nr, n_uniform, neigh[:, :near_k], n_near, seed=pair_seed)
    tg = gather_pairs(d_union, n_all, torch.as_tensor(pa, device="cuda"),
                      torch.as_tensor(pb, device="cuda"))
    if objective == "triplets":
        ta, tn, tf = synth.placement_triplets(nr, neigh, n_triplets, near_k=near_k,
                                              far_lo=near_k, seed=pair_seed + 1)
        d_near = gather_pairs(d_union, n_all, torch.as_tensor(ta, device="cuda"),
                              torch.as_tensor(tn, device="cuda"))
        d_far = gather_pairs(d_union, n_all, torch.as_tensor(ta, device="cuda"),
                             torch.as_tensor(tf, device="cuda"))
    del d_union
    # inputs
    pdims, psigns = synth.sparse_projection(tree.n_nodes, out_dim=dims[0], per_node=4, seed=proj_seed)
    sync()
    t1 = time.perf_counter()
    x_ref = project(t_tree, e_ref, pdims, psigns, out_dim=dims[0], scale=input_scale)
    sync()
    out["project_ref_s"] = time.perf_counter() - t1
    t2 = time.perf_counter()
    init = synth.mlp_init(dims, seed=init_seed)
    s_init = None
    if skip:
        # start from a linear metric: z = S x with the network's last layer at zero.
        # skip_init "pca": S = the top dims[-1] principal directions of the
        # projected reference set (uf_pca_basis), the linear map of that width that
        # keeps the most of the pairwise distances; "gaussian": a random map.  The
        # scale matches the median target.
        sel = torch.arange(min(4096, len(pa)), device="cuda")
        pa_t = torch.as_tensor(pa, device="cuda")[sel].long()
        pb_t = torch.as_tensor(pb, device="cuda")[sel].long()
        diff = x_ref[pa_t].float() - x_ref[pb_t].float()
        if skip_init == "pca":
            cols = min(dims[-1] + 32, 160, dims[0])
            omega = torch.tensor(synth.gaussian_matrix(dims[0], cols, seed=init_seed + 1),
                                 dtype=torch.float64, device="cuda")
            basis, pca_vals = pca_basis(x_ref, dims[-1], omega, power_iters=3)
            out["pca_init_s"] = time.perf_counter() - t2
            out["pca_top_eigenvalues"] = [float(v) for v in pca_vals[:5]]
            dx = (diff @ basis.T).norm(dim=1)
            ratio = float(tg[sel].median()) / max(float(dx.median()), 1e-30)
            s_init = basis.cpu().numpy() * np.float32(ratio)
        else:
            dx = diff.norm(dim=1)
            ratio = float(tg[sel].median()) / max(float(dx.median()), 1e-30)
            s_init = synth.gaussian_matrix(dims[-1], dims[0], seed=init_seed + 1) * np.float32(
                ratio / np.sqrt(dims[-1]))
        init[-1] = (np.zeros_like(init[-1][0]), np.zeros_like(init[-1][1]))
    profile_reset()
    profile_enable(True)
    if objective == "pairs":
        mlp, losses = train(x_ref, pa, pb, tg, dims, init, epochs=epochs, batch_pairs=batch_pairs,
                            lr=lr, rel_floor=rel_floor, skip=s_init, weight_decay=weight_decay,
                            log=log)
        rows_per_step, n_items = 2 * batch_pairs, len(pa)
        out["train_pairs"] = int(len(pa))
    else:
        # a batch of batch_pairs // 2 triples has 1.5x the rows of a pair batch
        bt = batch_pairs // 2
        mlp, losses = train_triplets(x_ref, ta, tn, tf, d_near, d_far, dims, init, epochs=epochs,
                                     batch_triples=bt, lr=lr, rank_weight=rank_weight, tau=tau,
                                     dist_weight=dist_weight, skip=s_init,
                                     weight_decay=weight_decay, log=log)
        rows_per_step, n_items, batch_pairs_eff = 3 * bt, len(ta), bt
        out["train_triplets"] = int(len(ta))
        out["rank_weight"], out["tau"], out["dist_weight"] = rank_weight, tau, dist_weight
    out["objective"] = objective
    sync()
    profile_enable(False)
    out["train_s"] = time.perf_counter() - t2
    out["train_losses"] = losses
    # the training GEMMs, timed with HIP events on the training stream
    per_batch = batch_pairs if objective == "pairs" else batch_pairs_eff
    steps = epochs * (n_items // per_batch if n_items >= per_batch else 1)
    flops = steps * train_step_flops(dims, rows_per_step, skip)
    out["train_steps"] = steps
    out["train_gemm_flops"] = flops
    for name in ("encoder_gemm", "encoder_colsum", "encoder_loss", "encoder_adam"):
        ms, cnt = profile_read(name)
        out[f"{name}_ms"] = ms
        out[f"{name}_launches"] = cnt
    gemm_s = out["encoder_gemm_ms"] / 1e3
    out["train_gemm_tflops"] = flops / gemm_s / 1e12 if gemm_s > 0 else None
    out["train_step_tflops"] = flops / max(out["train_s"], 1e-9) / 1e12

    def encode(x):
        z = torch.empty((x.shape[0], dims[-1]), dtype=torch.float32, device="cuda")
        rows = mlp.max_rows
        for r0 in range(0, x.shape[0], rows):
            mlp.forward(x[r0:r0 + rows], out=z[r0:r0 + rows])
        return z

    s_ref, s_q = Sparse(e_ref), Sparse(e_q)
    z_ref = encode(x_ref)
    sync()
    t3 = time.perf_counter()
    x_q = project(t_tree, e_q, pdims, psigns, out_dim=dims[0], scale=input_scale)
    z_q = encode(x_q)
    res = {}
    d_q = sqdist(z_q, z_ref)   # one z-space distance matrix serves every K'
    for kc in k_candidates:
        idx, ex, cand = place(z_ref, z_q, s_q, s_ref, kc, k, d=d_q)
        sync()
        res[kc] = (idx, ex, cand)
    del d_q
    out["placement_s"] = time.perf_counter() - t3          # project + encode + all kNN/re-rank
    for kc, (idx, ex, cand) in res.items():
        out[f"recall@{k}_kprime{kc}"] = recall_at_k(idx, cross, k)
        out[f"mean_abs_dist_err_kprime{kc}"] = distance_error(z_q, z_ref, idx, cross)
    # the method without the network: kNN on the projection itself
    xr, xq = x_ref.float(), x_q.float()
    for kc in k_candidates:
        idx, ex, cand = place(xr, xq, s_q, s_ref, kc, k)
        out[f"projection_only_recall@{k}_kprime{kc}"] = recall_at_k(idx, cross, k)
    # the encoder's starting point at its own width: the linear PCA map alone
    if skip and skip_init == "pca":
        zr_l, zq_l = (xr @ basis.T).contiguous(), (xq @ basis.T).contiguous()
        for kc in k_candidates:
            idx, ex, cand = place(zr_l, zq_l, s_q, s_ref, kc, k)
            out[f"pca_only_recall@{k}_kprime{kc}"] = recall_at_k(idx, cross, k)
        del zr_l, zq_l
    # encoder distances against exact ones on random pairs
    rng = np.random.default_rng(3)
    qi = torch.as_tensor(rng.integers(0, nq, 20000), device="cuda")
    ri = torch.as_tensor(rng.integers(0, nr, 20000), device="cuda")
    approx = torch.sqrt(((z_q[qi] - z_ref[ri]) ** 2).sum(1))
    out["mean_abs_dist_err_random_pairs"] = float((approx - cross[qi, ri]).abs().mean().item())
    # the projection as a distance estimate, with its best single scale (least
    # squares on the training pairs)
    sel = torch.arange(min(20000, len(pa)), device="cuda")
    pa_t = torch.as_tensor(pa, device="cuda")[sel].long()
    pb_t = torch.as_tensor(pb, device="cuda")[sel].long()
    dxt = (xr[pa_t] - xr[pb_t]).norm(dim=1).double()
    scale = float((dxt * tg[sel].double()).sum() / (dxt * dxt).sum().clamp_min(1e-300))
    dq = (xq[qi] - xr[ri]).norm(dim=1).double() * scale
    out["projection_only_mean_abs_dist_err_random_pairs"] = float(
        (dq - cross[qi, ri].double()).abs().mean().item())
    out["knn_dims_encoder"] = int(dims[-1])
    out["knn_dims_projection_only"] = int(dims[0])
    return out
