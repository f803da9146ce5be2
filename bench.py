#!/usr/bin/env python3
"""UniFrac distance-matrix benchmark on one MI355X.

Metric: UniFrac pair-node updates per second (one update = one sample pair
times one non-root branch; a full matrix is N(N-1)/2 * (M-1) updates).

Default workload (synthetic, the largest single-table size the paper names):
a random-merge rooted binary tree with 200,000 tips (399,999 nodes),
Exponential(mean 0.05) branch lengths; 50,000 samples with ~1,000 distinct
Zipf(1.1)-popular tips each and round(LogNormal(2, 1.5)) + 1 counts; seed 103.
The 25,000-sample table of the same laws (seed 102) is --workload C2.

One step = the whole hot path over that table from the inputs resident on the
device: the per-sample scalars, the sparse split of each variant (branch
sample counts, list fill, list sort), then the weighted-normalized matrix and
the unweighted matrix, each with the chunked dense embedding, accumulation,
FP64 finalize into a condensed FP64 matrix and the PCoA row means and grand
mean.  By default both run sparse aware: branches touched by many samples on
the dense kernel (fixed-point stripe kernel, weighted; split-BF16 Gram on MFMA,
unweighted), every other branch as exact fixed-point sums over the sample
pairs that share it, with the automatic dense-set cost model.  Printed: one
JSON line on stdout.

    python bench.py [--steps K] [--warmup W] [--workload C1|C2|C3|C4|C5]
                    [--weighted-precision P] [--unweighted-precision P]
                    [--split-threshold F] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Vector-ALU issue slots per second: the published vector peaks count one FMA
# (2 flops) per slot: FP32 157.3 TFLOP/s -> 7.86e13 slots/s, FP64 78.6 -> 3.93e13.
# A non-FMA add/subtract occupies one slot, so a kernel doing c ops per update
# is bounded by slots/c updates per second.
PEAK_VALU_SLOTS = {"fp32": 157.3e12 / 2, "fp64": 78.6e12 / 2}
PEAK_BF16_MFMA = 2.5e15                         # dense BF16 MFMA FLOP/s
PEAK_HBM = 8.0e12


# the distance kernels, and the host code whose split cost model fixes how much
# work each of their launches does
KERNEL_SOURCES = ("uf_kernels.hip", "uf_split.hip", "uf_device.h", "uf_internal.h", "uf_host.hip")


def kernel_source_hash() -> str:
    """Hash of the sources the committed counter summaries were taken with."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2107_05397_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    for line in open(path):
        parts = line.split()
        if len(parts) >= 6 and parts[0] == "traffic" and parts[1] == kernel and \
                parts[2] == f"workload={workload}" and parts[3] == f"sha={want}":
            fetch = float(parts[4].split("=")[1])
            write = float(parts[5].split("=")[1])
            return {"bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
                    "write_bytes_per_launch": write, "source": "profiles/hbm_traffic.md"}
    return None


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def sampled_error(tree, table, pairs, variant, got) -> float:
    """Max |GPU - oracle| over sampled pairs (CPU leg only)."""
    import numpy as np
    import oracle
    want = oracle.dm_pairs(tree, table, pairs, variant)
    return float(np.max(np.abs(np.asarray(got) - want)))


def cpu_baseline(tree, table, target_s: float, variants=("weighted_normalized", "unweighted")):
    """Time the C oracle (FP64, OpenMP on all host cores) on a bounded sample:
    all pairs among the first n samples, the given variants, full tree."""
    import numpy as np  # noqa: F401
    import synth
    from oracle import core
    core.build(force=False)
    nb = tree.n_nodes - 1

    def run(n):
        sub = synth.subset_rows(table, np.arange(n))
        t0 = time.perf_counter()
        for v in variants:
            _, used = core.dm(tree, sub, v)
        return time.perf_counter() - t0, used

    # pair work grows as n^2 and per-sample work as n: probe, then resize once if the
    # first sample ran well short of the target
    n = 64
    secs, used = run(n)
    for _ in range(2):
        if secs >= 0.5 * target_s:
            break
        n = int(min(n * (target_s / max(secs, 1e-3)) ** 0.5, 3000))
        log(f"cpu baseline: resizing the sample to {n} samples")
        secs, used = run(n)
    updates = len(variants) * n * (n - 1) / 2 * nb
    return {"value": updates / secs, "unit": "pair-node updates/s", "cores": int(used),
            "kind": "oracle",
            "sample": f"all {n * (n - 1) // 2} pairs among the first {n} samples, "
                      f"{' + '.join(variants)}, full {tree.n_nodes}-node tree, FP64 C oracle; "
                      f"{secs:.1f} s",
            "seconds": secs, "host_cpus": os.cpu_count()}


def bench_batch(args) -> int:
    """Batching workload: many rarefied tables of uneven size on one tree,
    weighted normalized FP32, one persistent launch per chunk, one graph."""
    import numpy as np
    import synth
    log(f"generating {args.tables} rarefied tables")
    procs = max(1, min(16, os.cpu_count() or 1))
    tree, tables = synth.batch_tables(n_tables=args.tables, processes=procs)
    import torch
    import paper_2107_05397_amd as uf
    torch.cuda.set_device(0)
    m = tree.n_nodes
    sizes = [t.n_samples for t in tables]
    pairs = sum(n * (n - 1) // 2 for n in sizes)
    U = pairs * (m - 1)
    log(f"tables={len(tables)} samples={sum(sizes)} (min {min(sizes)}, max {max(sizes)}) "
        f"pairs={pairs} updates={U:.3e}")
    ut = uf.Tree(tree.parent, tree.length)
    uts = [uf.Table(ut, t.indptr, t.tips, t.counts) for t in tables]
    b = uf.Batch(ut, uts, tune_cache=args.tune_cache)
    log(f"workspace {b.workspace_size() / 2**30:.1f} GiB, config {b.config()}")
    tune_ms = b.autotune(args.tune_cache)
    log(f"autotuned config {b.config()} (first-chunk band time {tune_ms:.1f} ms)")
    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        b.run(use_graph=True, stream=stream)
        torch.cuda.synchronize()
        log(f"warmup {k + 1}/{args.warmup} done")
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.run(use_graph=True, stream=stream)
        torch.cuda.synchronize()
        log(f"step {k + 1}/{args.steps} done")
    graph_s = (time.perf_counter() - t0) / args.steps
    t1 = time.perf_counter()
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t1
    # the same tables as separate single-table calls
    t2 = time.perf_counter()
    for tu in uts:
        if tu.n_samples >= 2:
            emb = uf.Embedding(ut, tu)
            uf.dm(emb, "weighted_normalized", "fp32", out_dtype=torch.float32, stream=stream)
    torch.cuda.synchronize()
    separate_s = time.perf_counter() - t2
    # the same tables through the sparse-aware split, one call each (embeddings and
    # splits built before the timed region, as for the batch)
    embs = [uf.Embedding(ut, tu) for tu in uts if tu.n_samples >= 2]
    uf.set_split_threshold(None)
    for e in embs:
        uf.split_stats(e, "weighted_normalized")
    split_outs = [torch.empty(e.n_samples * (e.n_samples - 1) // 2, dtype=torch.float32, device="cuda")
                  for e in embs]
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for e, o in zip(embs, split_outs):
        uf.dm(e, "weighted_normalized", "fp32_split", out_dtype=torch.float32, out=o, stream=stream)
    torch.cuda.synchronize()
    split_s = time.perf_counter() - t3
    log(f"per-table split calls: {split_s:.2f}s")
    del embs, split_outs
    # the batch itself in sparse-split mode: per-table splits on forked streams, one graph
    bs = uf.Batch(ut, uts)
    bs.set_precision("fp32_split")
    split_tune_ms = bs.autotune()
    bs.run(use_graph=True, stream=stream)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(max(args.steps, 1)):
        bs.run(use_graph=True, stream=stream)
    torch.cuda.synchronize()
    split_graph_s = (time.perf_counter() - t4) / max(args.steps, 1)
    log(f"split batch graph: {split_graph_s:.3f}s")
    del bs
    outs = b.run(use_graph=True, stream=stream)
    torch.cuda.synchronize()
    # GPU values of a few sampled pairs, compared with the oracle in the CPU leg
    rng = np.random.default_rng(1)
    samples = []
    for r in rng.choice(len(tables), size=3, replace=False):
        n = sizes[r]
        ii = rng.choice(n, size=8, replace=False)
        pr = [(int(min(a, c)), int(max(a, c))) for a, c in zip(ii[:4], ii[4:])]
        idx = torch.tensor([uf.condensed_index(n, a, c) for a, c in pr], device="cuda")
        samples.append((int(r), pr, outs[r][idx].double().cpu().numpy()))
    full_oracle = []
    if args.oracle_smallest > 0 and not args.no_cpu_baseline:
        # CPU leg: whole tables against the FP64 C oracle (all host cores)
        from oracle import core
        core.build(force=False)
        for r in np.argsort(sizes, kind="stable")[:args.oracle_smallest]:
            t1 = time.perf_counter()
            want, used = core.dm(tree, tables[int(r)], "weighted_normalized")
            secs = time.perf_counter() - t1
            got = outs[int(r)].double().cpu().numpy()
            err = np.abs(got - want)
            full_oracle.append({"table": int(r), "n_samples": int(sizes[r]), "pairs": int(err.size),
                                "max_abs_err": float(err.max()), "mean_abs_err": float(err.mean()),
                                "oracle_seconds": secs, "oracle_threads": int(used)})
            log(f"table {int(r)} (n={sizes[r]}) in full vs the oracle: max|err| {err.max():.3e}, "
                f"mean {err.mean():.3e} ({secs:.1f}s on {used} threads)")
    cpu = None
    if not args.no_cpu_baseline:
        # CPU leg: the oracle timed on a bounded sample of the smallest table, and the
        # sampled GPU pairs checked against it
        small = int(np.argmin(sizes))
        cpu = cpu_baseline(tree, tables[small], args.cpu_seconds, variants=("weighted_normalized",))
        cpu["sampled_parity_max_abs_err"] = max(
            sampled_error(tree, tables[r], pr, "weighted_normalized", got) for r, pr, got in samples)
        log(f"sampled parity vs oracle: {cpu['sampled_parity_max_abs_err']:.3e}")
    slots = 2 * U / graph_s
    rec = {
        "metric": "UniFrac pair-node updates/s (1 GPU), batched tables",
        "value": U / graph_s, "unit": "pair-node updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": graph_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C4: {len(tables)} rarefied tables (depth 5000), "
                               f"{min(sizes)}-{max(sizes)} samples each, {m}-node tree, "
                               f"weighted normalized FP32, one hipGraph",
                   "n_tables": len(tables), "samples": sum(sizes), "pairs": pairs,
                   "updates_per_step": U, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": slots / 1e12,
                     "peak": PEAK_VALU_SLOTS["fp32"] / 1e12, "unit": "Tops/s",
                     "frac": slots / PEAK_VALU_SLOTS["fp32"], "traffic": None,
                     "note": "VALU lane-ops (2 per update) over the whole batch (embed + "
                             "persistent band + finalize) per step; peak 256 CU x 128 lanes/clk "
                             "x 2.4 GHz"},
        "extra": {"graph_s": graph_s, "eager_batch_s": eager_s,
                  "separate_single_table_calls_s": separate_s,
                  "separate_split_calls_s": split_s,
                  "split_batch_graph_s": split_graph_s,
                  "split_batch_updates_per_s": U / split_graph_s,
                  "split_batch_autotune_ms": split_tune_ms,
                  "autotuned_config": dict(zip(("stage_branches", "wgs_per_cu", "chunk_nodes", "tile_stripes"),
                                               b.config())),
                  "autotune_first_chunk_ms": tune_ms,
                  "smallest_tables_vs_oracle": full_oracle},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    return 0


def bench_placement(args) -> int:
    """Learned placement: train the encoder on a 25,000-sample reference table
    (exact weighted-normalized targets), place 10,000 new samples."""
    import numpy as np
    import synth
    c = synth.CONFIGS["C5"]
    log("generating reference and query tables")
    tree, ref = synth.config("C2", n_samples=c["n_ref"])
    query = synth.gen_table_zipf(c["n_query"], np.arange(tree.n_tips), c["nnz"], c["query_seed"])
    import torch
    from paper_2107_05397_amd import placement
    torch.cuda.set_device(0)
    res = placement.experiment(tree, ref, query, epochs=args.epochs, objective=args.objective,
                               dist_weight=args.dist_weight, rank_weight=args.rank_weight,
                               tau=args.tau, lr=args.lr, skip_init=args.skip_init,
                               batch_pairs=args.batch_pairs, log=log)
    rec = {
        "metric": "placement queries/s (1 GPU) with recall@10 against exact UniFrac",
        "value": c["n_query"] / res["placement_s"], "unit": "queries/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": res["placement_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"C5: {res['n_ref']} reference + {res['n_query']} query samples "
                               f"on the {tree.n_nodes}-node tree; encoder {res['dims']}",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "kernel": "k_gemm_bf16 (encoder training GEMMs)",
                     "achieved": res["train_gemm_tflops"], "peak": PEAK_BF16_MFMA / 1e12,
                     "unit": "TFLOP/s",
                     "frac": (res["train_gemm_tflops"] * 1e12 / PEAK_BF16_MFMA
                              if res["train_gemm_tflops"] else None),
                     "traffic": None,
                     "note": "multiply-add flops of every training step's forward, data-gradient "
                             "and weight-gradient GEMMs over the GEMMs' own event-timed duration"},
        "extra": res,
    }
    print(json.dumps(rec), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--epochs", type=int, default=8, help="C5: training epochs")
    ap.add_argument("--objective", default="triplets", choices=["triplets", "pairs"],
                    help="C5: ranking loss over triples, or distance regression over pairs")
    ap.add_argument("--dist-weight", type=float, default=0.0, help="C5: regression weight")
    ap.add_argument("--rank-weight", type=float, default=1.0, help="C5: ranking weight")
    ap.add_argument("--tau", type=float, default=0.03, help="C5: ranking temperature")
    ap.add_argument("--lr", type=float, default=1e-4, help="C5: Adam learning rate")
    ap.add_argument("--batch-pairs", type=int, default=4096,
                    help="C5: pairs per training step (triples: half as many)")
    ap.add_argument("--skip-init", default="pca", choices=["pca", "gaussian"],
                    help="C5: start of the encoder's linear path")
    ap.add_argument("--tables", type=int, default=64, help="C4: number of tables")
    ap.add_argument("--tune-cache", default=None, help="C4: autotuner cache path")
    ap.add_argument("--samples", type=int, default=None, help="override the sample count")
    ap.add_argument("--weighted-precision", default="fp32_split",
                    choices=["fp32_split", "fp32", "fp64"])
    ap.add_argument("--split-threshold", type=float, default=None,
                    help="dense-set fraction of the sparse-aware split (default: automatic)")
    ap.add_argument("--split-threshold-weighted", type=float, default=None)
    ap.add_argument("--split-threshold-unweighted", type=float, default=None)
    ap.add_argument("--unweighted-precision", default="mfma_split",
                    choices=["mfma", "mfma_split", "fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-smallest", type=int, default=0,
                    help="C4: compare the N smallest tables in full with the FP64 C oracle")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target length of the one-core oracle run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy first (HBM counter calibration)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the plain weighted FP32 kernel over all branches")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the plain-kernel and all-branch MFMA comparison runs")
    ap.add_argument("--no-statistics", action="store_true",
                    help="skip the PCoA and Mantel timings on the step's matrices")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(stripe-range sharding across GPUs is a design note, not code). "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    if args.workload == "C4":
        return bench_batch(args)
    if args.workload == "C5":
        return bench_placement(args)

    return bench_matrix(args)


KERNEL_NAMES = ("sample_scalars", "branch_count", "split_fill", "sort_lists", "split_lengths",
                "embed_nm", "embed_pres", "band_wn_u32", "band_wn_f32", "band_wn_f64", "band_uw_f32",
                "band_uw_f64", "gram_mfma", "rare_slots_wn", "rare_slots_uw", "finalize", "row_sums")
PREP_KERNELS = ("sample_scalars", "branch_count", "split_fill", "sort_lists", "split_lengths")


def subset_ids(n: int, k: int = 2000):
    """k samples spread evenly over [0, n): every (n // k)-th (all of them if n <= k)."""
    import numpy as np
    step = max(1, n // k)
    return np.arange(0, n, step)[:k]


def bench_matrix(args) -> int:
    """Distance matrices of one table: C1, C2 or C3 (default)."""
    import numpy as np
    import torch

    import paper_2107_05397_amd as uf
    import synth

    torch.cuda.set_device(0)
    log(f"generating {args.workload} workload")
    tree, table = synth.config(args.workload, n_samples=args.samples)
    n = table.n_samples
    m = tree.n_nodes
    pairs = n * (n - 1) // 2
    U = pairs * (m - 1)
    log(f"n={n} nodes={m} pairs={pairs} updates/variant={U:.3e}")
    t = uf.Tree(tree.parent, tree.length)
    tb = uf.Table(t, table.indptr, table.tips, table.counts)
    emb = uf.Embedding(t, tb)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        # a plain copy kernel of known size: reads 1 GiB and writes 1 GiB
        src = torch.ones(2**28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB read + 1 GiB written")

    wp, up = args.weighted_precision, args.unweighted_precision
    split_w, split_u = wp == "fp32_split", up == "mfma_split"
    splits = {}
    uf.set_split_threshold(args.split_threshold)
    if args.split_threshold_weighted is not None:
        uf.set_split_threshold(args.split_threshold_weighted, "weighted_normalized")
    if args.split_threshold_unweighted is not None:
        uf.set_split_threshold(args.split_threshold_unweighted, "unweighted")
    for var, on in (("weighted_normalized", split_w), ("unweighted", split_u)):
        if on:
            splits[var] = uf.split_stats(emb, var)
            log(f"split {var}: {splits[var][0]} dense branches, {splits[var][1]} shared lists, "
                f"{splits[var][2]:.3e} pairs")
    out_w = torch.empty(pairs, dtype=torch.float64, device="cuda")
    out_u = torch.empty(pairs, dtype=torch.float64, device="cuda")
    ws_w = torch.empty(uf.workspace_size(emb, "weighted_normalized", wp, row_stats=True),
                       dtype=torch.uint8, device="cuda")
    ws_u = torch.empty(uf.workspace_size(emb, "unweighted", up, row_stats=True),
                       dtype=torch.uint8, device="cuda")
    log(f"workspace: weighted {ws_w.numel() / 2**30:.2f} GiB, unweighted {ws_u.numel() / 2**30:.2f} GiB")

    def prepare():
        # the device-side part of the embedding pass: per-sample scalars and the sparse
        # split of each variant, from the table and tree resident on the device
        emb.prepare(scalars=True, split_weighted=split_w, split_unweighted=split_u, stream=stream)

    def matrices():
        uf.dm(emb, "weighted_normalized", wp, out=out_w, row_means=True, workspace=ws_w,
              stream=stream)
        uf.dm(emb, "unweighted", up, out=out_u, row_means=True, workspace=ws_u, stream=stream)

    def step():
        prepare()
        matrices()

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {k + 1}/{args.warmup} done")
    uf.profile_reset()
    uf.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {k + 1}/{args.steps} done ({time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    uf.profile_enable(False)
    ms_step = elapsed / args.steps * 1e3
    value = 2 * U / (ms_step / 1e3)

    kern = {}
    for name in KERNEL_NAMES:
        tot, cnt = uf.profile_read(name)
        if cnt:
            kern[name] = {"total_ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps,
                          "avg_ms_per_launch": tot / cnt}
    # the same matrices with the preparation reused (split and scalars from the last step)
    warm_steps = max(1, min(args.steps, 5))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(warm_steps):
        matrices()
    torch.cuda.synchronize()
    warm_ms = (time.perf_counter() - t1) / warm_steps * 1e3
    t1 = time.perf_counter()
    prepare()
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t1) * 1e3
    log(f"step {ms_step:.1f} ms; matrices alone {warm_ms:.1f} ms; preparation alone {prep_ms:.1f} ms")

    # dominant kernel: the weighted stripe kernel (FP64, FP32, or the 32-bit
    # fixed-point pass of the split), counted in VALU issue slots.  FP32/FP64 take 2
    # full-rate ops per update (subtract, add of |.|); fixed point takes one v_sad_u32
    # (|a - b| + acc), which a register-only probe measured at half the issue rate
    # of v_add_u32 (3.61e13 vs 6.55e13 lane-ops/s), i.e. 2 slots as well.  The peak
    # is the published 157.3 TFLOP/s FP32 counted as 78.6e12 slots/s (an FMA is 2
    # flops in one slot; = 256 CU x 128 lanes/clk x 2.4 GHz), half that for FP64.
    # With the split the stripe kernel visits only the dense branches.
    if wp == "fp64":
        band, peak_ops, kname = "band_wn_f64", PEAK_VALU_SLOTS["fp64"], "k_band<double,weighted>"
    elif "band_wn_u32" in kern:
        band, peak_ops, kname = "band_wn_u32", PEAK_VALU_SLOTS["fp32"], "k_band<uint32_t,weighted>"
    else:
        band, peak_ops, kname = "band_wn_f32", PEAK_VALU_SLOTS["fp32"], "k_band<float,weighted>"
    band_ms = kern[band]["total_ms_per_step"]
    band_updates = pairs * splits["weighted_normalized"][0] if split_w else U
    slots = 2 * band_updates / (band_ms / 1e3)
    traffic = measured_traffic(band, args.workload)
    roofline = {"bound": "alu", "kernel": kname,
                "achieved": slots / 1e12, "peak": peak_ops / 1e12,
                "unit": "Tops/s", "frac": slots / peak_ops, "traffic": traffic,
                "avg_launch_ms": kern[band]["avg_ms_per_launch"],
                "launches_per_step": kern[band]["launches_per_step"],
                "updates_per_launch": band_updates / kern[band]["launches_per_step"],
                "note": "VALU issue slots: 2 per pair-branch update (FP: subtract + add of |.|; "
                        "fixed point: one v_sad_u32, which issues at half rate); peak = published "
                        "157.3 TFLOP/s FP32 / 2 flops per FMA slot = 78.6e12 slots/s "
                        "(256 CU x 128 lanes/clk x 2.4 GHz), half that for FP64"}
    prep_kernel_ms = sum(kern[k]["total_ms_per_step"] for k in PREP_KERNELS if k in kern)
    extra = {"kernels": kern,
             "preparation": {"kernel_ms_per_step": prep_kernel_ms, "wall_ms": prep_ms,
                             "fraction_of_step": prep_ms / ms_step,
                             "what": "per-sample scalars + both variants' sparse splits "
                                     "(branch counts, list fill, list sort, lengths), "
                                     "host round trips included"},
             "matrices_with_preparation_reused": {"ms_per_step": warm_ms,
                                                  "updates_per_s": 2 * U / (warm_ms / 1e3)}}
    if splits:
        extra["split"] = {"threshold": args.split_threshold if args.split_threshold is not None
                          else "automatic", "band_updates_per_step": band_updates}
        for var, v in splits.items():
            name = "rare_slots_wn" if var == "weighted_normalized" else "rare_slots_uw"
            r_ms = kern.get(name, {}).get("total_ms_per_step", 0.0)
            extra["split"][var] = {"dense_branches": v[0], "shared_lists": v[1],
                                   "pairs_enumerated": v[2],
                                   "slot_kernel_pairs_per_s": v[2] / (r_ms / 1e3) if r_ms else None}
    if "gram_mfma" in kern:
        g_ms = kern["gram_mfma"]["total_ms_per_step"]
        g_upd = pairs * splits["unweighted"][0] if split_u else U
        extra["mfma_roofline"] = {"bound": "mfma", "achieved": 4 * g_upd / (g_ms / 1e3) / 1e12,
                                  "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                                  "frac": 4 * g_upd / (g_ms / 1e3) / PEAK_BF16_MFMA,
                                  "note": "2 BF16 MACs (l_hi, l_lo) = 4 flops per update"}

    # the 2,000-sample subset the accuracy is stated on, and a few sampled pairs
    ids = subset_ids(n)
    ia, ib = np.triu_indices(len(ids), 1)
    si, sj = ids[ia], ids[ib]
    sub_idx = torch.from_numpy(n * si - si * (si + 1) // 2 + (sj - si - 1)).to("cuda")
    rng = np.random.default_rng(0)
    pick = rng.choice(n, size=24, replace=False)
    sampled_pairs = [(int(min(a, b)), int(max(a, b))) for a, b in zip(pick[:12], pick[12:])]
    sidx = torch.tensor([uf.condensed_index(n, a, b) for a, b in sampled_pairs], device="cuda")
    subset_got = {"step_unweighted": out_u[sub_idx].cpu().numpy()}
    sampled_got = {"step_weighted_normalized": ("weighted_normalized", out_w[sidx].cpu().numpy()),
                   "step_unweighted": ("unweighted", out_u[sidx].cpu().numpy())}

    # Principal coordinates of the weighted matrix (10 axes, 20-column test matrix,
    # 3 power passes): 5 products B X, each reading the condensed matrix.
    if not args.no_statistics:
        dims, cols, q = 10, 20, 3
        omega = torch.tensor(synth.gaussian_matrix(n, cols, seed=17), dtype=torch.float64,
                             device="cuda")
        _, rw, gw = uf.dm(emb, "weighted_normalized", wp, out=out_w, row_means=True,
                          workspace=ws_w, stream=stream)
        uf.pcoa(out_w, n, dims, omega, power_iters=q, row_means=rw, grand_mean=gw, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, vals, tr = uf.pcoa(out_w, n, dims, omega, power_iters=q, row_means=rw, grand_mean=gw,
                              stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        products = q + 2
        extra["pcoa"] = {"seconds": dt, "dims": dims, "test_matrix_cols": cols, "power_iters": q,
                         "products": products,
                         "condensed_bytes_per_product": pairs * 8,
                         "effective_GBps": products * pairs * 8 / dt / 1e9,
                         "eigenvalues": [float(v) for v in vals[:5]],
                         "proportion_explained": [float(v / tr) for v in vals[:5]]}
        log(f"pcoa: {dt * 1e3:.1f} ms, top eigenvalues {vals[:3]}")
        del omega
        # Mantel test between the two matrices: 999 permutations (Pearson), 99 (Spearman)
        prng = np.random.default_rng(23)
        perms = torch.tensor(np.stack([prng.permutation(n) for _ in range(999)]).astype(np.int32),
                             device="cuda")
        extra["mantel"] = {}
        for method, k in (("pearson", 999), ("spearman", 99)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r, pv, _ = uf.mantel(out_w, out_u, n, method, perms[:k], stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            extra["mantel"][method] = {"seconds": dt, "permutations": k, "statistic": r,
                                       "p_value": pv,
                                       "pair_products_per_s": (k + 1) * pairs / dt}
            log(f"mantel {method}: {dt:.2f}s for {k} permutations, r={r:.4f} p={pv:.4f}")
        del perms
    del ws_w, ws_u

    # Comparison runs, each a whole call over the full problem with the inputs resident:
    # the unweighted plain stripe kernel (FP32) vs the MFMA Gram over all branches (the
    # "MFMA vs plain" figure, both at <= 1e-4 error on the subset); --extra adds the
    # plain weighted FP32 kernel over all branches.
    comparisons = [("unweighted_plain_fp32", "unweighted", "fp32"),
                   ("unweighted_mfma_all_branches", "unweighted", "mfma")]
    if args.extra:
        comparisons.append(("weighted_plain_fp32", "weighted_normalized", "fp32"))
    if not args.no_comparisons:
        for name, var, prec in comparisons:
            ws = torch.empty(uf.workspace_size(emb, var, prec), dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            uf.dm(emb, var, prec, out=out_w, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            del ws
            dt = time.perf_counter() - t1
            extra[name] = {"seconds": dt, "updates_per_s": U / dt}
            sampled_got[name] = (var, out_w[sidx].cpu().numpy())
            if var == "unweighted":
                subset_got[name] = out_w[sub_idx].cpu().numpy()
            log(f"comparison {name}: {dt:.2f}s")
        extra["mfma_speedup_over_plain_fp32"] = (extra["unweighted_plain_fp32"]["seconds"] /
                                                 extra["unweighted_mfma_all_branches"]["seconds"])
        t_all = extra["unweighted_mfma_all_branches"]["seconds"]
        extra["unweighted_mfma_all_branches"]["mfma_frac_whole_call"] = 4 * U / t_all / PEAK_BF16_MFMA
        # the FP64 weighted kernel on one GPU's share of the stripes (an eighth), the
        # size it would take on each of eight GPUs
        S = n // 2
        se = max(1, S // 8)
        share = torch.empty(se * n, dtype=torch.float64, device="cuda")
        uf.profile_reset()
        uf.profile_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        uf.dm_stripes(emb, "weighted_normalized", "fp64", 0, se, out=share, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        uf.profile_enable(False)
        f64_ms, _ = uf.profile_read("band_wn_f64")
        share_updates = se * n * (m - 1)
        f64_slots = 2 * share_updates / (f64_ms / 1e3)
        extra["weighted_fp64_stripe_share"] = {
            "stripes": [0, se], "seconds": dt, "updates": share_updates,
            "updates_per_s": share_updates / dt, "band_ms": f64_ms,
            "roofline": {"bound": "alu", "kernel": "k_band<double,weighted>",
                         "achieved": f64_slots / 1e12, "peak": PEAK_VALU_SLOTS["fp64"] / 1e12,
                         "unit": "Tops/s", "frac": f64_slots / PEAK_VALU_SLOTS["fp64"]}}
        # sampled pairs inside the share: (i, (i + s + 1) mod n), s < se
        srng = np.random.default_rng(5)
        ss = srng.integers(0, se, size=12)
        si2 = srng.integers(0, n, size=12)
        share_pairs = [(int(i), int((i + s + 1) % n)) for i, s in zip(si2, ss)]
        sv = share.view(se, n)[torch.tensor(ss, device="cuda"), torch.tensor(si2, device="cuda")]
        sampled_got["weighted_fp64_stripe_share"] = ("weighted_normalized", sv.cpu().numpy(),
                                                     share_pairs)
        log(f"FP64 weighted on stripes [0, {se}): {dt:.2f}s, band {f64_ms:.0f} ms "
            f"({f64_slots / PEAK_VALU_SLOTS['fp64']:.2f} of the FP64 peak)")
        del share

    # arithmetic types of the kernels that ran: weighted dense part, split pair sums,
    # unweighted dense part
    parts = [{"band_wn_u32": "u32", "band_wn_f32": "f32", "band_wn_f64": "f64"}[band]]
    if splits:
        parts.append("u64")
    parts.append({"mfma": "bf16", "mfma_split": "bf16", "fp32": "f32", "fp64": "f64"}[up])
    dtype = "+".join(dict.fromkeys(parts))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_leg(tree, table, ids, subset_got, sampled_got, sampled_pairs, args.cpu_seconds)

    rec = {
        "metric": "UniFrac pair-node updates/s (1 GPU)",
        "value": value,
        "unit": "pair-node updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: random-merge tree {tree.n_tips} tips "
                               f"({m} nodes), {n} samples, both variants from the device-resident "
                               f"table (scalars, sparse splits, matrices), condensed FP64 "
                               f"output + PCoA means",
                   "n_samples": n, "n_nodes": m, "pairs": pairs, "updates_per_step": 2 * U,
                   "weighted_precision": wp, "unweighted_precision": up,
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)
    return 0


def cpu_leg(tree, table, ids, subset_got, sampled_got, sampled_pairs, one_core_seconds):
    """The FP64 C oracle on the host: all cores on the 2,000-sample subset's
    unweighted matrix (the reference of the MFMA accuracy figures), one core on a
    small leading sample for the per-core rate, and the sampled pairs."""
    import numpy as np
    import oracle
    import synth
    from oracle import core
    core.build(force=False)
    nb = tree.n_nodes - 1
    sub = synth.subset_rows(table, ids)
    k = len(ids)
    log(f"cpu leg: oracle on the {k}-sample subset (unweighted, all cores)")
    t0 = time.perf_counter()
    want, used = core.dm(tree, sub, "unweighted")
    secs = time.perf_counter() - t0
    updates = k * (k - 1) / 2 * nb
    subset_err = {}
    for name, got in subset_got.items():
        e = np.abs(got - want)
        subset_err[name] = {"max_abs_err": float(e.max()), "mean_abs_err": float(e.mean())}
    log(f"cpu leg: {secs:.1f}s on {used} threads; subset errors {subset_err}")
    # one core: all pairs among the first n1 samples, sized to about one_core_seconds
    n1 = 16
    t1 = time.perf_counter()
    core.dm(tree, synth.subset_rows(table, np.arange(n1)), "unweighted", n_threads=1)
    s1 = time.perf_counter() - t1
    n1 = int(min(max(16, n1 * (one_core_seconds / max(s1, 1e-3)) ** 0.5), 400))
    t1 = time.perf_counter()
    core.dm(tree, synth.subset_rows(table, np.arange(n1)), "unweighted", n_threads=1)
    s1 = time.perf_counter() - t1
    one = {"value": n1 * (n1 - 1) / 2 * nb / s1, "unit": "pair-node updates/s", "cores": 1,
           "sample": f"all {n1 * (n1 - 1) // 2} pairs among the first {n1} samples, unweighted; "
                     f"{s1:.1f} s"}
    sampled_err = {}
    for name, item in sampled_got.items():
        var, got = item[0], item[1]
        prs = item[2] if len(item) > 2 else sampled_pairs
        sampled_err[name] = float(np.max(np.abs(np.asarray(got) - oracle.dm_pairs(tree, table, prs, var))))
    log(f"cpu leg: sampled-pair errors {sampled_err}")
    return {"value": updates / secs, "unit": "pair-node updates/s", "cores": int(used),
            "kind": "oracle",
            "sample": f"all {k * (k - 1) // 2} pairs of a {k}-sample subset (every "
                      f"{int(ids[1] - ids[0]) if k > 1 else 1}th sample), unweighted, full "
                      f"{tree.n_nodes}-node tree, FP64 C oracle; {secs:.1f} s",
            "seconds": secs, "host_cpus": os.cpu_count(), "one_core": one,
            "subset_abs_err": subset_err, "sampled_pairs_max_abs_err": sampled_err}


if __name__ == "__main__":
    sys.exit(main())
