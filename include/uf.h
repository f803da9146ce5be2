/*
 * uf.h -- C ABI of the MI355X (gfx950) striped UniFrac library.
 *
 * What is computed.  The paper (section II) computes the all-pairs UniFrac
 * distance matrix, unweighted and weighted normalized, for the samples of a
 * sparse sample x feature count table whose features are the tips of a rooted
 * phylogeny, with the "Striped UniFrac" method: a postorder pass over the tree
 * gives every sample's embedded proportion on every branch, then the sample
 * pairs are accumulated stripe by stripe.  The definitions (standard UniFrac):
 *
 *   c[s,v] = sum of sample s's counts on the tips under node v;  T_s = total
 *   u[s,v] = c[s,v] / T_s ;  a[s,v] = (c[s,v] > 0)
 *   unweighted           d = sum_v l_v |a_iv - a_jv| / sum_v l_v max(a_iv, a_jv)
 *   weighted normalized  d = sum_v l_v |u_iv - u_jv| / sum_v l_v (u_iv + u_jv)
 *
 * with v over the non-root nodes and l_v the length of v's branch to its
 * parent.  A zero denominator gives d = 0.
 *
 * Stripes (the paper splits the problem into "a set of stripes" so a device
 * with little memory can compute it piece by piece, section II): with
 * S = floor(N/2) stripes, stripe s holds the N pairs (i, (i+s+1) mod N).  For
 * odd N every pair appears once; for even N the last stripe holds each of its
 * N/2 pairs twice.  Stripe-major output is [s_end - s_begin][N].  Condensed
 * output is the row-major upper triangle: pair i<j at N*i - i(i+1)/2 + j-i-1.
 *
 * PCoA inputs (the paper computes principal coordinates as part of the same
 * job, section II): with A_ij = -d_ij^2 / 2 (A_ii = 0), row means
 * r_i = (1/N) sum_j A_ij and grand mean g = (1/N) sum_i r_i, in FP64, summed
 * in a fixed order (bitwise reproducible).
 *
 * Conventions.  Every function returns uf_status (UF_OK = 0) and never throws
 * or aborts.  Host input arrays are copied during *_load; the caller may free
 * them afterwards.  Handles are owned by the library, immutable after creation
 * and may be shared between threads and streams.  Outputs, workspaces and
 * streams belong to the caller: device pointers (hipMalloc'd or torch CUDA
 * tensors on the current device) and a hipStream_t passed as void* (NULL =
 * the default stream).  Compute calls are asynchronous on that stream; errors
 * of a kernel surface at the next synchronising call.  On UF_ERR_ARG, _TREE,
 * _TABLE, _EMPTY_SAMPLE, _RANGE or _WORKSPACE nothing is written.  On
 * UF_ERR_DEVICE output contents are undefined.  uf_last_error_message()
 * describes the last failure of the calling thread.
 */
#ifndef UF_H
#define UF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UF_OK = 0,
    UF_ERR_ARG = 1,          /* null pointer, bad enum, size mismatch          */
    UF_ERR_TREE = 2,         /* not one root, cycle, bad parent, bad length     */
    UF_ERR_TABLE = 3,        /* bad CSR, feature not a tip, duplicate, count<0  */
    UF_ERR_EMPTY_SAMPLE = 4, /* a sample with zero total count                  */
    UF_ERR_RANGE = 5,        /* stripe range outside [0, floor(N/2)]            */
    UF_ERR_NOMEM = 6,        /* host or device allocation failed               */
    UF_ERR_DEVICE = 7,       /* HIP runtime error, or no usable gfx950 device   */
    UF_ERR_UNSUPPORTED = 8,  /* precision not offered for this variant          */
    UF_ERR_WORKSPACE = 9     /* workspace missing or smaller than required      */
} uf_status;

typedef enum {
    UF_FP64 = 0,        /* FP64 embedding and FP64 accumulation (vector ALU)           */
    UF_FP32 = 1,        /* FP32 embedding and FP32 accumulation, FP64 final division   */
    UF_MFMA_BF16X2 = 2, /* unweighted only: Gram product on MFMA, 0/1 x (l_hi + l_lo)  */
                        /* in BF16 with FP32 accumulation, FP64 final division         */
    UF_FP32_SPLIT = 3,  /* weighted only, sparse aware (the paper's "sparse-aware      */
                        /* optimizations", section II): branches touched by more than  */
                        /* a threshold fraction of the samples on the FP32 stripe      */
                        /* kernel; on every other branch only pairs that both touch it */
                        /* are visited, via sum|x-y| = sum x + sum y - 2 sum min(x,y), */
                        /* summed exactly in 2^-40 fixed point                         */
    UF_MFMA_SPLIT = 4   /* unweighted only, sparse aware: the dense branches as in     */
                        /* UF_MFMA_BF16X2; the Gram terms of every other branch, l for */
                        /* each pair of samples that both touch it, summed exactly in  */
                        /* 2^-40 fixed point.  Lengths are l_hi + l_lo throughout, as  */
                        /* in UF_MFMA_BF16X2                                           */
} uf_precision;

typedef enum { UF_CONDENSED = 0, UF_STRIPES = 1 } uf_layout;
typedef enum { UF_OUT_F64 = 0, UF_OUT_F32 = 1 } uf_out_dtype;

typedef struct uf_tree uf_tree;            /* host: validated tree in postorder    */
typedef struct uf_table uf_table;          /* host: validated table, tips by rank  */
typedef struct uf_embedding uf_embedding;  /* device: table + tree ready to stream */

/* ---- inputs ------------------------------------------------------------ */

/* Load a rooted tree given as a parent array.  parent[v] = -1 for the one
 * root, otherwise a node id in [0, n_nodes); ids may come in any order.
 * length[v] >= 0 and finite for every non-root v; the root's entry is
 * ignored.  Multifurcations, unary nodes and zero lengths are allowed.
 * Errors: UF_ERR_ARG (null, n_nodes < 1), UF_ERR_TREE. */
uf_status uf_tree_load(int64_t n_nodes, const int64_t* parent, const double* length,
                       uf_tree** out);
int64_t uf_tree_n_nodes(const uf_tree* tree);
int64_t uf_tree_n_tips(const uf_tree* tree);

/* Load a sample x tip count table in CSR form: indptr[n_samples+1] (indptr[0]
 * = 0, non-decreasing), tip_node[nnz] = node id of a tip of `tree`,
 * counts[nnz] >= 0.  A tip may appear at most once per sample.
 * Errors: UF_ERR_ARG, UF_ERR_TABLE, UF_ERR_EMPTY_SAMPLE (zero total). */
uf_status uf_table_load(const uf_tree* tree, int64_t n_samples, const int64_t* indptr,
                        const int64_t* tip_node, const int64_t* counts, uf_table** out);
int64_t uf_table_n_samples(const uf_table* table);

/* Upload tree + table to the current HIP device (library-owned memory) and
 * compute the per-sample FP64 scalars on `hip_stream`: the weighted
 * denominator part sum_v l_v u_sv (= sum_t D_t p_st, D_t = root distance)
 * and the unweighted sum_v l_v a_sv (for FP64, FP32-rounded and BF16
 * hi+lo lengths).  The dense per-branch embedding itself is produced chunk by
 * chunk inside the uf_dm_* calls.  The call synchronises `hip_stream` before
 * returning.  Errors: UF_ERR_ARG, UF_ERR_NOMEM, UF_ERR_DEVICE. */
uf_status uf_embed(const uf_tree* tree, const uf_table* table, void* hip_stream,
                   uf_embedding** out);
int64_t uf_embedding_n_samples(const uf_embedding* emb);

/* Copy the per-sample scalars to host arrays of n_samples doubles (nullable):
 * sw = sum_v l_v u_sv, wu = sum_v l_v a_sv (FP64 lengths). */
uf_status uf_embedding_scalars(const uf_embedding* emb, double* sw, double* wu);

/* Re-run the device-side preparation of an uploaded embedding on `hip_stream`,
 * from the table and tree already resident on the device: UF_PREP_SCALARS
 * recomputes the per-sample scalars (as uf_embed does); UF_PREP_SPLIT_WEIGHTED /
 * UF_PREP_SPLIT_UNWEIGHTED rebuild that variant's sparse-aware split (the part
 * of the embedding pass that lists, for every branch few samples touch, the
 * samples touching it, sorted, with their values) at the current threshold,
 * replacing the cached one; the per-branch sample counts are taken once for
 * both.  Without this call the split precisions build a missing split on first
 * use.  Results are identical either way; this exists so that the whole path
 * can be run, and timed, from device-resident inputs.  Synchronises hip_stream.
 * Errors: UF_ERR_ARG (NULL, unknown flag), UF_ERR_UNSUPPORTED (split limits),
 * UF_ERR_NOMEM, UF_ERR_DEVICE. */
enum { UF_PREP_SCALARS = 1, UF_PREP_SPLIT_UNWEIGHTED = 2, UF_PREP_SPLIT_WEIGHTED = 4 };
uf_status uf_embedding_prepare(const uf_embedding* emb, int what, void* hip_stream);

/* ---- workspace --------------------------------------------------------- */

/* Bytes of device workspace needed by a uf_dm_* call with the same
 * arguments.  weighted: 1 for the weighted-normalized variant, 0 for
 * unweighted.  want_row_stats: non-zero if the call will request row sums /
 * means.  The node-chunk length follows uf_set_chunk_nodes(). */
uf_status uf_workspace_size(const uf_embedding* emb, int weighted, uf_precision precision,
                            int64_t stripe_begin, int64_t stripe_end, int want_row_stats,
                            size_t* bytes);

/* Number of branches streamed per chunk (0 = automatic: as many as fit in
 * 8 GiB of chunk buffer).  Process-wide; affects later workspace sizes. */
void uf_set_chunk_nodes(int64_t nodes);

/* UF_FP32_SPLIT (weighted != 0), UF_MFMA_SPLIT (weighted == 0): the dense set
 * of that variant's split.  fraction in [0, 1]: a branch is dense when more
 * than fraction x N samples touch it.  fraction < 0 (the default): automatic,
 * a branch is dense when its c(c-1)/2 sample pairs would take longer as
 * fixed-point atomics than one pass of the variant's dense kernel over all
 * N x floor(N/2) stripe slots (rates measured on MI355X).  Process-wide; the
 * split of an embedding is built on first use and rebuilt when its variant's
 * threshold changes.  The split takes fewer than 2^24 samples and fewer than
 * 2^40 (sample, shared branch) memberships; beyond that the split
 * precisions return UF_ERR_UNSUPPORTED.  UF_ERR_ARG for fraction > 1 or NaN. */
uf_status uf_set_split_threshold(int weighted, double fraction);
/* Size of the split of `emb` for one variant at its current threshold: dense
 * branches, shared non-dense branches, and sample pairs enumerated over them
 * (builds the split if needed; synchronous). */
uf_status uf_split_stats(const uf_embedding* emb, int weighted, int64_t* n_dense,
                         int64_t* n_lists, int64_t* n_pairs);

/* ---- distance matrices --------------------------------------------------- */

/* Full N x N matrix, condensed layout (length N(N-1)/2, dtype out_dtype).
 * row_means (device, N doubles) and grand_mean (device, 1 double) are the
 * PCoA centring terms defined above; either may be NULL.
 * ws/ws_bytes: device workspace of at least uf_workspace_size(..., 0,
 * floor(N/2), row_means || grand_mean) bytes.
 * Precisions: weighted {UF_FP64, UF_FP32, UF_FP32_SPLIT}; unweighted
 * {UF_FP64, UF_FP32, UF_MFMA_BF16X2, UF_MFMA_SPLIT}.  Errors: UF_ERR_ARG,
 * UF_ERR_UNSUPPORTED,
 * UF_ERR_WORKSPACE, UF_ERR_DEVICE. */
uf_status uf_dm_unweighted(const uf_embedding* emb, uf_precision precision,
                           uf_out_dtype out_dtype, void* out_condensed,
                           double* row_means, double* grand_mean,
                           void* ws, size_t ws_bytes, void* hip_stream);
uf_status uf_dm_weighted_normalized(const uf_embedding* emb, uf_precision precision,
                                    uf_out_dtype out_dtype, void* out_condensed,
                                    double* row_means, double* grand_mean,
                                    void* ws, size_t ws_bytes, void* hip_stream);

/* Stripe range [stripe_begin, stripe_end) of the matrix, 0 <= begin <= end
 * <= floor(N/2).  layout UF_STRIPES: out is [end-begin][N] stripe-major.
 * layout UF_CONDENSED: out is a full condensed buffer of N(N-1)/2 entries of
 * which only the pairs in the range are written (so disjoint ranges fill it
 * piece by piece).  row_sums (device, N doubles, nullable) receives, for each
 * sample, the sum of -d^2/2 over the distinct pairs of the range that contain
 * it (overwritten, not accumulated).  The per-pair values are bitwise equal
 * to those of the full call with the same precision.
 * Errors: as above plus UF_ERR_RANGE. */
uf_status uf_dm_unweighted_stripes(const uf_embedding* emb, uf_precision precision,
                                   int64_t stripe_begin, int64_t stripe_end,
                                   uf_layout layout, uf_out_dtype out_dtype, void* out,
                                   double* row_sums, void* ws, size_t ws_bytes,
                                   void* hip_stream);
uf_status uf_dm_weighted_normalized_stripes(const uf_embedding* emb, uf_precision precision,
                                            int64_t stripe_begin, int64_t stripe_end,
                                            uf_layout layout, uf_out_dtype out_dtype,
                                            void* out, double* row_sums, void* ws,
                                            size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the full weighted-
 * normalized matrix as uf_dm_weighted_normalized, with the workspace taken from
 * a fixed device array of UF_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the caller still
 * passes the output and the optional row_means / grand_mean.  The node chunk
 * is sized to fit the array (at least 32 branches per chunk); larger matrices
 * return UF_ERR_RANGE with nothing written.  The largest N that fits: FP64
 * 2,877 with row means or grand mean requested, 4,064 without; FP32 3,328 and
 * 5,761.  Precisions:
 * UF_FP64, UF_FP32 (UF_ERR_UNSUPPORTED otherwise: the split precisions build
 * device-side lists).  Per-pair values are bitwise equal to those of
 * uf_dm_weighted_normalized with the same precision.  All calls on one device
 * share its array and leave their contents in it: calls that overlap on one
 * device (concurrent streams or threads) race.
 * Errors: UF_ERR_ARG, UF_ERR_UNSUPPORTED, UF_ERR_RANGE, UF_ERR_DEVICE. */
#define UF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
uf_status uf_dm_weighted_normalized_noalloc(const uf_embedding* emb, uf_precision precision,
                                            uf_out_dtype out_dtype, void* out_condensed,
                                            double* row_means, double* grand_mean,
                                            void* hip_stream);

/* ---- batches: many tables on one tree --------------------------------------- */

/* Many tables of uneven size on one tree -- e.g. rarefied replicates of a study
 * -- computed together: weighted normalized, FP32 accumulation, FP64 division,
 * condensed FP32 output per table.  Per node chunk, one kernel embeds every
 * table and one persistent kernel (#CU x wgs_per_cu resident blocks) drains
 * the (table, band tile) items of all tables from per-XCD atomic queues; the
 * whole sequence (all chunks, then finalize of every table) is captured once
 * into a hipGraph and replayed with one launch.  Per-pair values are bitwise
 * equal to uf_dm_weighted_normalized(UF_FP32) on each table alone.
 *
 * uf_batch_create: tables must have been loaded against `tree`; they are
 * concatenated and uploaded (library-owned device memory; synchronises
 * `hip_stream`).  tune_cache (nullable; else $UF_TUNE_CACHE, else defaults):
 * JSON written by uf_autotune; its entry for the batch's size bucket
 * ceil(log2(mean N)) sets the launch configuration.
 * Errors: UF_ERR_ARG, UF_ERR_NOMEM, UF_ERR_DEVICE. */
typedef struct uf_batch uf_batch;
uf_status uf_batch_create(const uf_tree* tree, const uf_table* const* tables, int64_t n_tables,
                          const char* tune_cache, void* hip_stream, uf_batch** out);
/* uf_batch_create followed by uf_batch_set_precision(prec) (UF_FP32 or
 * UF_FP32_SPLIT): the batch is the plan, and uf_batch_run executes it.  On an
 * error no batch is returned. */
uf_status uf_batch_plan_create(const uf_tree* tree, const uf_table* const* tables, int64_t n_tables,
                               uf_precision prec, const char* tune_cache, void* hip_stream,
                               uf_batch** out);
int64_t uf_batch_n_tables(const uf_batch* batch);
uf_status uf_batch_workspace_size(const uf_batch* batch, size_t* bytes);
/* Current launch configuration: branches staged per LDS block (8, 16 or 32),
 * resident blocks per CU, stripes per band tile (64, 128 or 256; a tile is 128
 * samples x that many stripes) and branches per chunk (each pointer nullable). */
uf_status uf_batch_config(const uf_batch* batch, int* stage_branches, int* wgs_per_cu,
                          int* tile_stripes, int64_t* chunk_nodes);
/* Set the launch configuration.  Valid when that many blocks of the kernel for
 * (stage_branches, tile_stripes) fit on one CU (LDS and registers, as the HIP
 * occupancy query reports).  A new tile size rebuilds the work items
 * (synchronous).  Results do not depend on the configuration.
 * Errors: UF_ERR_ARG (NULL, invalid configuration), UF_ERR_DEVICE. */
uf_status uf_batch_set_config(uf_batch* batch, int stage_branches, int wgs_per_cu,
                              int tile_stripes);
/* Arithmetic of the batch: UF_FP32 (default; the persistent stripe kernel above)
 * or UF_FP32_SPLIT: every table through the sparse-aware split of
 * uf_dm_weighted_normalized(UF_FP32_SPLIT) (results equal to that call on each
 * table alone).  The split mode builds one embedding and split per table here
 * (tables: the same ones, in the same order, as at creation; they and the tree
 * must stay alive), then runs the tables on up to 8 streams forked from and
 * joined back into the caller's stream, largest first, each stream with its own
 * workspace slot; the graph captures that fork and join.  uf_autotune picks the
 * stream count (1, 2, 4 or 8) in this mode.  The workspace size depends on the
 * mode: query it after this call.  Synchronous.
 * Errors: UF_ERR_ARG, UF_ERR_UNSUPPORTED (other precisions), UF_ERR_NOMEM,
 * UF_ERR_DEVICE. */
uf_status uf_batch_set_precision(uf_batch* batch, uf_precision prec, const uf_table* const* tables,
                                 void* hip_stream);
/* Compute every table: outs[r] is a device buffer of N_r(N_r-1)/2 floats
 * (NULL allowed for tables with fewer than 2 samples).  use_graph: replay the
 * captured graph (captured on first use and again whenever ws or outs change)
 * instead of launching kernel by kernel.  Asynchronous on hip_stream. */
uf_status uf_batch_run(uf_batch* batch, float* const* outs, int use_graph, void* ws,
                       size_t ws_bytes, void* hip_stream);
/* The self-written tile/stripe autotuner: time every tile size (64, 128, 256
 * stripes) x stage size (8, 16, 32 branches) at the two highest resident-block
 * counts that configuration allows, on the first 2,048 branches of the batch's
 * first chunk; keep the fastest (results are identical for all) and record it
 * in the JSON cache at tune_cache (nullable; else $UF_TUNE_CACHE; no file if
 * neither), keyed by the size bucket.
 * best_ms (nullable) receives the winner's time.  Synchronises hip_stream. */
uf_status uf_autotune(uf_batch* batch, void* ws, size_t ws_bytes, const char* tune_cache,
                      void* hip_stream, double* best_ms);
void uf_free_batch(uf_batch* batch);

/* ---- learned placement -------------------------------------------------------- */

/* Placing new samples against an existing reference set (the paper's
 * introduction: data reuse places new sample collections into the context of
 * existing data).  A sample's embedded proportions are projected, an MLP maps
 * them to a space whose Euclidean distances approximate weighted-normalized
 * UniFrac, the nearest references there are candidates, and the exact
 * distance re-ranks them.
 *
 * uf_project: x = scale * R (l * u) with R[d, v] = signs[v][j] / 2 at d = dims[v][j],
 * j < per_node (scale > 0 sets the input scale of the network); dims/signs are HOST arrays indexed by node id
 * ([n_nodes][per_node]; the root's row is ignored).  out_bf16: device
 * [N][out_dim] bfloat16.  Sums are exact fixed point (2^-40), so the result
 * is deterministic.  Synchronises hip_stream. */
uf_status uf_project(const uf_tree* tree, const uf_embedding* emb, const int32_t* dims,
                     const int8_t* signs, int64_t per_node, int64_t out_dim, double scale,
                     void* out_bf16, void* hip_stream);

/* A multilayer perceptron d0 -> d1 -> ... -> dL (ReLU between layers, none
 * after the last): BF16 weights and activations on MFMA with FP32
 * accumulation, FP32 master weights, biases and Adam moments.  Widths must be
 * multiples of 32; max_rows bounds the rows of one forward pass (2 x pairs
 * for training).  skip != 0 adds a trainable linear path: z = MLP(x) + S x
 * with S [dL][d0] (layer index n_layers in uf_mlp_set / uf_mlp_get).
 * Parameters start at zero; set them with uf_mlp_set. */
typedef struct uf_mlp uf_mlp;
uf_status uf_mlp_create(int64_t n_layers, const int64_t* dims, int64_t max_rows, int skip,
                        uf_mlp** out);
/* Host FP32 weights [d_{l+1}][d_l] and bias [d_{l+1}] of one layer (either
 * may be NULL; for the linear path only w).  Ordered on hip_stream: waits for
 * the work queued on it, copies, and synchronises it before returning. */
uf_status uf_mlp_set(uf_mlp* mlp, int64_t layer, const float* w, const float* b,
                     void* hip_stream);
/* Copy out one layer: what 0 = parameters, 1 = gradients, 2 = Adam first
 * moments, 3 = second moments.  Ordered after the work queued on hip_stream;
 * synchronises it. */
uf_status uf_mlp_get(const uf_mlp* mlp, int64_t layer, int what, float* w, float* b,
                     void* hip_stream);
/* z[i] = MLP(x[rows ? rows[i] : i]) for i < n; x: device BF16 rows of stride
 * ldx (>= d0, multiple of 8); z: device FP32 [n][dL]. */
uf_status uf_mlp_forward(uf_mlp* mlp, const void* x_bf16, int64_t ldx, const int32_t* rows,
                         int64_t n, float* z, void* hip_stream);
/* Gradients of every parameter (and of S) for the n rows of the preceding
 * uf_mlp_forward, given dz = dLoss/dz as device BF16 [n][dL]: x, ldx and rows
 * must be the ones that forward pass was given (its hidden activations are
 * held in the MLP until the next forward).  Weight gradients are dz^T h and
 * (g W) masked by the ReLU of each hidden layer, bias gradients column sums
 * (FP64, fixed order).  Left in the MLP for uf_mlp_adam / uf_mlp_get. */
uf_status uf_mlp_backward(uf_mlp* mlp, const void* x_bf16, int64_t ldx, const int32_t* rows,
                          int64_t n, const void* dz_bf16, void* hip_stream);
/* Loss mean_p (w_p (||z_a - z_b||_2 - target_p))^2 over n_pairs pairs
 * (device index arrays into x), written to loss (device, 1 float); w_p = 1,
 * or 1 / max(target_p, rel_floor) when rel_floor > 0 (relative error, which
 * weights the near pairs a nearest-neighbour search depends on).  The
 * gradients of every weight and bias are left in the MLP for uf_mlp_adam /
 * uf_mlp_get. */
uf_status uf_mlp_loss_grad(uf_mlp* mlp, const void* x_bf16, int64_t ldx, const int32_t* pair_a,
                           const int32_t* pair_b, const float* target, int64_t n_pairs,
                           float rel_floor, float* loss, void* hip_stream);
/* Ranking loss over n_triples triples (anchor a, near p, far n; device index
 * arrays into x) with exact distances d_near = d(a, p), d_far = d(a, n)
 * (device FP32).  With e_p = ||z_a - z_p||, e_n = ||z_a - z_n||:
 *   loss = mean_t [ dist_weight * ((e_p - d_p)^2 + (e_n - d_n)^2)
 *                   + rank_weight * tau * softplus((e_p - e_n) / tau) ]
 * -- both pairs' distance regression plus a smooth hinge (tau -> 0 gives
 * rank_weight * max(e_p - e_n, 0)) that asks the encoder to keep the order of
 * exact distances, which is what a nearest-neighbour search of the encoded
 * reference set needs.  3 * n_triples <= max_rows.  The gradients are left in
 * the MLP as for uf_mlp_loss_grad; loss (device, 1 float) receives the mean.
 * Errors: UF_ERR_ARG (NULL, sizes, a negative weight, tau <= 0), UF_ERR_DEVICE. */
uf_status uf_mlp_triplet_loss_grad(uf_mlp* mlp, const void* x_bf16, int64_t ldx,
                                   const int32_t* anchor, const int32_t* near, const int32_t* far,
                                   const float* d_near, const float* d_far, int64_t n_triples,
                                   float dist_weight, float rank_weight, float tau, float* loss,
                                   void* hip_stream);
/* One Adam step (bias-corrected, step >= 1) on every parameter, with
 * decoupled weight decay on the weight matrices (weight_decay = 0: plain
 * Adam). */
uf_status uf_mlp_adam(uf_mlp* mlp, float lr, float beta1, float beta2, float eps,
                      float weight_decay, int64_t step, void* hip_stream);
/* Plain Adam: uf_mlp_adam with weight_decay = 0. */
uf_status uf_adam_step(uf_mlp* mlp, float lr, float beta1, float beta2, float eps, int64_t step,
                       void* hip_stream);
void uf_free_mlp(uf_mlp* mlp);

/* out[i][j] = ||a_i - b_j||^2 (FP32, device [na][dim], [nb][dim] -> [na][nb]). */
uf_status uf_sqdist(const float* a, int64_t na, const float* b, int64_t nb, int64_t dim,
                    float* out, void* hip_stream);
/* The k smallest entries of each row of a non-negative FP32 matrix, sorted,
 * ties to the smaller column (exact radix select); 1 <= k <= 128 <= ... cols.
 * idx: device [rows][k]; vals (nullable): device [rows][k]. */
uf_status uf_topk_rows(const float* values, int64_t rows, int64_t cols, int64_t k, int32_t* idx,
                       float* vals, void* hip_stream);
/* Read a condensed matrix of n samples (dtype F64/F32): a dense FP32 block
 * out[r][c] = d(row_off + r, col_off + c) (+inf on the diagonal), or the
 * entries d(a_p, b_p) of a pair list (0 where a_p = b_p). */
uf_status uf_condensed_block(const void* cond, uf_out_dtype dtype, int64_t n, int64_t row_off,
                             int64_t n_rows, int64_t col_off, int64_t n_cols, float* out,
                             void* hip_stream);
uf_status uf_gather_pairs(const void* cond, uf_out_dtype dtype, int64_t n, const int32_t* a,
                          const int32_t* b, int64_t count, float* out, void* hip_stream);

/* Per-sample lists of the branches a sample touches, with l_v u_sv in FP64
 * (library-owned device memory).  Synchronises hip_stream. */
typedef struct uf_sparse uf_sparse;
uf_status uf_sparse_build(const uf_embedding* emb, void* hip_stream, uf_sparse** out);
int64_t uf_sparse_nnz(const uf_sparse* sparse);
void uf_free_sparse(uf_sparse* sparse);
/* Exact weighted-normalized distances across two tables on the same tree:
 * out[i][c] = d(queries[query_ids[i]], refs[cand[i][c]]) in FP64, for
 * i < n_queries, c < k (device arrays).  Uses sum|x-y| = s_x + s_y -
 * 2 sum min(x, y), the min being nonzero only where both samples touch a
 * branch.  ws: device workspace of uf_rerank_workspace_size bytes. */
uf_status uf_rerank_workspace_size(const uf_sparse* queries, int64_t n_queries, size_t* bytes);
uf_status uf_dm_rerank_weighted_normalized(const uf_sparse* queries, const uf_sparse* refs,
                                           const int32_t* query_ids, const int32_t* cand,
                                           int64_t n_queries, int64_t k, double* out, void* ws,
                                           size_t ws_bytes, void* hip_stream);

/* Exact weighted-normalized distances of arbitrary pairs across two tables on
 * the same tree: out[p] = d(a[pairs[p]], b[pairs[n_pairs + p]]) in FP64 for
 * p < n_pairs; pairs is a device int32 array [2][n_pairs].  Same arithmetic as
 * uf_dm_rerank_weighted_normalized (one candidate per query); ws of
 * uf_rerank_workspace_size(a, n_pairs) bytes. */
uf_status uf_dm_pairs_weighted_normalized(const uf_sparse* a, const uf_sparse* b,
                                          const int32_t* pairs, int64_t n_pairs, double* out,
                                          void* ws, size_t ws_bytes, void* hip_stream);

/* ---- principal coordinates (PCoA) ----------------------------------------- */

/* PCoA of a condensed distance matrix, the ordination the paper computes as
 * part of the UniFrac job (section II).  Definition (Gower): A = -d^2/2,
 * B = A - r 1^T - 1 r^T + g 11^T with r_i the row means of A (zero diagonal
 * included) and g their mean; the principal coordinates are the top eigen-
 * vectors v_k of B scaled by sqrt(max(lambda_k, 0)), lambda decreasing.  They are
 * found by randomized subspace iteration with a Rayleigh-Ritz projection
 * (Halko, Martinsson, Tropp 2011): Y = B Omega, power_iters passes of
 * Q = orth(B Q), then the eigenpairs of Q^T B Q.  B is never formed; each
 * product reads the condensed matrix once.
 *
 * dm:         device, condensed FP64 (length n(n-1)/2, SciPy order), read only.
 * row_means, grand_mean: device FP64 [n] and [1] as returned by uf_dm_*, or both
 *             NULL to have them computed here.
 * dims:       coordinates wanted; n_cols: columns of the test matrix
 *             (dims <= n_cols <= 48; oversampling n_cols - dims >= 5 advised).
 * power_iters: 0..64 (each adds one pass over dm; 2-4 typical).
 * omega:      device FP64 [n][n_cols], row major: the caller's random test matrix
 *             (i.i.d. standard normal), read only.
 * coords:     device FP64 [n][dims], row major, written; each column's largest-
 *             magnitude entry (first on ties) is positive.
 * eigvals:    host FP64 [dims], written (Ritz values, decreasing; 0 past the
 *             numerical rank of B).
 * trace:      host FP64 [1] or NULL: trace(B) = -n g, the sum of all eigenvalues
 *             (for proportions explained).
 * ws:         device workspace of uf_pcoa_workspace_size(n, n_cols) bytes.
 * stream:     hipStream_t; the call returns after the stream has drained.
 * Errors: UF_ERR_ARG (NULL pointers, sizes), UF_ERR_WORKSPACE, UF_ERR_DEVICE. */
uf_status uf_pcoa_workspace_size(int64_t n, int64_t n_cols, size_t* bytes);
uf_status uf_pcoa(const double* dm, int64_t n, const double* row_means, const double* grand_mean,
                  int64_t dims, int64_t n_cols, int power_iters, const double* omega,
                  double* coords, double* eigvals, double* trace, void* ws, size_t ws_bytes,
                  void* stream);

/* Principal directions of a data matrix, used to start the placement encoder's
 * linear path at the best linear map of its output width (the covariance's top
 * eigenvectors give the rank-k projection that keeps the most of the rows'
 * pairwise Euclidean distances).  The same randomized subspace iteration as
 * uf_pcoa, on C = Xc^T Xc / n with Xc = X minus its column means; C is never
 * formed (C Q = Xc^T (Xc Q), two passes over X in FP64 arithmetic).
 *
 * x_bf16:     device BF16 [n][ldx], the first d columns used (e.g. the
 *             projected reference set of uf_project).
 * k, n_cols:  directions wanted and columns of the test matrix
 *             (1 <= k <= n_cols <= min(160, d)).
 * power_iters: 0..64 passes of Q = orth(C Q).
 * omega:      device FP64 [d][n_cols] row major: the caller's i.i.d. standard
 *             normal test matrix.
 * basis:      device FP32 [k][d], written: orthonormal rows, by decreasing
 *             eigenvalue (signs arbitrary; zero rows past the rank of Xc).
 * eigvals:    host FP64 [k] or NULL: the Ritz values (variances along the rows).
 * ws:         device workspace of uf_pca_workspace_size(n, d, n_cols) bytes.
 * The call returns after the stream has drained.
 * Errors: UF_ERR_ARG (NULL pointers, sizes), UF_ERR_WORKSPACE, UF_ERR_DEVICE. */
uf_status uf_pca_workspace_size(int64_t n, int64_t d, int64_t n_cols, size_t* bytes);
uf_status uf_pca_basis(const void* x_bf16, int64_t n, int64_t d, int64_t ldx, int64_t k,
                       int64_t n_cols, int power_iters, const double* omega, float* basis,
                       double* eigvals, void* ws, size_t ws_bytes, void* hip_stream);

/* ---- Mantel test -------------------------------------------------------------- */

/* Correlation between two distance matrices with a permutation p-value (the
 * paper's section III).  Statistic: Pearson's r between the condensed vectors x
 * and y, or Spearman's (Pearson's on their ranks, ties sharing the average
 * rank).  Permutation b relabels the samples of the first matrix, rows and
 * columns together: x'_ij = x_{perm_b(i) perm_b(j)}.  p = (number of permuted
 * statistics at least as extreme as r, + 1) / (n_perm + 1); "as extreme" is
 * |r_b| >= |r| (UF_TWO_SIDED), r_b >= r (UF_GREATER) or r_b <= r (UF_LESS).
 *
 * x, y:       device, condensed FP64, length n(n-1)/2 each, read only.
 * perms:      device int32 [n_perm][n], each row a permutation of 0..n-1 drawn by
 *             the caller (entries outside [0, n) are rejected with UF_ERR_ARG).
 * stat, p_value: host, written.  perm_stats: host [n_perm] or NULL.
 * ws:         device workspace of uf_mantel_workspace_size(n, method, n_perm)
 *             bytes (holds x as a full n x n FP64 matrix).
 * If either matrix is constant, r is undefined: stat = 0, p = 1.
 * Errors: UF_ERR_ARG, UF_ERR_UNSUPPORTED (Spearman above 65,535 samples),
 * UF_ERR_WORKSPACE, UF_ERR_DEVICE. */
typedef enum { UF_MANTEL_PEARSON = 0, UF_MANTEL_SPEARMAN = 1 } uf_mantel_method;
typedef enum { UF_TWO_SIDED = 0, UF_GREATER = 1, UF_LESS = 2 } uf_alternative;
uf_status uf_mantel_workspace_size(int64_t n, int method, int64_t n_perm, size_t* bytes);
uf_status uf_mantel(const double* x, const double* y, int64_t n, int method, const int32_t* perms,
                    int64_t n_perm, int alternative, double* stat, double* p_value,
                    double* perm_stats, void* ws, size_t ws_bytes, void* stream);

/* ---- kernel timing --------------------------------------------------------- */

/* Per-kernel timing with HIP events recorded on the call's stream around each
 * launch (process-wide; off by default).  Names: "embed_nm", "embed_pres",
 * "band_wn_f64", "band_wn_f32", "band_wn_u32", "band_uw_f64", "band_uw_f32",
 * "gram_mfma", "rare_slots_wn", "rare_slots_uw", "finalize", "row_sums", and
 * the embedding preparation: "sample_scalars", "branch_count", "split_fill",
 * "sort_lists", "split_lengths".  uf_profile_read synchronises the recorded
 * events and returns the total milliseconds and launch count of one kernel
 * name since the last reset.  Errors: UF_ERR_ARG (NULL), UF_ERR_DEVICE. */
void uf_profile_enable(int on);
void uf_profile_reset(void);
uf_status uf_profile_read(const char* kernel, double* total_ms, int64_t* launches);

/* ---- helpers --------------------------------------------------------------- */
int64_t uf_n_stripes(int64_t n);                          /* floor(n/2)                 */
int64_t uf_condensed_index(int64_t n, int64_t i, int64_t j); /* i != j, -1 if invalid  */

void uf_free_tree(uf_tree* tree);
void uf_free_table(uf_table* table);
void uf_free_embedding(uf_embedding* emb);

const char* uf_status_string(uf_status status);
const char* uf_last_error_message(void);   /* thread-local; never NULL */

#ifdef __cplusplus
}
#endif

#endif /* UF_H */
