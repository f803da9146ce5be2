// Internal declarations shared by the host side (uf_host.hip) and the kernels
// (uf_kernels.hip) of the striped UniFrac library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "uf.h"

// ---------------------------------------------------------------------------
// Host handles
// ---------------------------------------------------------------------------

// A validated rooted tree, re-indexed in depth-first postorder.  "Position"
// k in [0, n_nodes) is the postorder rank; the root is the last position and
// positions [0, n_nodes-1) are the branches in the order they are streamed.
// Tips are ranked by position; node k covers the tip ranks [lo[k], hi[k]).
struct uf_tree {
    int64_t n_nodes = 0;
    int64_t n_tips = 0;
    std::vector<int64_t> node_at;     // node id at position k
    std::vector<int64_t> pos_of;      // position of node id
    std::vector<int32_t> parent_pos;  // parent position, -1 for the root
    std::vector<double> len;          // branch length at position (root: 0)
    std::vector<int32_t> lo, hi;      // tip-rank interval under position k
    std::vector<int32_t> tip_rank;    // by node id, -1 for internal nodes
    std::vector<int32_t> tip_pos;     // position of the tip with rank r
};

// A validated table: per sample, its nonzero entries sorted by tip rank.
struct uf_table {
    int64_t n_samples = 0;
    int64_t n_tips = 0;               // of the tree it was validated against
    std::vector<int64_t> row_ptr;     // [n_samples+1]
    std::vector<int32_t> rank;        // tip rank of each entry, ascending per row
    std::vector<int64_t> count;       // > 0
    std::vector<int64_t> total;       // per sample, > 0
};

// Sparse-aware split of one embedding at one threshold (uf_host.hip).
namespace ufs {
struct SlotEntry;
}

struct SplitCache {
    uint64_t build_id = 0;        // unique per build (graph keys)
    double threshold = 0.0;       // requested fraction, < 0 for the cost model
    int64_t n_dense = 0;          // branches in the dense set
    int64_t n_lists = 0;          // shared non-dense branches (>= 2 samples)
    int64_t n_entries = 0;        // entries of their sample lists
    int64_t n_pairs = 0;          // sample pairs over all lists
    void* arena = nullptr;
    int32_t* dense = nullptr;     // [n_dense] positions, ascending
    int32_t* cls = nullptr;       // [nb] class per position (list id, or ufs::kClass*)
    int64_t* roff = nullptr;      // [n_lists+1]
    int32_t* rs = nullptr;        // unweighted: [n_entries] sample of each entry, ascending per list
    unsigned long long* rw = nullptr;  // weighted: [n_entries] rint(l*u/unit) << 24 | sample
    double unit = 0x1p-40;        // weighted: value of one fixed-point step of rw, sigma and M
    unsigned long long* sigma = nullptr;   // [n] weighted: sum over non-dense branches, in unit
    int64_t n_dense_pad = 0;      // n_dense rounded up to the MFMA K step
    uint16_t* dlen_hi = nullptr;  // [n_dense_pad] bf16 high part of each dense length, 0-padded
    uint16_t* dlen_lo = nullptr;  // [n_dense_pad] bf16 low part
    int64_t* rl = nullptr;        // [n_lists] (hi+lo) length of each list's branch, 2^-40 fixed point
    int64_t* soff = nullptr;      // [n+1] per-sample rows of `entries`
    ufs::SlotEntry* entries = nullptr;   // [n_entries] the sample's list memberships
    double q_scale = 0.0;         // weighted: 32-bit fixed-point scale of the dense pass (0: FP32)
    int32_t* lo_ord = nullptr;    // weighted: [n_dense] indices into dense, by ascending lo
    SplitCache() = default;
    SplitCache(const SplitCache&) = delete;
    SplitCache& operator=(const SplitCache&) = delete;
    ~SplitCache() {
        if (arena) (void)hipFree(arena);   // hipFree waits for work in flight on the device
    }
};

// Device temporaries of a split build, kept per embedding and grown on demand so
// that rebuilding a split does not allocate again (guarded by split_mu).
struct SplitScratch {
    void* buf = nullptr;
    size_t bytes = 0;
    SplitScratch() = default;
    SplitScratch(const SplitScratch&) = delete;
    SplitScratch& operator=(const SplitScratch&) = delete;
    ~SplitScratch() {
        if (buf) (void)hipFree(buf);
    }
};

// Device-resident inputs of the distance calls.  All arrays are on `device`.
struct uf_embedding {
    int device = 0;
    int64_t n = 0;          // samples
    int64_t nb = 0;         // branches (non-root nodes) = positions [0, nb)
    int64_t nnz = 0;
    int64_t max_total = 0;  // largest sample total T_s (host copy)
    // table
    int64_t* row_ptr = nullptr;   // [n+1]
    int32_t* rank = nullptr;      // [nnz]
    int64_t* cum = nullptr;       // [nnz + n]: exclusive prefix of counts, per row
    double* total = nullptr;      // [n]  T_s as double (exact below 2^53)
    // tree, by position
    int32_t* lo = nullptr;        // [nb+1] (last entry: the root)
    int32_t* hi = nullptr;        // [nb+1]
    double* len = nullptr;        // [nb]
    float* len32 = nullptr;       // [nb] FP32-rounded lengths
    uint16_t* len_hi = nullptr;   // [nb] bf16 bits of RNE(len)
    uint16_t* len_lo = nullptr;   // [nb] bf16 bits of RNE(len - hi)
    // per-sample scalars (FP64)
    double* sw = nullptr;         // sum_v l_v u_sv
    double* wu = nullptr;         // sum_v l_v a_sv, FP64 lengths
    double* wu32 = nullptr;       // same with FP32-rounded lengths
    double* wub = nullptr;        // same with hi+lo bf16 lengths
    // sparse-aware split, built on first use (guarded by split_mu).  A call that
    // uses a split holds its own reference, so a rebuild by another thread (new
    // threshold) never frees a split that is still being enqueued.
    std::shared_ptr<SplitCache> split[2];   // [0] unweighted, [1] weighted
    SplitScratch split_tmp;
    std::mutex split_mu;
    int32_t* parent_pos = nullptr;  // [nb+1], -1 for the root
    int32_t* tip_pos = nullptr;     // [n_tips] position of the tip with rank r
    std::vector<int32_t> sub_first; // host, [nb]: first position of each position's subtree
    // root distances by position for the three length roundings (per-sample scalars)
    double* d64 = nullptr;
    double* d32 = nullptr;
    double* dbf = nullptr;
    void* arena = nullptr;        // one allocation holding all of the above
};

// Shared host helpers (uf_host.hip): record a thread-local error message and
// return the status; check that a gfx950 device is current.
namespace ufh {
uf_status fail(uf_status st, const std::string& msg);
uf_status hip_fail(hipError_t e, const char* what);
uf_status check_device(int* dev_out);
// Timing of the launches enqueued on s during the guard's lifetime, under a
// kernel name of uf_profile_read (events recorded only while profiling is on).
struct ProfHandle;
ProfHandle* prof_begin(const char* name, hipStream_t s);
void prof_end(ProfHandle* h);
class ProfGuard {
  public:
    ProfGuard(const char* name, hipStream_t s) : h_(prof_begin(name, s)) {}
    ~ProfGuard() { prof_end(h_); }
    ProfGuard(const ProfGuard&) = delete;
    ProfGuard& operator=(const ProfGuard&) = delete;

  private:
    ProfHandle* h_;
};
}  // namespace ufh

// One table of a batch, as the batched kernels see it.
struct BatchTable {
    int64_t n;        // samples
    int64_t off;      // first sample in the concatenated table
    int64_t e_off;    // element offset of its node-major chunk block [kc][n]
    int64_t acc_off;  // element offset of its stripe-major accumulator [n/2][n]
    int64_t n_iblk;   // 128-sample blocks
};

// ---------------------------------------------------------------------------
// Kernel launchers (uf_kernels.hip).  All are asynchronous on `st` and return
// the hipError_t of the launch.
// ---------------------------------------------------------------------------
namespace ufk {

constexpr int kBandI = 128;       // samples per band tile
constexpr int kBandS = 128;       // stripes per band tile
constexpr int kGramT = 256;       // square tile of the MFMA Gram kernel
constexpr int kGramK = 128;        // K step of the MFMA Gram kernel
constexpr int kGramKPad = 256;    // K of its presence matrix is padded to this (steps go in pairs)

// Per-sample scalars from the postorder leaf intervals (one wave per sample).
hipError_t sample_scalars(const uf_embedding& e, const int32_t* parent_pos,
                          const int32_t* tip_pos, const double* d64, const double* d32,
                          const double* dbf, hipStream_t st);

// Node-major chunk E[k][s] for positions [k0, k0+kc): weighted -> T(l * c/T_s),
// presence -> T(c > 0).
hipError_t embed_node_major_f64(const uf_embedding& e, int64_t k0, int64_t kc, int weighted,
                                double* out, hipStream_t st);
hipError_t embed_node_major_f32(const uf_embedding& e, int64_t k0, int64_t kc, int weighted,
                                float* out, hipStream_t st);
// Sample-major presence P[s][k]: FP8 e4m3 -2.0 (0xC0) where present, else 0, k < kpad (zero beyond
// kc), for positions [k0, k0+kc), or for positions list[k0 .. k0+kc) when list is
// non-null.  kpad is a multiple of kGramKPad.
hipError_t embed_presence_fp8(const uf_embedding& e, int64_t k0, int64_t kc, int64_t kpad,
                              uint8_t* out, hipStream_t st, const int32_t* list = nullptr);

// Band accumulation over one node chunk for stripes [sb, se):
// weighted: acc += sum_k |E[k][i] - E[k][j]|;  unweighted: acc += sum_k l_k E[k][i] E[k][j].
hipError_t band_f64(const double* E, const double* lenk, int64_t kc, int64_t n, int64_t sb,
                    int64_t se, int weighted, int first, double* acc, hipStream_t st);
hipError_t band_f32(const float* E, const float* lenk, int64_t kc, int64_t n, int64_t sb,
                    int64_t se, int weighted, int first, float* acc, hipStream_t st);
// Weighted only, 32-bit fixed point: acc += sum_k |E[k][i] - E[k][j]| (exact integers;
// the caller keeps the sum below 2^32).
hipError_t band_u32(const uint32_t* E, int64_t kc, int64_t n, int64_t sb, int64_t se, int first,
                    uint32_t* acc, hipStream_t st);

// MFMA Gram over one chunk: for every upper-triangle 256x256 tile (bi <= bj) that holds
// a pair of stripes [sb, se), G_ij (+)= sum_k [P_ik != 0][P_jk != 0] (hi_k + lo_k), scattered
// into the FP32 stripe-major accumulator (first: overwrite, else add).  P: presence bytes as
// above; hi and lo hold kpad values from the chunk's first position (zero past its end).
hipError_t gram_mfma(const uint8_t* P, const uint16_t* hi, const uint16_t* lo, int64_t kpad,
                     int64_t n, int64_t sb, int64_t se, int first, float* acc, hipStream_t st);

// Distances from the accumulators.  kind 0: weighted (num / (s_i + s_j));
// kind 1: unweighted Gram form ((w_i + w_j - 2G) / (w_i + w_j - G)), clamped to [0, 1].
// acc_type (kAcc*) selects the accumulator type; its values are multiplied by
// acc_scale.  q (nullable) receives -d^2/2 in FP64, stripe-major.  layout/out dtype
// as in uf.h.  split_m (nullable, fixed point with step split_unit, sample-major:
// M[i*(se-sb) + s-sb]) carries the non-dense branches: kind 0 adds sigma_i + sigma_j -
// 2 M to the numerator, kind 1 adds M to the Gram value.
constexpr int kAccF32 = 0, kAccF64 = 1, kAccU32 = 2;
hipError_t finalize(int kind, const void* acc, int acc_type, double acc_scale, const double* scal,
                    int64_t n, int64_t sb, int64_t se, int layout, int out_f32, void* out, double* q,
                    hipStream_t st, const unsigned long long* split_m = nullptr,
                    const unsigned long long* sigma = nullptr, double split_unit = 0x1p-40);

// Row sums of -d^2/2 over the distinct pairs of stripes [sb, se): two fixed-order stages.
hipError_t row_sums(const double* q, int64_t n, int64_t sb, int64_t se, double* partial,
                    int64_t n_parts, double scale, double* out, hipStream_t st);
hipError_t grand_mean(const double* row_means, int64_t n, double* out, hipStream_t st);

// ---- batches (many tables on one tree, weighted normalized, FP32) --------
// Node-major chunk of every table: table r's block at e_off, row stride n_r.
hipError_t embed_batch_f32(const uf_embedding& e, const BatchTable* tabs, const int32_t* tab_of,
                           int64_t k0, int64_t kc, float* out, hipStream_t st);
// Persistent band kernel over (table, tile) items.  items: int32 pairs; queue q
// holds items [qbeg[q], qend[q]) and its counter counters[q] (8 queues, one per
// XCD; exhausted queues are stolen from).  stage_branches in {8, 16, 32};
// tile_stripes in {64, 128, 256}: a tile is kBandI samples x tile_stripes
// stripes, and item (r, t) is tile t of table r with its i-block fastest.
hipError_t band_persistent_f32(const float* E, const BatchTable* tabs, const int2* items,
                               const int64_t* qbeg, const int64_t* qend, unsigned* counters,
                               int64_t kc, int first, float* acc, int stage_branches,
                               int tile_stripes, int n_blocks, hipStream_t st);
// Resident blocks per CU of that kernel (0 for an unknown configuration).
int band_persistent_max_blocks(int stage_branches, int tile_stripes);
// Zero n unsigned counters (a kernel, so that graph replays stay valid).
hipError_t zero_u32(unsigned* p, int64_t n, hipStream_t st);

}  // namespace ufk
