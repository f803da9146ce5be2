// Internal declarations of the sparse-aware split (uf_split.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_place.h"

struct BatchTable;

namespace ufs {

constexpr int32_t kClassDense = -1;    // branch in the dense set
constexpr int32_t kClassAlone = -2;    // touched by at most one sample: no pairs
constexpr int kSampleBits = 24;         // packed weighted list member: value << 24 | sample

constexpr int kBaseBits = 40;           // SlotEntry::bw: list start in the low 40 bits

// Stripes per slot workgroup: its LDS row takes 8 bytes per stripe, up to the
// 160 KiB of a gfx950 CU.
constexpr int64_t kSegStripes = 20480;
// Stripes per segment when the slot kernel covers stripes [sb, se).
inline int64_t slot_segment_len(int64_t sb, int64_t se) {
    const int64_t nseg = (se - sb + kSegStripes - 1) / kSegStripes;
    return nseg > 0 ? (se - sb + nseg - 1) / nseg : 0;
}

// One list membership of a sample, as the slot kernel reads it:
// * bw: the list's first entry (low kBaseBits bits) and the window length w (high
//   24 bits): the members at cyclic distance 1..floor(N/2) after the sample, which
//   follow it in the sorted list;
// * mpw: the list length m (bits 0-23), the sample's position p in it (24-47), and
//   w0 (48-63), the members of the window at distance <= slot_segment_len(0,
//   floor(N/2)) (the first segment boundary of a full-range call);
// * v: its value (weighted: the sample's own l*u in the split's fixed-point step;
//   unweighted: the branch length l_hi + l_lo in 2^-40).
struct SlotEntry {
    int64_t bw;
    unsigned long long mpw;
    unsigned long long v;
};

// Per position, +1 for every sample with that tip and -1 for every sample whose
// consecutive tips meet there: the sum over a subtree is the number of samples
// touching the branch above it.
hipError_t branch_points(const ufp::Emb& e, int32_t* pt, hipStream_t st);
// Unsorted list members and per-sample list counts (scnt); weighted, also each
// member's fixed-point l*u (rq), sigma and per-sample counts of dense branches of
// nonzero length (dnnz), which the unweighted split leaves untouched.  nodes:
// device scratch of max(nb, 1) records (filled here: the walk's node fields).
hipError_t split_fill(const ufp::Emb& e, bool weighted, const int32_t* cls, int4* nodes,
                      const int64_t* roff, int32_t* rfill, int32_t* rs, int64_t* rq,
                      unsigned long long* sigma, int32_t* scnt, int32_t* dnnz, double fix,
                      hipStream_t st);
// Lists of at most kSortSmall members are ranked by one wave each; longer ones by
// one workgroup each.
constexpr int kSortSmall = 64;
// Lists sorted by sample, into rs_out (sample ids) or, when rw_out is non-null, into
// rw_out as packed words rq << kSampleBits | sample; per-sample index rows
// [soff[s], soff[s+1]) of SlotEntry filled through the cursors scur (zeroed by the
// caller); v holds the sample's value (weighted) or the list id (unweighted).
// small_ids / large_ids: the list ids of at most / more than kSortSmall members.
hipError_t sort_lists(const int64_t* roff, const int32_t* small_ids, int64_t n_small,
                      const int32_t* large_ids, int64_t n_large, int64_t n, int64_t seg0,
                      const int32_t* rs_in, const int64_t* rq_in, int32_t* rs_out,
                      unsigned long long* rw_out, const int64_t* soff, int32_t* scur,
                      SlotEntry* se, hipStream_t st);
// Unweighted: replace each entry's list id (left in v by sort_lists) by rl[list].
hipError_t entry_lengths(SlotEntry* se, int64_t n_entries, const int64_t* rl, hipStream_t st);
// Node-major chunk E[k][s] over positions list[k0 .. k0+kc): x = l * c / T as FP32,
// or as rint(x * q) in 32-bit fixed point.  merge (every T_s < 2^32) with lo_ord
// (the n_list entries of list ordered by lo): two forward-merge passes; else one
// binary search per element.  Same values either way.
hipError_t embed_list_f32(const ufp::Emb& e, const int32_t* list, const int32_t* lo_ord,
                          int64_t n_list, bool merge, int64_t k0, int64_t kc, float* out,
                          hipStream_t st);
hipError_t embed_list_u32(const ufp::Emb& e, const int32_t* list, const int32_t* lo_ord,
                          int64_t n_list, bool merge, int64_t k0, int64_t kc, double q,
                          uint32_t* out, hipStream_t st);
// The same two merge passes for a batch: every position of [k0, k0+kc) (FP32),
// each sample's values into its table's block [kc][n_t] at e_off.  lo_ord_chunk:
// the chunk's kc positions ordered by lo.  Every T_s must be below 2^32.
hipError_t embed_batch_merge_f32(const ufp::Emb& e, const BatchTable* tabs, const int32_t* tab_of,
                                 const int32_t* lo_ord_chunk, int64_t k0, int64_t kc, float* out,
                                 hipStream_t st);
// Per-list (hi+lo) branch length in fixed point, and the bf16 length parts of the
// dense set gathered in order (zero beyond n_dense up to n_pad).
hipError_t split_lengths(const int32_t* cls, int64_t nb, const int32_t* dense, int64_t n_dense,
                         int64_t n_pad, const uint16_t* len_hi, const uint16_t* len_lo,
                         uint16_t* dlen_hi, uint16_t* dlen_lo, int64_t* rl, hipStream_t st);
// M[i*(se-sb) + (s-sb)] (sample-major) = sum over the pairs (i, (i+s+1) mod n), s in
// [sb, se), that share a non-dense branch: rw non-null: weighted, min of the two values;
// else unweighted (sample ids rs), the branch length.  Writes every element of the range.
hipError_t rare_slots(const int32_t* rs, const unsigned long long* rw, const int64_t* soff,
                      const SlotEntry* entries, int64_t n, int64_t sb, int64_t se,
                      unsigned long long* M, hipStream_t st);

}  // namespace ufs
