// Internal declarations of the sparse-aware split (uf_split.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_place.h"

namespace ufs {

constexpr int32_t kClassDense = -1;    // branch in the dense set
constexpr int32_t kClassAlone = -2;    // touched by at most one sample: no pairs

// A range of pair indices of one shared branch's sample list.
struct RareItem {
    int64_t list;
    int64_t p0, p1;
};

hipError_t branch_count(const ufp::Emb& e, int32_t* cnt, hipStream_t st);
hipError_t split_fill(const ufp::Emb& e, const int32_t* cls, const int64_t* roff, int32_t* rfill,
                      int32_t* rs, int64_t* rq, unsigned long long* sigma, hipStream_t st);
hipError_t embed_list_f32(const ufp::Emb& e, const int32_t* list, int64_t k0, int64_t kc, float* out,
                          hipStream_t st);
hipError_t zero_u64(unsigned long long* p, int64_t n, hipStream_t st);
// Per-list (hi+lo) branch length in fixed point, and the bf16 length parts of the
// dense set gathered in order (zero beyond n_dense up to n_pad).
hipError_t split_lengths(const int32_t* cls, int64_t nb, const int32_t* dense, int64_t n_dense,
                         int64_t n_pad, const uint16_t* len_hi, const uint16_t* len_lo,
                         uint16_t* dlen_hi, uint16_t* dlen_lo, int64_t* rl, hipStream_t st);
// M[(s-sb)*n + slot] += contribution of every pair sharing a non-dense branch, for
// stripes [sb, se).  rl == nullptr: weighted, min(rq_a, rq_b); else unweighted, rl[list].
hipError_t rare_pairs(const int64_t* roff, const int32_t* rs, const int64_t* rq, const int64_t* rl,
                      const RareItem* items, int64_t n_items, int64_t n, int64_t sb, int64_t se,
                      unsigned long long* M, hipStream_t st);

}  // namespace ufs
