// Device helpers shared by several kernel files: the embedded count of a
// sample on a branch, and the enumeration of the branches a sample touches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_place.h"

namespace ufd {

// first index in [a, b) whose tip rank is >= key
__device__ __forceinline__ int64_t lower_bound_rank(const int32_t* __restrict__ rank, int64_t a,
                                                    int64_t b, int32_t key) {
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (rank[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a;
}

// sum of sample s's counts on the tips with rank in [lo, hi) (exact, integer)
__device__ __forceinline__ int64_t count_in(const ufp::Emb& e, int64_t s, int32_t lo, int32_t hi) {
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    const int64_t p1 = lower_bound_rank(e.rank, a, b, lo);
    const int64_t p2 = lower_bound_rank(e.rank, p1, b, hi);
    return e.cum[p2 + s] - e.cum[p1 + s];
}

// The branches a sample touches, each exactly once: walking up from the tip
// of entry `entry`, branch v is reported when the previous tip of the row
// lies outside v's subtree (lo_v > rank[entry-1]); the walk stops at the first
// ancestor that also covers the previous tip.  The root is never reported.
template <typename F>
__device__ __forceinline__ void for_each_branch(const ufp::Emb& e, int64_t entry, int64_t row_start,
                                                F&& f) {
    const int32_t r = e.rank[entry];
    const int32_t prev = entry > row_start ? e.rank[entry - 1] : -1;
    int32_t v = e.tip_pos[r];
    while (v < e.root_pos && e.lo[v] > prev) {
        f(v);
        v = e.parent_pos[v];
    }
}

}  // namespace ufd
