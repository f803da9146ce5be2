// Sparse-aware weighted-normalized numerator (gfx950).
//
//   sum_v |x_iv - x_jv| = sum_{v in D} |x_iv - x_jv|
//                         + sigma_i + sigma_j - 2 sum_{v not in D} min(x_iv, x_jv),
//   sigma_s = sum_{v not in D} x_sv,  x = l * u.
//
// D ("dense") holds the branches that more than a set fraction of the samples
// touch; they go through the stripe-band kernel (uf_kernels.hip) unchanged.  On
// every other branch min(x_i, x_j) is nonzero only for the pairs that both touch
// it, so those pairs are enumerated from per-branch sample lists and summed by
// integer atomics in fixed point (2^-40): exact and independent of the order in
// which the atomics land, so results are bitwise reproducible.
//
// Unweighted, the same lists serve the Gram form: with presence a in {0, 1},
// min(l a_i, l a_j) = l a_i a_j, so the non-dense part of G_ij is the sum of l
// over the branches both samples touch; the dense part is the MFMA Gram.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "uf_device.h"
#include "uf_internal.h"
#include "uf_split.h"

namespace ufs {
namespace {

constexpr double kFix = 1099511627776.0;   // 2^40

__global__ __launch_bounds__(256) void k_branch_count(ufp::Emb e, int32_t* __restrict__ cnt) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256)
        ufd::for_each_branch(e, ent, a, [&](int32_t v) { atomicAdd(&cnt[v], 1); });
}

__global__ __launch_bounds__(256) void k_split_fill(ufp::Emb e, const int32_t* __restrict__ cls,
                                                    const int64_t* __restrict__ roff,
                                                    int32_t* __restrict__ rfill,
                                                    int32_t* __restrict__ rs,
                                                    int64_t* __restrict__ rq,
                                                    unsigned long long* __restrict__ sigma) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    const double inv_t = 1.0 / e.total[s];
    unsigned long long part = 0;
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256)
        ufd::for_each_branch(e, ent, a, [&](int32_t v) {
            const int32_t c = cls[v];
            if (c == kClassDense) return;
            const int64_t cn = ufd::count_in(e, s, e.lo[v], e.hi[v]);
            const long long q = llrint(e.len[v] * (double(cn) * inv_t) * kFix);
            part += (unsigned long long)q;
            if (c >= 0) {
                const int32_t slot = atomicAdd(&rfill[c], 1);
                rs[roff[c] + slot] = int32_t(s);
                rq[roff[c] + slot] = q;
            }
        });
    atomicAdd(&sigma[s], part);
}

// node-major FP32 chunk over a list of branch positions (the dense set)
__global__ __launch_bounds__(256) void k_embed_list_f32(ufp::Emb e, const int32_t* __restrict__ list,
                                                        int64_t k0, int64_t kc,
                                                        float* __restrict__ out) {
    constexpr int TK = 256, TS = 64;
    __shared__ float tile[TK][TS + 1];
    const int tid = threadIdx.x;
    const int64_t kb = int64_t(blockIdx.x) * TK;
    const int64_t sb = int64_t(blockIdx.y) * TS;
    const int64_t k = kb + tid;
    const bool kin = k < kc;
    int32_t lk = 0, hk = 0;
    double lv = 0.0;
    if (kin) {
        const int32_t pos = list[k0 + k];
        lk = e.lo[pos];
        hk = e.hi[pos];
        lv = e.len[pos];
    }
    for (int j = 0; j < TS; ++j) {
        const int64_t s = sb + j;
        float v = 0.0f;
        if (kin && s < e.n) v = float(lv * (double(ufd::count_in(e, s, lk, hk)) / e.total[s]));
        tile[tid][j] = v;
    }
    __syncthreads();
    for (int r = tid / TS; r < TK; r += 256 / TS) {
        const int64_t kk = kb + r;
        const int64_t s = sb + (tid % TS);
        if (kk < kc && s < e.n) out[kk * e.n + s] = tile[r][tid % TS];
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Pairs of one shared branch's sample list: pair index p in [0, m(m-1)/2)
// maps to (a, b), a < b, row-major over the upper triangle.
__device__ __forceinline__ void pair_of(int64_t p, int64_t m, int64_t& a, int64_t& b) {
    const double t = double(2 * m - 1);
    int64_t r = int64_t((t - sqrt(t * t - 8.0 * double(p))) * 0.5);
    // fix rounding: first index of row r is r*m - r(r+1)/2
    while (r > 0 && r * m - r * (r + 1) / 2 > p) --r;
    while ((r + 1) * m - (r + 1) * (r + 2) / 2 <= p) ++r;
    a = r;
    b = p - (r * m - r * (r + 1) / 2) + r + 1;
}

__device__ __forceinline__ uint32_t bf16_to_bits32(uint16_t h) { return uint32_t(h) << 16; }

__global__ __launch_bounds__(256) void k_split_lengths(const int32_t* __restrict__ cls, int64_t nb,
                                                       const int32_t* __restrict__ dense,
                                                       int64_t n_dense, int64_t n_pad,
                                                       const uint16_t* __restrict__ len_hi,
                                                       const uint16_t* __restrict__ len_lo,
                                                       uint16_t* __restrict__ dlen_hi,
                                                       uint16_t* __restrict__ dlen_lo,
                                                       int64_t* __restrict__ rl) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < n_pad) {
        const bool in = t < n_dense;
        dlen_hi[t] = in ? len_hi[dense[t]] : uint16_t(0);
        dlen_lo[t] = in ? len_lo[dense[t]] : uint16_t(0);
    }
    if (t < nb && cls[t] >= 0) {
        const double l = double(__uint_as_float(bf16_to_bits32(len_hi[t]))) +
                         double(__uint_as_float(bf16_to_bits32(len_lo[t])));
        rl[cls[t]] = llrint(l * kFix);
    }
}

template <bool W>
__global__ __launch_bounds__(256) void k_rare_pairs(const int64_t* __restrict__ roff,
                                                    const int32_t* __restrict__ rs,
                                                    const int64_t* __restrict__ rq,
                                                    const int64_t* __restrict__ rl,
                                                    const RareItem* __restrict__ items, int64_t n,
                                                    int64_t sb, int64_t se,
                                                    unsigned long long* __restrict__ M) {
    const RareItem it = items[blockIdx.x];
    const int64_t base = roff[it.list];
    const int64_t m = roff[it.list + 1] - base;
    const int64_t S = n / 2;
    const bool even = (n & 1) == 0;
    const unsigned long long lq = W ? 0ull : (unsigned long long)rl[it.list];
    for (int64_t p = it.p0 + threadIdx.x; p < it.p1; p += 256) {
        int64_t a, b;
        pair_of(p, m, a, b);
        int64_t i = rs[base + a], j = rs[base + b];
        if (i > j) {
            const int64_t t = i;
            i = j;
            j = t;
        }
        unsigned long long mn = lq;
        if (W) {
            const long long qa = rq[base + a], qb = rq[base + b];
            mn = (unsigned long long)(qa < qb ? qa : qb);
        }
        const int64_t d = j - i;
        int64_t s, slot;
        if (d <= S) {
            s = d - 1;
            slot = i;
        } else {
            s = n - d - 1;
            slot = j;
        }
        if (s < sb || s >= se) continue;
        atomicAdd(&M[(s - sb) * n + slot], mn);
        if (even && d == S) atomicAdd(&M[(s - sb) * n + j], mn);
    }
}

}  // namespace

hipError_t branch_count(const ufp::Emb& e, int32_t* cnt, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_branch_count, dim3(unsigned(e.n)), dim3(256), 0, st, e, cnt);
    return hipGetLastError();
}

hipError_t split_fill(const ufp::Emb& e, const int32_t* cls, const int64_t* roff, int32_t* rfill,
                      int32_t* rs, int64_t* rq, unsigned long long* sigma, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_fill, dim3(unsigned(e.n)), dim3(256), 0, st, e, cls, roff, rfill, rs,
                       rq, sigma);
    return hipGetLastError();
}

hipError_t embed_list_f32(const ufp::Emb& e, const int32_t* list, int64_t k0, int64_t kc, float* out,
                          hipStream_t st) {
    if (kc <= 0 || e.n <= 0) return hipSuccess;
    const int64_t gy = (e.n + 63) / 64;
    if (gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_embed_list_f32, dim3(unsigned((kc + 255) / 256), unsigned(gy)), dim3(256), 0,
                       st, e, list, k0, kc, out);
    return hipGetLastError();
}

hipError_t zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t split_lengths(const int32_t* cls, int64_t nb, const int32_t* dense, int64_t n_dense,
                         int64_t n_pad, const uint16_t* len_hi, const uint16_t* len_lo,
                         uint16_t* dlen_hi, uint16_t* dlen_lo, int64_t* rl, hipStream_t st) {
    const int64_t t = std::max(nb, n_pad);
    if (t <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_lengths, dim3(unsigned((t + 255) / 256)), dim3(256), 0, st, cls, nb,
                       dense, n_dense, n_pad, len_hi, len_lo, dlen_hi, dlen_lo, rl);
    return hipGetLastError();
}

hipError_t rare_pairs(const int64_t* roff, const int32_t* rs, const int64_t* rq, const int64_t* rl,
                      const RareItem* items, int64_t n_items, int64_t n, int64_t sb, int64_t se,
                      unsigned long long* M, hipStream_t st) {
    if (n_items <= 0 || se <= sb) return hipSuccess;
    if (n_items > 0x7fffffff) return hipErrorInvalidValue;
    if (rl)
        hipLaunchKernelGGL(k_rare_pairs<false>, dim3(unsigned(n_items)), dim3(256), 0, st, roff, rs,
                           rq, rl, items, n, sb, se, M);
    else
        hipLaunchKernelGGL(k_rare_pairs<true>, dim3(unsigned(n_items)), dim3(256), 0, st, roff, rs,
                           rq, rl, items, n, sb, se, M);
    return hipGetLastError();
}

}  // namespace ufs
