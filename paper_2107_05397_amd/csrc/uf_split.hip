// Sparse-aware split of the UniFrac numerators (gfx950).
//
//   sum_v |x_iv - x_jv| = sum_{v in D} |x_iv - x_jv|
//                         + sigma_i + sigma_j - 2 sum_{v not in D} min(x_iv, x_jv),
//   sigma_s = sum_{v not in D} x_sv,  x = l * u.
//
// D ("dense") holds the branches that many samples touch; they go through the
// stripe-band kernel or the MFMA Gram (uf_kernels.hip) unchanged.  On every
// other branch min(x_i, x_j) is nonzero only for the pairs that both touch it.
// Those branches keep a list of the samples touching them, sorted by sample,
// and every sample keeps the lists it is in.  The slot kernel gives one
// workgroup to one sample i and a range of stripes: for each list of i it walks
// the members j that follow i cyclically at distance d = (j - i) mod N inside
// the stripe window (stripe d - 1), and adds min(x_i, x_j) into an LDS row
// indexed by stripe.  Sums are in 2^-40 fixed point: exact, so the order of the
// additions does not matter and the result is bitwise reproducible.  Each
// accumulator element of the range is written once, by its sample's workgroup.
//
// Unweighted, the same lists serve the Gram form: with presence a in {0, 1},
// min(l a_i, l a_j) = l a_i a_j, so the non-dense part of G_ij is the sum of l
// over the branches both samples touch; the dense part is the MFMA Gram.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "uf_device.h"
#include "uf_internal.h"
#include "uf_split.h"

namespace ufs {
namespace {

constexpr double kFix = 1099511627776.0;   // 2^40

// Points whose subtree sums count the samples touching each branch: per sample,
// +1 at each of its tips and -1 at the lowest common ancestor of each tip and
// the sample's previous tip (in rank order).  The tips of a sample below a node
// are consecutive in rank order, so a subtree holding k >= 1 of them holds the
// k - 1 ancestors of their consecutive pairs and sums to 1.  The walk up from a
// tip stops at exactly that ancestor (the first node whose leaf interval also
// covers the previous tip); the root is never counted.
__global__ __launch_bounds__(256) void k_branch_points(ufp::Emb e, int32_t* __restrict__ pt) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256) {
        const int32_t r = e.rank[ent];
        const int32_t prev = ent > a ? e.rank[ent - 1] : -1;
        const int32_t tip = e.tip_pos[r];
        int32_t v = tip;
        while (v < e.root_pos && e.lo[v] > prev) v = e.parent_pos[v];
        if (tip < e.root_pos) atomicAdd(&pt[tip], 1);
        if (v < e.root_pos) atomicAdd(&pt[v], -1);
    }
}

// The fields the list fill reads at every node of its walks, packed in one
// 16-byte record per position (leaf interval, parent, class) so that a step of a
// walk touches one cache line.
__global__ __launch_bounds__(256) void k_pack_nodes(ufp::Emb e, const int32_t* __restrict__ cls,
                                                    int64_t nb, int4* __restrict__ nodes) {
    const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (v < nb) nodes[v] = make_int4(e.lo[v], e.hi[v], e.parent_pos[v], cls[v]);
}

// Unsorted list fill: members of each shared non-dense branch's list and the
// number of lists of each sample; weighted (W) also each member's fixed-point
// l*u, sigma per sample and the number of dense branches of nonzero length it
// touches (the unweighted lists need the samples alone).  The walk is the one of
// ufd::for_each_branch over the packed node records.
template <bool W>
__global__ __launch_bounds__(256) void k_split_fill(ufp::Emb e, const int4* __restrict__ nodes,
                                                    const int64_t* __restrict__ roff,
                                                    int32_t* __restrict__ rfill,
                                                    int32_t* __restrict__ rs,
                                                    int64_t* __restrict__ rq,
                                                    unsigned long long* __restrict__ sigma,
                                                    int32_t* __restrict__ scnt,
                                                    int32_t* __restrict__ dnnz, double fix) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    const double inv_t = 1.0 / e.total[s];
    unsigned long long part = 0;
    int32_t lists = 0, dense = 0;
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256) {
        const int32_t prev = ent > a ? e.rank[ent - 1] : -1;
        // the sample's entries under a branch v of this walk are [ent, p2): none
        // before ent lies under v (v does not cover the previous tip), and p2, the
        // first entry at rank >= hi_v, only moves forward as the walk climbs
        int64_t p2 = ent + 1;
        int32_t v = e.tip_pos[e.rank[ent]];
        while (v < e.root_pos) {
            const int4 nd = nodes[v];   // lo, hi, parent, class
            if (nd.x <= prev) break;
            const int32_t c = nd.w;
            if (c == kClassDense) {
                if constexpr (W) dense += e.len[v] > 0.0;
            } else {
                long long q = 0;
                if constexpr (W) {
                    p2 = ufd::lower_bound_rank(e.rank, p2, b, nd.y);
                    const int64_t cn = e.cum[p2 + s] - e.cum[ent + s];
                    q = llrint(e.len[v] * (double(cn) * inv_t) * fix);
                    part += (unsigned long long)q;
                }
                if (c >= 0) {
                    const int32_t slot = atomicAdd(&rfill[c], 1);
                    rs[roff[c] + slot] = int32_t(s);
                    if constexpr (W) rq[roff[c] + slot] = q;
                    ++lists;
                }
            }
            v = nd.z;
        }
    }
    if constexpr (W) {
        atomicAdd(&sigma[s], part);
        if (dense) atomicAdd(&dnnz[s], dense);
    }
    if (lists) atomicAdd(&scnt[s], lists);
}

// Sort each list by sample: a member's new position is the number of members
// with a smaller sample id (ids in a list are distinct).  Also records, in the
// sample's row of the per-sample index, the list, the member's position and the
// sizes of its window.

__device__ __forceinline__ void place_member(int64_t L, int64_t base, int64_t k, int32_t smp,
                                             int32_t r, int32_t w, int32_t w0,
                                             const int64_t* __restrict__ rq_in,
                                             int32_t* __restrict__ rs_out,
                                             unsigned long long* __restrict__ rw_out,
                                             const int64_t* __restrict__ soff,
                                             int32_t* __restrict__ scur, int32_t m,
                                             SlotEntry* __restrict__ se) {
    const unsigned long long q = rw_out ? (unsigned long long)rq_in[base + k] : 0ull;
    if (rw_out)
        rw_out[base + r] = (q << kSampleBits) | unsigned(smp);
    else
        rs_out[base + r] = smp;
    const int32_t slot = atomicAdd(&scur[smp], 1);
    SlotEntry ent;
    ent.bw = int64_t((unsigned long long)base | ((unsigned long long)w << kBaseBits));
    ent.mpw = (unsigned long long)unsigned(m) | ((unsigned long long)unsigned(r) << 24) |
              ((unsigned long long)unsigned(w0) << 48);
    ent.v = rw_out ? q : (unsigned long long)L;
    se[soff[smp] + slot] = ent;
}

// Rank of sample smp in its list (members are distinct), the size of its window
// (members at cyclic distance 1..floor(N/2) after it) and of the window's part
// at distance <= seg0, by comparing with every member.
struct RankWin {
    int32_t r = 0, w = 0, w0 = 0;
    __device__ __forceinline__ void add(int32_t other, int32_t smp, int64_t n, int64_t seg0) {
        r += other < smp;
        int64_t d = int64_t(other) - smp;
        if (d < 0) d += n;
        w += d >= 1 && d <= n / 2;
        w0 += d >= 1 && d <= n / 2 && d <= seg0;
    }
};

// Lists of at most 64 members: one wave each, a member per lane, compared with
// every other member through lane broadcasts.
__global__ __launch_bounds__(256) void k_sort_small(const int64_t* __restrict__ roff,
                                                    const int32_t* __restrict__ ids, int64_t n_ids,
                                                    int64_t n, int64_t seg0,
                                                    const int32_t* __restrict__ rs_in,
                                                    const int64_t* __restrict__ rq_in,
                                                    int32_t* __restrict__ rs_out,
                                                    unsigned long long* __restrict__ rw_out,
                                                    const int64_t* __restrict__ soff,
                                                    int32_t* __restrict__ scur,
                                                    SlotEntry* __restrict__ se) {
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= n_ids) return;   // wave-uniform
    const int lane = threadIdx.x & 63;
    const int64_t L = ids[t];
    const int64_t base = roff[L];
    const int32_t m = int32_t(roff[L + 1] - base);
    const int32_t smp = lane < m ? rs_in[base + lane] : -1;
    RankWin rw;
    for (int32_t k = 0; k < m; ++k) rw.add(__shfl(smp, k, 64), smp, n, seg0);
    if (lane < m)
        place_member(L, base, lane, smp, rw.r, rw.w, rw.w0, rq_in, rs_out, rw_out, soff, scur, m, se);
}

// Longer lists: one workgroup each.  When the samples fit an LDS bitmap
// (bitmap_words > 0, one bit per sample), the members set their bits, an
// exclusive scan of the words' population counts gives, for any sample id x,
// the number of members below x in O(1); the rank and both window sizes are
// differences of such counts.  Otherwise every member is compared with every
// other one.
constexpr int kSortLds = 4096;

__device__ __forceinline__ int32_t members_below(const uint32_t* __restrict__ bits,
                                                 const uint32_t* __restrict__ pre, int64_t words,
                                                 int32_t m, int64_t x) {
    const int64_t wd = x >> 5;
    if (wd >= words) return m;
    const uint32_t below = (uint32_t(1) << (x & 31)) - 1u;
    return int32_t(pre[wd]) + __popc(bits[wd] & below);
}

// members at cyclic distance 1..len after s (len < n)
__device__ __forceinline__ int32_t members_after(const uint32_t* __restrict__ bits,
                                                 const uint32_t* __restrict__ pre, int64_t words,
                                                 int32_t m, int64_t n, int64_t s, int64_t len) {
    const int64_t a = s + 1, b = s + 1 + len;
    const int32_t at_a = members_below(bits, pre, words, m, a);
    if (b <= n) return members_below(bits, pre, words, m, b) - at_a;
    return (m - at_a) + members_below(bits, pre, words, m, b - n);
}

__global__ __launch_bounds__(256) void k_sort_large(const int64_t* __restrict__ roff,
                                                    const int32_t* __restrict__ ids, int64_t n,
                                                    int64_t seg0, int64_t bitmap_words,
                                                    const int32_t* __restrict__ rs_in,
                                                    const int64_t* __restrict__ rq_in,
                                                    int32_t* __restrict__ rs_out,
                                                    unsigned long long* __restrict__ rw_out,
                                                    const int64_t* __restrict__ soff,
                                                    int32_t* __restrict__ scur,
                                                    SlotEntry* __restrict__ se) {
    extern __shared__ uint32_t sh[];
    const int tid = threadIdx.x;
    const int64_t L = ids[blockIdx.x];
    const int64_t base = roff[L];
    const int64_t m = roff[L + 1] - base;
    if (bitmap_words > 0) {   // block-uniform
        const int64_t W = bitmap_words;
        uint32_t* bits = sh;
        uint32_t* pre = sh + W;
        __shared__ uint32_t wave_tot[4];
        for (int64_t k = tid; k < W; k += 256) bits[k] = 0u;
        __syncthreads();
        for (int64_t k = tid; k < m; k += 256) {
            const int32_t smp = rs_in[base + k];
            atomicOr(&bits[smp >> 5], uint32_t(1) << (smp & 31));
        }
        __syncthreads();
        // exclusive scan of the words' population counts: thread t owns a run of
        // consecutive words; runs are combined by a wave scan and the wave totals
        const int64_t per = (W + 255) / 256;
        const int64_t w0 = int64_t(tid) * per, w1 = min(W, w0 + per);
        uint32_t own = 0;
        for (int64_t k = w0; k < w1; ++k) own += __popc(bits[k]);
        const int lane = tid & 63, wave = tid >> 6;
        uint32_t inc = own;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wave_tot[wave] = inc;
        __syncthreads();
        uint32_t run = inc - own;
        for (int q = 0; q < wave; ++q) run += wave_tot[q];
        for (int64_t k = w0; k < w1; ++k) {
            pre[k] = run;
            run += __popc(bits[k]);
        }
        __syncthreads();
        const int32_t m32 = int32_t(m);
        const int64_t half = n / 2, part = min(half, seg0);
        for (int64_t k = tid; k < m; k += 256) {
            const int32_t smp = rs_in[base + k];
            const int32_t r = members_below(bits, pre, W, m32, smp);
            const int32_t w = members_after(bits, pre, W, m32, n, smp, half);
            const int32_t wz = members_after(bits, pre, W, m32, n, smp, part);
            place_member(L, base, k, smp, r, w, wz, rq_in, rs_out, rw_out, soff, scur, m32, se);
        }
        return;
    }
    int32_t* ks = reinterpret_cast<int32_t*>(sh);
    if (m <= kSortLds) {   // block-uniform
        for (int64_t k = tid; k < m; k += 256) ks[k] = rs_in[base + k];
        __syncthreads();
        for (int64_t k = tid; k < m; k += 256) {
            const int32_t smp = ks[k];
            RankWin rw;
            for (int64_t t = 0; t < m; ++t) rw.add(ks[t], smp, n, seg0);
            place_member(L, base, k, smp, rw.r, rw.w, rw.w0, rq_in, rs_out, rw_out, soff, scur,
                         int32_t(m), se);
        }
    } else {
        for (int64_t k = tid; k < m; k += 256) {
            const int32_t smp = rs_in[base + k];
            RankWin rw;
            for (int64_t t = 0; t < m; ++t) rw.add(rs_in[base + t], smp, n, seg0);
            place_member(L, base, k, smp, rw.r, rw.w, rw.w0, rq_in, rs_out, rw_out, soff, scur,
                         int32_t(m), se);
        }
    }
}

// Node-major chunk over a list of branch positions (the dense set): x = l * c / T
// as FP32, or as 32-bit fixed point rint(x * q) (T = uint32_t).
template <typename T>
__global__ __launch_bounds__(256) void k_embed_list(ufp::Emb e, const int32_t* __restrict__ list,
                                                    int64_t k0, int64_t kc, double q,
                                                    T* __restrict__ out) {
    constexpr int TK = 256, TS = 64;
    __shared__ T tile[TK][TS + 1];
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
        T v = T(0);
        if (kin && s < e.n) {
            const double x = lv * (double(ufd::count_in(e, s, lk, hk)) / e.total[s]);
            if constexpr (std::is_same<T, uint32_t>::value) v = uint32_t(llrint(x * q));
            else v = T(x);
        }
        tile[tid][j] = v;
    }
    __syncthreads();
    for (int r = tid / TS; r < TK; r += 256 / TS) {
        const int64_t kk = kb + r;
        const int64_t s = sb + (tid % TS);
        if (kk < kc && s < e.n) out[kk * e.n + s] = tile[r][tid % TS];
    }
}

// The same chunk by a forward merge, in two passes over the list (thread =
// sample; block = 256 samples x a run of kMergeQ list entries, whose positions
// and bounds are staged in LDS first; k in [k0, k0+kc)).
// Pass lo: visiting the entries in increasing lo (lo_ord: indices into list),
// the cursor over the sample's tips only moves forward; out[k - k0][s] takes the
// low 32 bits of the sample's count prefix below lo_k.  Pass hi: along the list
// (ascending positions, so non-decreasing hi) the prefix below hi_k minus that
// value is the count on branch k; it needs T_s < 2^32, so the 32-bit difference
// is exact.  Both passes give the values of k_embed_list bit for bit.  The
// prefix is re-read only in lanes whose cursor moved.
constexpr int kMergeQ = 64;

// Where element (k - k0, s) of the chunk goes: row-major [kc][n] (tabs null), or
// the block [kc][n_t] of the sample's table in a batch.
struct ChunkSlot {
    int64_t base, stride;
    __device__ ChunkSlot(int64_t s, int64_t n, const BatchTable* tabs, const int32_t* tab_of) {
        if (tabs) {
            const BatchTable t = tabs[tab_of[s]];
            base = t.e_off + (s - t.off);
            stride = t.n;
        } else {
            base = s;
            stride = n;
        }
    }
    __device__ size_t at(int64_t kk) const { return size_t(base + kk * stride); }
};

template <typename T>
__global__ __launch_bounds__(256) void k_embed_list_lo(ufp::Emb e, const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ lo_ord,
                                                       int64_t n_list, int64_t k0, int64_t kc,
                                                       const BatchTable* __restrict__ tabs,
                                                       const int32_t* __restrict__ tab_of,
                                                       T* __restrict__ out) {
    __shared__ int32_t qk[kMergeQ], ql[kMergeQ];
    const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
    uint32_t* o = reinterpret_cast<uint32_t*>(out);
    const int64_t nseg = (n_list + kMergeQ - 1) / kMergeQ;
    for (int64_t g = blockIdx.y; g < nseg; g += gridDim.y) {
        const int64_t t0 = g * kMergeQ;
        const int nq = n_list - t0 < kMergeQ ? int(n_list - t0) : kMergeQ;
        __syncthreads();
        if (threadIdx.x < nq) {
            const int32_t k = lo_ord[t0 + threadIdx.x];
            qk[threadIdx.x] = k;
            ql[threadIdx.x] = e.lo[list ? list[k] : k];
        }
        __syncthreads();
        if (s >= e.n) continue;
        const ChunkSlot slot(s, e.n, tabs, tab_of);
        const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
        int64_t cur = ufd::lower_bound_rank(e.rank, a, b, ql[0]);
        uint32_t below = uint32_t(e.cum[cur + s]);
        int32_t nxt = cur < b ? e.rank[cur] : 0x7fffffff;   // rank at the cursor
        for (int t = 0; t < nq; ++t) {
            const int32_t l = ql[t];
            const int64_t from = cur;
            while (nxt < l) {
                ++cur;
                nxt = cur < b ? e.rank[cur] : 0x7fffffff;
            }
            if (cur != from) below = uint32_t(e.cum[cur + s]);
            const int64_t k = qk[t];
            if (k >= k0 && k < k0 + kc) o[slot.at(k - k0)] = below;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_embed_list_hi(ufp::Emb e, const int32_t* __restrict__ list,
                                                       int64_t k0, int64_t kc, double q,
                                                       const BatchTable* __restrict__ tabs,
                                                       const int32_t* __restrict__ tab_of,
                                                       T* __restrict__ out) {
    __shared__ int32_t qh[kMergeQ];
    __shared__ double qlen[kMergeQ];
    const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t nseg = (kc + kMergeQ - 1) / kMergeQ;
    const double tot = s < e.n ? e.total[s] : 1.0;
    for (int64_t g = blockIdx.y; g < nseg; g += gridDim.y) {
        const int64_t t0 = k0 + g * kMergeQ;
        const int nq = k0 + kc - t0 < kMergeQ ? int(k0 + kc - t0) : kMergeQ;
        __syncthreads();
        if (threadIdx.x < nq) {
            const int64_t pos = list ? int64_t(list[t0 + threadIdx.x]) : t0 + threadIdx.x;
            qh[threadIdx.x] = e.hi[pos];
            qlen[threadIdx.x] = e.len[pos];
        }
        __syncthreads();
        if (s >= e.n) continue;
        const ChunkSlot slot(s, e.n, tabs, tab_of);
        const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
        int64_t cur = ufd::lower_bound_rank(e.rank, a, b, qh[0]);
        uint32_t below = uint32_t(e.cum[cur + s]);
        int32_t nxt = cur < b ? e.rank[cur] : 0x7fffffff;   // rank at the cursor
        for (int t = 0; t < nq; ++t) {
            const int32_t h = qh[t];
            const int64_t from = cur;
            while (nxt < h) {
                ++cur;
                nxt = cur < b ? e.rank[cur] : 0x7fffffff;
            }
            if (cur != from) below = uint32_t(e.cum[cur + s]);
            const size_t idx = slot.at(t0 + t - k0);
            const int64_t c = int64_t(below - reinterpret_cast<const uint32_t*>(out)[idx]);
            const double x = qlen[t] * (double(c) / tot);
            T v;
            if constexpr (std::is_same<T, uint32_t>::value) v = uint32_t(llrint(x * q));
            else v = T(x);
            out[idx] = v;
        }
    }
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

__global__ __launch_bounds__(256) void k_entry_lengths(SlotEntry* __restrict__ se, int64_t n_entries,
                                                       const int64_t* __restrict__ rl) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < n_entries) se[k].v = (unsigned long long)rl[se[k].v];
}

// Workgroup -> sample: each XCD takes a contiguous range of samples (blocks are
// dealt to the 8 XCDs round-robin), so neighbouring workgroups of an XCD write
// adjacent rows of the sample-major sums.
__device__ __forceinline__ int64_t xcd_sample(int64_t b, int64_t n) {
    const int64_t per = n / 8, rem = n % 8;
    const int64_t x = b % 8, k = b / 8;
    return x * per + (x < rem ? x : rem) + k;
}

constexpr int kSlotThreads = 1024;
constexpr int kSlotWaves = kSlotThreads / 64;

template <bool W>
__global__ __launch_bounds__(kSlotThreads) void k_rare_slots(
    const int32_t* __restrict__ rs, const unsigned long long* __restrict__ rw,
    const int64_t* __restrict__ soff, const SlotEntry* __restrict__ entries, int64_t n,
    int64_t sb, int64_t se, int64_t seg_len, int64_t seg0, unsigned long long* __restrict__ M) {
    extern __shared__ unsigned long long acc[];   // [seg_len]
    const int64_t i = xcd_sample(blockIdx.x, n);
    const int64_t g0 = sb + int64_t(blockIdx.y) * seg_len;
    const int64_t g1 = min(se, g0 + seg_len);
    const int64_t width = g1 - g0;
    for (int64_t k = threadIdx.x; k < width; k += kSlotThreads) acc[k] = 0ull;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr unsigned long long kMask = (1ull << kSampleBits) - 1;
    // stripe s pairs i with its cyclic successor at distance d = s + 1; stripes
    // run below floor(N/2), so the window is d in [g0 + 1, min(g1, N/2)]
    const int64_t dlo = g0 + 1;
    const int64_t dhi = min(g1, n / 2);
    const int64_t k_end = soff[i + 1];
    int64_t k = soff[i] + wave;
    SlotEntry nxt{};
    if (k < k_end) nxt = entries[k];
    for (; k < k_end; k += kSlotWaves) {
        const SlotEntry ent = nxt;
        if (k + kSlotWaves < k_end) nxt = entries[k + kSlotWaves];  // in flight meanwhile
        const int64_t base = ent.bw & ((int64_t(1) << kBaseBits) - 1);
        const int64_t w = int64_t((unsigned long long)ent.bw >> kBaseBits);
        const int64_t m = int64_t(ent.mpw & 0xFFFFFFull);
        const int64_t p = int64_t((ent.mpw >> 24) & 0xFFFFFFull);
        const int64_t w0 = int64_t(ent.mpw >> 48);
        const unsigned long long vi = ent.v;
        // the c-th member after i, cyclically, sits at position (p + 1 + c) mod m;
        // its distance from i grows with c, and members c < w lie within N/2
        auto pos_of = [&](int64_t c) {
            const int64_t q = p + 1 + c;
            return q >= m ? q - m : q;
        };
        auto sample_at = [&](int64_t q) -> int64_t {
            if constexpr (W) return int64_t(rw[base + q] & kMask);
            else return rs[base + q];
        };
        auto dist_of = [&](int64_t q) {
            const int64_t d = sample_at(q) - i;
            return d <= 0 ? d + n : d;
        };
        // first c in [lo, hi) whose distance reaches dt, else hi: 64-way search,
        // one probe per lane
        auto first_reaching = [&](int64_t dt, int64_t lo, int64_t hi) {
            while (lo < hi) {
                const int64_t step = (hi - lo + 63) / 64;
                const int64_t c = lo + int64_t(lane) * step;
                const bool pred = c < hi && dist_of(pos_of(c)) >= dt;
                const unsigned long long ball = __ballot(pred);
                if (ball) {
                    const int64_t f = __ffsll((long long)ball) - 1;
                    if (f == 0) {
                        hi = lo;
                    } else {
                        hi = lo + f * step;
                        lo = lo + (f - 1) * step + 1;
                    }
                } else {
                    lo = lo + ((hi - 1 - lo) / step) * step + 1;
                }
            }
            return hi;
        };
        // segment edges at distance 0, floor(N/2) or seg0 need no search
        const int64_t c_lo = dlo == 1 ? 0 : (dlo == seg0 + 1 ? w0 : first_reaching(dlo, 0, w));
        const int64_t c_hi = dhi >= n / 2 ? w : (dhi == seg0 ? w0 : first_reaching(dhi + 1, c_lo, w));
        // members c in [c_lo, c_hi) all fall in this segment: rounds of eight loads
        // in flight per lane, then their LDS adds.  Full rounds run unchecked, with
        // per-lane positions and distances in 32 bits (samples, N, list lengths
        // and stripes are below 2^24); the last round loads and adds only below
        // c_hi.
        constexpr int U = 8;
        int64_t c0 = c_lo;
        {
            const int32_t m32 = int32_t(m), i32 = int32_t(i), n32 = int32_t(n), a0 = int32_t(g0) + 1;
            const int32_t q_first = int32_t(p + 1);
            for (; c0 + 64 * U <= c_hi; c0 += 64 * U) {
                unsigned long long word[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int32_t q = q_first + int32_t(c0) + lane + 64 * u;
                    q -= q >= m32 ? m32 : 0;
                    if constexpr (W) word[u] = rw[base + uint32_t(q)];
                    else word[u] = (unsigned long long)(unsigned)rs[base + uint32_t(q)];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t j = int32_t(word[u] & kMask);
                    unsigned long long v = vi;
                    if constexpr (W) {
                        const unsigned long long vj = word[u] >> kSampleBits;
                        v = vj < vi ? vj : vi;
                    }
                    int32_t d = j - i32;
                    d += d <= 0 ? n32 : 0;
                    atomicAdd(&acc[d - a0], v);
                }
            }
        }
        if (c0 < c_hi) {
            unsigned long long word[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t c = c0 + lane + 64 * u;
                word[u] = 0;
                if (c < c_hi) {
                    if constexpr (W) word[u] = rw[base + pos_of(c)];
                    else word[u] = (unsigned long long)(unsigned)rs[base + pos_of(c)];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (c0 + lane + 64 * u >= c_hi) continue;
                const int64_t j = int64_t(word[u] & kMask);
                unsigned long long v = vi;
                if constexpr (W) {
                    const unsigned long long vj = word[u] >> kSampleBits;
                    v = vj < vi ? vj : vi;
                }
                int64_t d = j - i;
                if (d <= 0) d += n;
                atomicAdd(&acc[d - 1 - g0], v);
            }
        }
    }
    __syncthreads();
    // sample-major: this sample's row of M is written contiguously
    const int64_t sr = se - sb;
    for (int64_t k = threadIdx.x; k < width; k += kSlotThreads) M[i * sr + (g0 + k - sb)] = acc[k];
}

}  // namespace

hipError_t branch_points(const ufp::Emb& e, int32_t* pt, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_branch_points, dim3(unsigned(e.n)), dim3(256), 0, st, e, pt);
    return hipGetLastError();
}

hipError_t split_fill(const ufp::Emb& e, bool weighted, const int32_t* cls, int4* nodes,
                      const int64_t* roff, int32_t* rfill, int32_t* rs, int64_t* rq,
                      unsigned long long* sigma, int32_t* scnt, int32_t* dnnz, double fix,
                      hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    const int64_t nb = e.root_pos;
    if (nb > 0) {
        hipLaunchKernelGGL(k_pack_nodes, dim3(unsigned((nb + 255) / 256)), dim3(256), 0, st, e, cls,
                           nb, nodes);
        hipError_t er = hipGetLastError();
        if (er != hipSuccess) return er;
    }
    if (weighted)
        hipLaunchKernelGGL(k_split_fill<true>, dim3(unsigned(e.n)), dim3(256), 0, st, e, nodes, roff,
                           rfill, rs, rq, sigma, scnt, dnnz, fix);
    else
        hipLaunchKernelGGL(k_split_fill<false>, dim3(unsigned(e.n)), dim3(256), 0, st, e, nodes, roff,
                           rfill, rs, rq, sigma, scnt, dnnz, fix);
    return hipGetLastError();
}

hipError_t sort_lists(const int64_t* roff, const int32_t* small_ids, int64_t n_small,
                      const int32_t* large_ids, int64_t n_large, int64_t n, int64_t seg0,
                      const int32_t* rs_in, const int64_t* rq_in, int32_t* rs_out,
                      unsigned long long* rw_out, const int64_t* soff, int32_t* scur,
                      SlotEntry* se, hipStream_t st) {
    if (n_small > 0) {
        const int64_t blocks = (n_small + 3) / 4;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sort_small, dim3(unsigned(blocks)), dim3(256), 0, st, roff, small_ids,
                           n_small, n, seg0, rs_in, rq_in, rs_out, rw_out, soff, scur, se);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_large <= 0) return hipSuccess;
    if (n_large > 0x7fffffff) return hipErrorInvalidValue;
    // a bitmap of the samples and the scan of its words, while they fit in 64 KiB
    // (N up to about 260,000); else the pairwise comparison with a 16 KiB list copy
    // (UF_SPLIT_SORT=pairwise in the environment forces the pairwise ranking)
    constexpr int64_t kBitmapBytes = 64 * 1024;
    const int64_t words = (n + 31) / 32;
    const char* mode = std::getenv("UF_SPLIT_SORT");
    const bool pairwise = mode && std::strcmp(mode, "pairwise") == 0;
    const bool bitmap = words * 8 <= kBitmapBytes && !pairwise;
    const size_t lds = bitmap ? size_t(words) * 8 : size_t(kSortLds) * 4;
    static const bool attr_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_large),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    int(kBitmapBytes)) == hipSuccess;
    if (!attr_ok) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_large, dim3(unsigned(n_large)), dim3(256), lds, st, roff, large_ids, n,
                       seg0, bitmap ? words : int64_t(0), rs_in, rq_in, rs_out, rw_out, soff, scur,
                       se);
    return hipGetLastError();
}

hipError_t entry_lengths(SlotEntry* se, int64_t n_entries, const int64_t* rl, hipStream_t st) {
    if (n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_entry_lengths, dim3(unsigned((n_entries + 255) / 256)), dim3(256), 0, st, se,
                       n_entries, rl);
    return hipGetLastError();
}

template <typename T>
static hipError_t embed_list(const ufp::Emb& e, const int32_t* list, const int32_t* lo_ord,
                             int64_t n_list, bool merge, int64_t k0, int64_t kc, double q, T* out,
                             hipStream_t st) {
    if (kc <= 0 || e.n <= 0) return hipSuccess;
    if (merge && lo_ord && n_list >= k0 + kc) {
        const int64_t gx = (e.n + 255) / 256;
        const int64_t gy_lo = std::min<int64_t>((n_list + kMergeQ - 1) / kMergeQ, 65535);
        const int64_t gy_hi = std::min<int64_t>((kc + kMergeQ - 1) / kMergeQ, 65535);
        if (gx > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_embed_list_lo<T>, dim3(unsigned(gx), unsigned(gy_lo)), dim3(256), 0, st,
                           e, list, lo_ord, n_list, k0, kc, static_cast<const BatchTable*>(nullptr),
                           static_cast<const int32_t*>(nullptr), out);
        hipError_t rc = hipGetLastError();
        if (rc != hipSuccess) return rc;
        hipLaunchKernelGGL(k_embed_list_hi<T>, dim3(unsigned(gx), unsigned(gy_hi)), dim3(256), 0, st,
                           e, list, k0, kc, q, static_cast<const BatchTable*>(nullptr),
                           static_cast<const int32_t*>(nullptr), out);
        return hipGetLastError();
    }
    const int64_t gy = (e.n + 63) / 64;
    if (gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_embed_list<T>, dim3(unsigned((kc + 255) / 256), unsigned(gy)), dim3(256), 0,
                       st, e, list, k0, kc, q, out);
    return hipGetLastError();
}

hipError_t embed_list_f32(const ufp::Emb& e, const int32_t* list, const int32_t* lo_ord,
                          int64_t n_list, bool merge, int64_t k0, int64_t kc, float* out,
                          hipStream_t st) {
    return embed_list<float>(e, list, lo_ord, n_list, merge, k0, kc, 1.0, out, st);
}

hipError_t embed_list_u32(const ufp::Emb& e, const int32_t* list, const int32_t* lo_ord,
                          int64_t n_list, bool merge, int64_t k0, int64_t kc, double q,
                          uint32_t* out, hipStream_t st) {
    return embed_list<uint32_t>(e, list, lo_ord, n_list, merge, k0, kc, q, out, st);
}

hipError_t embed_batch_merge_f32(const ufp::Emb& e, const BatchTable* tabs, const int32_t* tab_of,
                                 const int32_t* lo_ord_chunk, int64_t k0, int64_t kc, float* out,
                                 hipStream_t st) {
    if (kc <= 0 || e.n <= 0) return hipSuccess;
    const int64_t gx = (e.n + 255) / 256;
    const int64_t gy = std::min<int64_t>((kc + kMergeQ - 1) / kMergeQ, 65535);
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_embed_list_lo<float>, dim3(unsigned(gx), unsigned(gy)), dim3(256), 0, st, e,
                       static_cast<const int32_t*>(nullptr), lo_ord_chunk, kc, k0, kc, tabs, tab_of,
                       out);
    hipError_t rc = hipGetLastError();
    if (rc != hipSuccess) return rc;
    hipLaunchKernelGGL(k_embed_list_hi<float>, dim3(unsigned(gx), unsigned(gy)), dim3(256), 0, st, e,
                       static_cast<const int32_t*>(nullptr), k0, kc, 1.0, tabs, tab_of, out);
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

hipError_t rare_slots(const int32_t* rs, const unsigned long long* rw, const int64_t* soff,
                      const SlotEntry* entries, int64_t n, int64_t sb, int64_t se,
                      unsigned long long* M, hipStream_t st) {
    if (se <= sb || n <= 0) return hipSuccess;
    if (n > 0x7fffffff || (rw && n > (int64_t(1) << kSampleBits))) return hipErrorInvalidValue;
    const int64_t seg_len = slot_segment_len(sb, se);
    const int64_t nseg = (se - sb + seg_len - 1) / seg_len;
    const int64_t seg0 = slot_segment_len(0, n / 2);   // boundary the entries count w0 for
    if (nseg > 65535) return hipErrorInvalidValue;
    const dim3 grid{unsigned(n), unsigned(nseg)};
    const size_t lds = size_t(seg_len) * 8;
    static const bool attr_ok = [] {
        const int most = int(kSegStripes * 8);
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rare_slots<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, most) == hipSuccess &&
               hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rare_slots<false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, most) == hipSuccess;
    }();
    if (!attr_ok) return hipErrorInvalidValue;
    if (rw)
        hipLaunchKernelGGL(k_rare_slots<true>, grid, dim3(kSlotThreads), lds, st, rs, rw, soff,
                           entries, n, sb, se, seg_len, seg0, M);
    else
        hipLaunchKernelGGL(k_rare_slots<false>, grid, dim3(kSlotThreads), lds, st, rs, rw, soff,
                           entries, n, sb, se, seg_len, seg0, M);
    return hipGetLastError();
}

}  // namespace ufs
