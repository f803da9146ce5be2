// Mantel test between two condensed distance matrices (gfx950).
//
// Statistic: Pearson's r between the condensed vectors x and y, or Spearman's
// (Pearson's on the average-tie ranks).  With x' and y' centred and scaled to
// unit norm, r = sum_k x'_k y'_k, and a relabelling pi of the first matrix's
// samples gives r_pi = sum_{i<j} y'_ij x'_{pi(i) pi(j)} (the multiset of x' and
// so its mean and norm do not change).  x' is expanded to a full square matrix
// S so that x'_{pi(i) pi(j)} lies in row pi(i).  One workgroup takes the rows i
// and N-2-i (together N-1 partners) for a batch of permutations, one permutation
// after another: it holds its partners' y'_ij and pi(j) in registers, stages
// row pi(i) of S in LDS part by part (coalesced), and gathers from LDS, so each
// permutation streams S once in order and the random access stays inside LDS.
// The observed statistic runs through the same kernel with the identity, so the
// comparisons behind the p-value see identical arithmetic.  Every reduction runs
// in a fixed order.
//
// Ranks (Spearman): a stable LSD radix sort of the order-preserving 64-bit
// images of the values, 8 bits per pass (per-block digit histograms, their
// exclusive scan, a stable scatter; bytes in which no two keys differ are
// skipped), then runs of equal keys get the mean of the positions they span,
// plus one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "uf.h"
#include "uf_internal.h"

namespace ufm {
namespace {

constexpr int kPB = 8;                 // permutations per batch
constexpr int kRowThreads = 1024;      // threads of the permutation kernel
constexpr int kJPT = 32;               // partners held in registers per thread
constexpr int64_t kPartMax = 19456;    // LDS row part: 152 KiB, + 8 KiB for the reduction
constexpr int64_t kChunk = 1 << 16;    // elements per partial sum
constexpr int kScanBlock = 1024;       // elements per scan block (256 threads x 4)
constexpr int kTile = 64;

__device__ __forceinline__ int64_t cidx(int64_t n, int64_t a, int64_t b) {   // a < b
    return a * n - a * (a + 1) / 2 + (b - a - 1);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// parts[b] = sum over chunk b of (v - shift)^power (power 1 or 2)
__global__ __launch_bounds__(256) void k_chunk_sums(const double* __restrict__ v, int64_t m,
                                                    double shift, int power,
                                                    double* __restrict__ parts) {
    __shared__ double red[256];
    const int64_t a = int64_t(blockIdx.x) * kChunk, b = min(m, a + kChunk);
    double s = 0.0;
    for (int64_t k = a + threadIdx.x; k < b; k += 256) {
        const double d = v[k] - shift;
        s += power == 2 ? d * d : d;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// out[k] = (v[k] - mean) * scale
__global__ __launch_bounds__(256) void k_standardize(const double* __restrict__ v, int64_t m,
                                                     double mean, double scale,
                                                     double* __restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < m) out[k] = (v[k] - mean) * scale;
}

// Full square S[i][j] = (v_ij - mean) * scale for i != j, 0 on the diagonal.  Block
// (bi, bj), bi <= bj: the tile is read from the condensed rows (contiguous in j)
// and written to S[i][j] and, through LDS, to S[j][i], both coalesced.
__global__ __launch_bounds__(256) void k_square(const double* __restrict__ v, int64_t n,
                                                double mean, double scale,
                                                double* __restrict__ S) {
    __shared__ double t[kTile][kTile + 1];
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi) return;
    const int64_t i0 = bi * kTile, j0 = bj * kTile;
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int r = e / kTile, c = e % kTile;
        const int64_t i = i0 + r, j = j0 + c;
        double x = 0.0;
        if (i < n && j < n && i != j) {
            const double d = i < j ? v[cidx(n, i, j)] : v[cidx(n, j, i)];
            x = (d - mean) * scale;
        }
        t[r][c] = x;
        if (i < n && j < n) S[i * n + j] = x;
    }
    if (bi == bj) return;
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int r = e / kTile, c = e % kTile;   // output row j0 + r, column i0 + c
        const int64_t j = j0 + r, i = i0 + c;
        if (i < n && j < n) S[j * n + i] = t[c][r];
    }
}

// part[b][w] for permutations b0 + [0, nb) (perm == nullptr: identity, nb = 1):
// sum over the rows w and n-2-w of sum_{j>i} y'_ij S[pi(i)][pi(j)].
// One block of kRowThreads threads per (row pair, batch).  The block keeps its
// partners' y'_ij (up to kJPT per thread) and pi(j) in registers and streams the
// permuted row S[pi(i)] through LDS in parts of part_len: each part goes in with
// direct-to-LDS loads, all of it in flight at once, then the block gathers
// S[pi(i)][pi(j)] from it.  Each permutation reads S once, in order.
__global__ __launch_bounds__(kRowThreads) void k_perm_rows(const double* __restrict__ S,
                                                           const double* __restrict__ yv, int64_t n,
                                                           const int32_t* __restrict__ perm,
                                                           int64_t b0, int nb, int64_t n_pairs,
                                                           int64_t part_len,
                                                           double* __restrict__ part) {
    extern __shared__ double lds[];           // [part_len], then kRowThreads for the reduction
    double* red = lds + part_len;
    const int64_t w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nparts = (n + part_len - 1) / part_len;
    for (int q = 0; q < nb; ++q) {            // one permutation at a time; y' rows stay in L2
        const int32_t* pb = perm ? perm + (b0 + q) * n : nullptr;
        double a = 0.0;
        for (int side = 0; side < 2; ++side) {
            const int64_t i = side == 0 ? w : n - 2 - w;
            if (side == 1 && i == w) break;
            if (i < 0 || i >= n - 1) continue;
            const int64_t base = cidx(n, i, i + 1);   // y'_{i, i+1 ..}
            const int64_t pi = pb ? int64_t(pb[i]) : i;
            const uint32_t* srow = reinterpret_cast<const uint32_t*>(S + pi * n);
            // part k of the row into LDS, 64 dwords per wave instruction
            auto issue = [&](int64_t k) {
                const int64_t lo = k * part_len;
                const int len2 = int(2 * min(part_len, n - lo));
                const uint32_t* src = srow + 2 * lo;
                uint32_t* dst = reinterpret_cast<uint32_t*>(lds);
                for (int c = 64 * wave; c < len2; c += kRowThreads)
                    if (c + lane < len2) __builtin_amdgcn_global_load_lds(src + c + lane, dst + c, 4, 0, 0);
            };
            for (int64_t jc = i + 1; jc < n; jc += int64_t(kRowThreads) * kJPT) {
                double yr[kJPT];
                int32_t pr[kJPT];
#pragma unroll
                for (int t = 0; t < kJPT; ++t) {
                    const int64_t j = jc + tid + int64_t(kRowThreads) * t;
                    yr[t] = j < n ? yv[base + (j - i - 1)] : 0.0;
                    pr[t] = j < n ? (pb ? pb[j] : int32_t(j)) : -1;
                }
                for (int64_t k = 0; k < nparts; ++k) {
                    __syncthreads();   // every wave done with the previous part
                    issue(k);
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();   // part k in LDS for every wave
                    const double* row = lds;
                    const int lo32 = int(k * part_len);
                    const int len = int(min(part_len, n - k * part_len));
#pragma unroll
                    for (int t = 0; t < kJPT; ++t) {
                        const int c = pr[t] - lo32;
                        if (c >= 0 && c < len) a = fma(yr[t], row[c], a);
                    }
                }
            }
        }
        red[tid] = a;
        __syncthreads();
        for (int s2 = kRowThreads / 2; s2 > 0; s2 >>= 1) {
            if (tid < s2) red[tid] += red[tid + s2];
            __syncthreads();
        }
        if (tid == 0) part[(b0 + q) * n_pairs + w] = red[0];
        __syncthreads();
    }
}

// tot[b] = sum_w part[b][w] (one block per permutation, fixed order)
__global__ __launch_bounds__(256) void k_perm_total(const double* __restrict__ part, int64_t n_pairs,
                                                    double* __restrict__ tot) {
    __shared__ double red[256];
    const int64_t b = blockIdx.x;
    double s = 0.0;
    for (int64_t w = threadIdx.x; w < n_pairs; w += 256) s += part[b * n_pairs + w];
    s = block_sum(s, red);
    if (threadIdx.x == 0) tot[b] = s;
}

// ---------------------------------------------------------------- ranks
__device__ __forceinline__ unsigned long long order_key(double v) {
    if (v == 0.0) v = 0.0;   // -0 and +0 are the same value
    const unsigned long long u = __double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_keys(const double* __restrict__ v, int64_t m,
                                              unsigned long long* __restrict__ key,
                                              uint32_t* __restrict__ idx) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < m) {
        key[k] = order_key(v[k]);
        idx[k] = uint32_t(k);
    }
}

// z[k] = 1 if bit `bit` of key[k] is 0
// ---- stable LSD radix sort of the order keys, 8 bits per pass ----
constexpr int kRadixItems = 16;                      // elements per thread per block
constexpr int64_t kRadixBlock = 256 * kRadixItems;   // elements per block

// vary |= OR over all keys of (key ^ key[0]): the bits in which keys differ
__global__ __launch_bounds__(256) void k_key_vary(const unsigned long long* __restrict__ key,
                                                  int64_t m, unsigned long long* __restrict__ vary) {
    const unsigned long long k0 = key[0];
    unsigned long long acc = 0;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < m; k += int64_t(gridDim.x) * 256)
        acc |= key[k] ^ k0;
    for (int off = 32; off > 0; off >>= 1) acc |= __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr(vary, acc);
}

// H[d * nblk + b]: elements of block b whose digit (key >> sh) & 255 is d
__global__ __launch_bounds__(256) void k_digit_hist(const unsigned long long* __restrict__ key,
                                                    int64_t m, int sh, int64_t nblk,
                                                    uint32_t* __restrict__ H) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x, base = b * kRadixBlock;
    h[tid] = 0;
    unsigned long long kk[kRadixItems];
#pragma unroll
    for (int u = 0; u < kRadixItems; ++u) {
        const int64_t k = base + u * 256 + tid;
        kk[u] = k < m ? key[k] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRadixItems; ++u)
        if (base + u * 256 + tid < m) atomicAdd(&h[(kk[u] >> sh) & 255ull], 1u);
    __syncthreads();
    H[int64_t(tid) * nblk + b] = h[tid];
}

// Stable scatter by digit: Hs is the exclusive scan of H (digit-major), so
// Hs[d * nblk + b] is where block b's first element of digit d goes.  Within
// the block the elements are taken in order, 256 per round: a lane's rank
// among the same digit in its wave comes from eight ballots on the digit bits;
// the waves of a round and the earlier rounds add their counts (LDS).
__global__ __launch_bounds__(256) void k_digit_scatter(const unsigned long long* __restrict__ key,
                                                       const uint32_t* __restrict__ idx, int64_t m,
                                                       int sh, int64_t nblk,
                                                       const uint32_t* __restrict__ Hs,
                                                       unsigned long long* __restrict__ key_out,
                                                       uint32_t* __restrict__ idx_out) {
    __shared__ uint32_t cnt[4][256];   // per wave of the round: count, then its offset
    __shared__ uint32_t run[256];      // elements of each digit in earlier rounds
    __shared__ uint32_t start[256];    // global position of the block's first element of d
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b = blockIdx.x, base = b * kRadixBlock;
    start[tid] = Hs[int64_t(tid) * nblk + b];
    run[tid] = 0;
    unsigned long long kk[kRadixItems];
    uint32_t ii[kRadixItems];
#pragma unroll
    for (int u = 0; u < kRadixItems; ++u) {
        const int64_t k = base + u * 256 + tid;
        kk[u] = k < m ? key[k] : 0ull;
        ii[u] = k < m ? idx[k] : 0u;
    }
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int u = 0; u < kRadixItems; ++u) {
        const bool valid = base + u * 256 + tid < m;
        const uint32_t d = uint32_t((kk[u] >> sh) & 255ull);
        for (int w = 0; w < 4; ++w) cnt[w][tid] = 0;
        __syncthreads();
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long bb = __ballot(set);
            same &= set ? bb : ~bb;
        }
        const uint32_t r = uint32_t(__popcll(same & below));
        if (valid && r == 0) cnt[wave][d] = uint32_t(__popcll(same));
        __syncthreads();
        {
            const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
            const uint32_t r0 = run[tid];
            cnt[0][tid] = r0;
            cnt[1][tid] = r0 + c0;
            cnt[2][tid] = r0 + c0 + c1;
            cnt[3][tid] = r0 + c0 + c1 + c2;
            run[tid] = r0 + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dest = start[d] + cnt[wave][d] + r;
            key_out[dest] = kk[u];
            idx_out[dest] = ii[u];
        }
        __syncthreads();
    }
}

// Block-level exclusive scan of kScanBlock elements; block totals to agg.
__global__ __launch_bounds__(256) void k_scan_block(const uint32_t* __restrict__ in, int64_t m,
                                                    uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ agg) {
    __shared__ uint32_t s[256];
    const int64_t base = int64_t(blockIdx.x) * kScanBlock + threadIdx.x * 4;
    uint32_t v[4];
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = base + q < m ? in[base + q] : 0u;
        t += v[q];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele
        const uint32_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - t;   // exclusive prefix of this thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < m) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255) agg[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* __restrict__ out, int64_t m,
                                                  const uint32_t* __restrict__ off) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < m) out[k] += off[k / kScanBlock];
}

// run starts (flag) over sorted keys
__global__ __launch_bounds__(256) void k_run_starts(const unsigned long long* __restrict__ key,
                                                    int64_t m, uint32_t* __restrict__ f) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < m) f[k] = (k == 0 || key[k] != key[k - 1]) ? 1u : 0u;
}

// run r = (exclusive scan of starts) at its start, inclusive at any member; record
// first and last positions of each run
__global__ __launch_bounds__(256) void k_run_bounds(const unsigned long long* __restrict__ key,
                                                    const uint32_t* __restrict__ f,
                                                    const uint32_t* __restrict__ fpos, int64_t m,
                                                    uint32_t* __restrict__ first,
                                                    uint32_t* __restrict__ last) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= m) return;
    const uint32_t run = fpos[k] + f[k] - 1u;
    if (f[k]) first[run] = uint32_t(k);
    if (k == m - 1 || key[k] != key[k + 1]) last[run] = uint32_t(k);
}

__global__ __launch_bounds__(256) void k_assign_ranks(const uint32_t* __restrict__ idx,
                                                      const uint32_t* __restrict__ f,
                                                      const uint32_t* __restrict__ fpos,
                                                      const uint32_t* __restrict__ first,
                                                      const uint32_t* __restrict__ last, int64_t m,
                                                      double* __restrict__ rank) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= m) return;
    const uint32_t run = fpos[k] + f[k] - 1u;
    rank[idx[k]] = 0.5 * (double(first[run]) + double(last[run])) + 1.0;
}

// bad[0] = 1 if any permutation entry lies outside [0, n)
__global__ __launch_bounds__(256) void k_check_perms(const int32_t* __restrict__ perm, int64_t total,
                                                     int64_t n, uint32_t* __restrict__ bad) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < total && (perm[k] < 0 || int64_t(perm[k]) >= n)) atomicOr(bad, 1u);
}

unsigned grid_of(int64_t m) { return unsigned((m + 255) / 256); }

}  // namespace
}  // namespace ufm

using ufh::fail;
using ufh::hip_fail;

#define UFM_HIP(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

namespace {

struct MantelPlan {
    int64_t n = 0, m = 0, n_pairs = 0, n_perm = 0;
    size_t off_sq = 0, off_y = 0, off_part = 0, off_tot = 0, off_cs = 0, off_rx = 0, off_ry = 0,
           off_ka = 0, off_kb = 0, off_ia = 0, off_ib = 0, off_z = 0, off_zp = 0, off_agg = 0,
           off_first = 0, off_last = 0, off_h = 0, off_hs = 0, off_vary = 0, total = 0;
    int64_t agg_len = 0, nblk = 0;
};

size_t take(size_t& off, size_t bytes) {
    const size_t at = (off + 255) & ~size_t(255);
    off = at + bytes;
    return at;
}

MantelPlan mantel_plan(int64_t n, int method, int64_t n_perm) {
    MantelPlan p;
    p.n = n;
    p.m = n * (n - 1) / 2;
    p.n_pairs = n / 2;   // row pairs (w, n-2-w) over rows 0..n-2: ceil((n-1)/2) = floor(n/2)
    p.n_perm = n_perm;
    size_t off = 0;
    p.off_sq = take(off, size_t(n) * size_t(n) * 8);
    p.off_y = take(off, size_t(p.m) * 8);
    p.off_part = take(off, size_t(n_perm + 1) * size_t(p.n_pairs) * 8);
    p.off_tot = take(off, size_t(n_perm + 1) * 8);
    p.off_cs = take(off, size_t((p.m + ufm::kChunk - 1) / ufm::kChunk + 1) * 8);
    if (method == UF_MANTEL_SPEARMAN) {
        p.off_rx = take(off, size_t(p.m) * 8);
        p.off_ry = take(off, size_t(p.m) * 8);
        p.off_ka = take(off, size_t(p.m) * 8);
        p.off_kb = take(off, size_t(p.m) * 8);
        p.off_ia = take(off, size_t(p.m) * 4);
        p.off_ib = take(off, size_t(p.m) * 4);
        p.off_z = take(off, size_t(p.m) * 4);
        p.off_zp = take(off, size_t(p.m) * 4);
        // radix passes: per-block digit histograms and their scan
        p.nblk = (p.m + ufm::kRadixBlock - 1) / ufm::kRadixBlock;
        p.off_h = take(off, size_t(256 * p.nblk) * 4);
        p.off_hs = take(off, size_t(256 * p.nblk) * 4);
        p.off_vary = take(off, 8);
        // scan_u32 at a level of v values uses nb aggregates, and when nb > 1 their
        // scan (nb) plus one spare slot, then the next level's space; it scans m
        // run flags and 256 * nblk histogram entries
        auto agg_for = [](int64_t lv) {
            int64_t len = 0;
            for (;;) {
                const int64_t nb = (lv + ufm::kScanBlock - 1) / ufm::kScanBlock;
                len += nb;
                if (nb <= 1) break;
                len += nb + 1;
                lv = nb;
            }
            return len + 1;
        };
        p.agg_len = std::max(agg_for(p.m), agg_for(256 * p.nblk));
        p.off_agg = take(off, size_t(p.agg_len) * 4);
        p.off_first = take(off, size_t(p.m) * 4);
        p.off_last = take(off, size_t(p.m) * 4);
    }
    p.total = off + 256;
    return p;
}

// exclusive scan of m uint32 values, recursive over block aggregates
hipError_t scan_u32(const uint32_t* in, uint32_t* out, int64_t m, uint32_t* agg, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t nb = (m + ufm::kScanBlock - 1) / ufm::kScanBlock;
    hipLaunchKernelGGL(ufm::k_scan_block, dim3(unsigned(nb)), dim3(256), 0, s, in, m, out, agg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    uint32_t* agg_scan = agg + nb;   // exclusive scan of the aggregates, then the next level
    e = scan_u32(agg, agg_scan, nb, agg_scan + nb + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ufm::k_scan_add, dim3(ufm::grid_of(m)), dim3(256), 0, s, out, m, agg_scan);
    return hipGetLastError();
}

// fixed-order sum of (v - shift)^power over m values (host finishes the chunk sums)
uf_status chunk_sum(const double* v, int64_t m, double shift, int power, double* parts, hipStream_t s,
                    double* out) {
    const int64_t nb = (m + ufm::kChunk - 1) / ufm::kChunk;
    hipLaunchKernelGGL(ufm::k_chunk_sums, dim3(unsigned(nb)), dim3(256), 0, s, v, m, shift, power,
                       parts);
    UFM_HIP(hipGetLastError());
    std::vector<double> h(static_cast<size_t>(nb));
    UFM_HIP(hipMemcpyAsync(h.data(), parts, size_t(nb) * 8, hipMemcpyDeviceToHost, s));
    UFM_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double x : h) t += x;
    *out = t;
    return UF_OK;
}

// average-tie ranks of v (m values) into rank
uf_status ranks(const MantelPlan& p, char* base, const double* v, double* rank, hipStream_t s) {
    using namespace ufm;
    const int64_t m = p.m;
    auto* ka = reinterpret_cast<unsigned long long*>(base + p.off_ka);
    auto* kb = reinterpret_cast<unsigned long long*>(base + p.off_kb);
    auto* ia = reinterpret_cast<uint32_t*>(base + p.off_ia);
    auto* ib = reinterpret_cast<uint32_t*>(base + p.off_ib);
    auto* z = reinterpret_cast<uint32_t*>(base + p.off_z);
    auto* zp = reinterpret_cast<uint32_t*>(base + p.off_zp);
    auto* agg = reinterpret_cast<uint32_t*>(base + p.off_agg);
    auto* first = reinterpret_cast<uint32_t*>(base + p.off_first);
    auto* last = reinterpret_cast<uint32_t*>(base + p.off_last);
    auto* H = reinterpret_cast<uint32_t*>(base + p.off_h);
    auto* Hs = reinterpret_cast<uint32_t*>(base + p.off_hs);
    auto* vary = reinterpret_cast<unsigned long long*>(base + p.off_vary);
    hipLaunchKernelGGL(k_keys, dim3(grid_of(m)), dim3(256), 0, s, v, m, ka, ia);
    UFM_HIP(hipGetLastError());
    // bytes in which the keys differ; the passes over the others change nothing
    UFM_HIP(hipMemsetAsync(vary, 0, 8, s));
    hipLaunchKernelGGL(k_key_vary, dim3(std::min<unsigned>(grid_of(m), 4096u)), dim3(256), 0, s, ka,
                       m, vary);
    UFM_HIP(hipGetLastError());
    unsigned long long hvary = 0;
    UFM_HIP(hipMemcpyAsync(&hvary, vary, 8, hipMemcpyDeviceToHost, s));
    UFM_HIP(hipStreamSynchronize(s));
    for (int sh = 0; sh < 64; sh += 8) {
        if (((hvary >> sh) & 255ull) == 0) continue;
        hipLaunchKernelGGL(k_digit_hist, dim3(unsigned(p.nblk)), dim3(256), 0, s, ka, m, sh, p.nblk,
                           H);
        UFM_HIP(hipGetLastError());
        UFM_HIP(scan_u32(H, Hs, 256 * p.nblk, agg, s));
        hipLaunchKernelGGL(k_digit_scatter, dim3(unsigned(p.nblk)), dim3(256), 0, s, ka, ia, m, sh,
                           p.nblk, Hs, kb, ib);
        UFM_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(ia, ib);
    }
    hipLaunchKernelGGL(k_run_starts, dim3(grid_of(m)), dim3(256), 0, s, ka, m, z);
    UFM_HIP(hipGetLastError());
    UFM_HIP(scan_u32(z, zp, m, agg, s));
    hipLaunchKernelGGL(k_run_bounds, dim3(grid_of(m)), dim3(256), 0, s, ka, z, zp, m, first, last);
    UFM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_assign_ranks, dim3(grid_of(m)), dim3(256), 0, s, ia, z, zp, first, last, m,
                       rank);
    UFM_HIP(hipGetLastError());
    return UF_OK;
}

}  // namespace

extern "C" {

uf_status uf_mantel_workspace_size(int64_t n, int method, int64_t n_perm, size_t* bytes) {
    if (!bytes) return fail(UF_ERR_ARG, "bytes is NULL");
    if (n < 3) return fail(UF_ERR_ARG, "need at least 3 samples");
    if (method != UF_MANTEL_PEARSON && method != UF_MANTEL_SPEARMAN)
        return fail(UF_ERR_ARG, "unknown method");
    if (method == UF_MANTEL_SPEARMAN && n > 65535)
        return fail(UF_ERR_UNSUPPORTED, "Spearman ranks take at most 65,535 samples");
    if (n_perm < 0) return fail(UF_ERR_ARG, "n_perm < 0");
    *bytes = mantel_plan(n, method, n_perm).total;
    return UF_OK;
}

uf_status uf_mantel(const double* x, const double* y, int64_t n, int method, const int32_t* perms,
                    int64_t n_perm, int alternative, double* stat, double* p_value,
                    double* perm_stats, void* ws, size_t ws_bytes, void* stream) {
    using namespace ufm;
    if (!x || !y || !stat || !p_value) return fail(UF_ERR_ARG, "NULL argument");
    if (n < 3) return fail(UF_ERR_ARG, "need at least 3 samples");
    if (method != UF_MANTEL_PEARSON && method != UF_MANTEL_SPEARMAN)
        return fail(UF_ERR_ARG, "unknown method");
    if (method == UF_MANTEL_SPEARMAN && n > 65535)
        return fail(UF_ERR_UNSUPPORTED, "Spearman ranks take at most 65,535 samples");
    if (alternative != UF_TWO_SIDED && alternative != UF_GREATER && alternative != UF_LESS)
        return fail(UF_ERR_ARG, "unknown alternative");
    if (n_perm < 0 || (n_perm > 0 && !perms)) return fail(UF_ERR_ARG, "permutations missing");
    int dev = 0;
    uf_status st = ufh::check_device(&dev);
    if (st != UF_OK) return st;
    const MantelPlan p = mantel_plan(n, method, n_perm);
    if (!ws || ws_bytes < p.total) return fail(UF_ERR_WORKSPACE, "workspace missing or too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    double* S = reinterpret_cast<double*>(base + p.off_sq);
    double* yv = reinterpret_cast<double*>(base + p.off_y);
    double* part = reinterpret_cast<double*>(base + p.off_part);
    double* tot = reinterpret_cast<double*>(base + p.off_tot);
    double* cs = reinterpret_cast<double*>(base + p.off_cs);
    const int64_t m = p.m;
    if (n_perm > 0) {   // every permutation index must address a sample
        uint32_t* bad = reinterpret_cast<uint32_t*>(base + p.off_tot);
        UFM_HIP(hipMemsetAsync(bad, 0, 4, s));
        hipLaunchKernelGGL(k_check_perms, dim3(grid_of(n_perm * n)), dim3(256), 0, s, perms, n_perm * n,
                           n, bad);
        UFM_HIP(hipGetLastError());
        uint32_t hbad = 0;
        UFM_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
        UFM_HIP(hipStreamSynchronize(s));
        if (hbad) return fail(UF_ERR_ARG, "permutation entries must lie in [0, n)");
    }

    const double* xs = x;
    const double* ys = y;
    if (method == UF_MANTEL_SPEARMAN) {
        double* rx = reinterpret_cast<double*>(base + p.off_rx);
        double* ry = reinterpret_cast<double*>(base + p.off_ry);
        st = ranks(p, base, x, rx, s);
        if (st != UF_OK) return st;
        st = ranks(p, base, y, ry, s);
        if (st != UF_OK) return st;
        xs = rx;
        ys = ry;
    }
    // centre and scale both vectors to unit norm
    double sx = 0.0, sy = 0.0, qx = 0.0, qy = 0.0;
    if ((st = chunk_sum(xs, m, 0.0, 1, cs, s, &sx)) != UF_OK) return st;
    if ((st = chunk_sum(ys, m, 0.0, 1, cs, s, &sy)) != UF_OK) return st;
    const double mx = sx / double(m), my = sy / double(m);
    if ((st = chunk_sum(xs, m, mx, 2, cs, s, &qx)) != UF_OK) return st;
    if ((st = chunk_sum(ys, m, my, 2, cs, s, &qy)) != UF_OK) return st;
    if (!(qx > 0.0) || !(qy > 0.0)) {   // a constant matrix: r undefined, reported as 0
        *stat = 0.0;
        *p_value = 1.0;
        if (perm_stats) std::fill(perm_stats, perm_stats + n_perm, 0.0);
        return UF_OK;
    }
    const int64_t nt = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_square, dim3(unsigned(nt), unsigned(nt)), dim3(256), 0, s, xs, n, mx,
                       1.0 / std::sqrt(qx), S);
    UFM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_standardize, dim3(grid_of(m)), dim3(256), 0, s, ys, m, my, 1.0 / std::sqrt(qy),
                       yv);
    UFM_HIP(hipGetLastError());
    // observed statistic (identity) in slot n_perm, then the permutations
    const int64_t nparts = (n + kPartMax - 1) / kPartMax;
    const int64_t part_len = (n + nparts - 1) / nparts;
    const size_t lds = size_t(part_len + kRowThreads) * 8;
    static const bool attr_ok =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_perm_rows),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            int((kPartMax + kRowThreads) * 8)) == hipSuccess;
    if (!attr_ok) return fail(UF_ERR_DEVICE, "cannot enable 160 KiB of LDS for the permutation kernel");
    hipLaunchKernelGGL(k_perm_rows, dim3(unsigned(p.n_pairs)), dim3(kRowThreads), lds, s, S, yv, n,
                       static_cast<const int32_t*>(nullptr), n_perm, 1, p.n_pairs, part_len, part);
    UFM_HIP(hipGetLastError());
    for (int64_t b0 = 0; b0 < n_perm; b0 += kPB) {
        const int nb = int(std::min<int64_t>(kPB, n_perm - b0));
        hipLaunchKernelGGL(k_perm_rows, dim3(unsigned(p.n_pairs)), dim3(kRowThreads), lds, s, S, yv, n,
                           perms, b0, nb, p.n_pairs, part_len, part);
        UFM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_perm_total, dim3(unsigned(n_perm + 1)), dim3(256), 0, s, part, p.n_pairs, tot);
    UFM_HIP(hipGetLastError());
    std::vector<double> h(static_cast<size_t>(n_perm + 1));
    UFM_HIP(hipMemcpyAsync(h.data(), tot, h.size() * 8, hipMemcpyDeviceToHost, s));
    UFM_HIP(hipStreamSynchronize(s));
    const double r = h[size_t(n_perm)];
    int64_t count = 0;
    for (int64_t b = 0; b < n_perm; ++b) {
        const double v = h[size_t(b)];
        if (alternative == UF_TWO_SIDED) count += std::fabs(v) >= std::fabs(r);
        else if (alternative == UF_GREATER) count += v >= r;
        else count += v <= r;
    }
    *stat = r;
    *p_value = double(count + 1) / double(n_perm + 1);
    if (perm_stats) std::memcpy(perm_stats, h.data(), size_t(n_perm) * 8);
    return UF_OK;
}

}  // extern "C"
