// HIP kernels of the striped UniFrac library, written for gfx950 (CDNA4):
// 64-lane waves, 160 KB LDS per CU, MFMA matrix cores.
//
//   k_sample_scalars   per-sample FP64 scalars from the postorder leaf intervals
//   k_embed_nm<T>      node-major chunk of the embedding (weighted or 0/1)
//   k_embed_pres_fp8  sample-major FP8 (e4m3) 0/1 presence for the MFMA Gram path (merge)
//   k_band<T, W>       stripe-band accumulation on the vector ALUs (LDS-tiled);
//                      T = uint32_t: weighted, 32-bit fixed point, one v_sad_u32
//                      (|a - b| + acc) per update
//   k_gram_mfma        unweighted Gram product on MFMA (split-precision lengths)
//   k_finalize         FP64 division, output layouts, -d^2/2 for PCoA
//   k_rowsum_*         fixed-order two-stage row sums; k_grand_mean
#include <hip/hip_runtime.h>

#include <type_traits>

#include "uf_internal.h"

namespace ufk {
namespace {

// ----------------------------------------------------------------------------
// Embedded count of sample s on the branch at postorder position k: the sum
// of the sample's counts on the tips whose rank lies in [lo_k, hi_k).  Rows
// are sorted by tip rank and carry an exclusive prefix of the counts, so the
// count is a difference of two prefix values found by binary search.  This
// equals the postorder sum of the children's counts (a subtree is a contiguous
// run of postorder positions), exactly, in integers.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int64_t lower_bound_rank(const int32_t* __restrict__ rank, int64_t a,
                                                    int64_t b, int32_t key) {
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (rank[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a;
}

__device__ __forceinline__ int64_t embedded_count(const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ rank,
                                                  const int64_t* __restrict__ cum, int64_t s,
                                                  int32_t lo, int32_t hi) {
    const int64_t a = row_ptr[s], b = row_ptr[s + 1];
    const int64_t p1 = lower_bound_rank(rank, a, b, lo);
    const int64_t p2 = lower_bound_rank(rank, p1, b, hi);
    return cum[p2 + s] - cum[p1 + s];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ----------------------------------------------------------------------------
// Per-sample scalars, one wave per sample.
//   sw = sum_t x_t D_t / T   (= sum_v l_v u_v: every branch above t counts x_t/T)
//   w  = total length of the union of the root paths of the sample's tips
//      = sum_k D(t_k) - sum_k D(lca(t_k, t_{k+1}))  for tips in rank order,
// which is sum_v l_v a_v.  D is the root distance with FP64, FP32-rounded or
// BF16 hi+lo lengths.  Lane sums and the wave reduction run in a fixed order.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample_scalars(
    int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ rank,
    const int64_t* __restrict__ cum, const double* __restrict__ total,
    const int32_t* __restrict__ parent_pos, const int32_t* __restrict__ hi,
    const int32_t* __restrict__ tip_pos, const double* __restrict__ d64,
    const double* __restrict__ d32, const double* __restrict__ dbf, double* __restrict__ sw,
    double* __restrict__ wu, double* __restrict__ wu32, double* __restrict__ wub) {
    const int lane = threadIdx.x & 63;
    const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (s >= n) return;
    const int64_t a = row_ptr[s], b = row_ptr[s + 1];
    double x = 0.0, w = 0.0, w32 = 0.0, wb = 0.0;
    for (int64_t e = a + lane; e < b; e += 64) {
        const int32_t r = rank[e];
        const int32_t tp = tip_pos[r];
        const double cnt = double(cum[e + 1 + s] - cum[e + s]);
        x += cnt * d64[tp];
        w += d64[tp];
        w32 += d32[tp];
        wb += dbf[tp];
        if (e + 1 < b) {
            const int32_t r2 = rank[e + 1];
            int32_t p = tp;
            while (hi[p] <= r2) p = parent_pos[p];   // first ancestor covering the next tip
            w -= d64[p];
            w32 -= d32[p];
            wb -= dbf[p];
        }
    }
    x = wave_sum(x);
    w = wave_sum(w);
    w32 = wave_sum(w32);
    wb = wave_sum(wb);
    if (lane == 0) {
        sw[s] = x / total[s];
        wu[s] = w;
        wu32[s] = w32;
        wub[s] = wb;
    }
}

// ----------------------------------------------------------------------------
// Node-major embedding chunk: out[k][s] for k in [0, kc), positions k0 + k.
// A block covers 256 consecutive branches x TS samples.  The counts are found
// sample by sample (all lanes search the same row, which stays in L1), kept in
// an LDS tile, then written branch-row by branch-row (TS consecutive samples
// per row: coalesced).
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_embed_nm(
    int64_t n, int64_t k0, int64_t kc, int weighted, const int64_t* __restrict__ row_ptr,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ cum,
    const double* __restrict__ total, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const double* __restrict__ len, T* __restrict__ out) {
    constexpr int TK = 256, TS = 256 / int(sizeof(T));   // FP32: 64 samples, FP64: 32
    __shared__ T tile[TK][TS + 1];
    const int tid = threadIdx.x;
    const int64_t kb = int64_t(blockIdx.x) * TK;
    const int64_t sb = int64_t(blockIdx.y) * TS;
    const int64_t k = kb + tid;
    const bool kin = k < kc;
    int32_t lk = 0, hk = 0;
    double lv = 0.0;
    if (kin) {
        lk = lo[k0 + k];
        hk = hi[k0 + k];
        lv = len[k0 + k];
    }
    for (int j = 0; j < TS; ++j) {
        const int64_t s = sb + j;
        T v = T(0);
        if (kin && s < n) {
            const int64_t c = embedded_count(row_ptr, rank, cum, s, lk, hk);
            if (weighted) v = T(lv * (double(c) / total[s]));
            else v = c > 0 ? T(1) : T(0);
        }
        tile[tid][j] = v;
    }
    __syncthreads();
    constexpr int ROWS_PER_PASS = 256 / TS;
    for (int r = tid / TS; r < TK; r += ROWS_PER_PASS) {
        const int64_t kk = kb + r;
        const int64_t s = sb + (tid % TS);
        if (kk < kc && s < n) out[kk * n + s] = tile[r][tid % TS];
    }
}

// Sample-major presence out[s][k], k in [0, kpad): FP8 e4m3 -2.0 (0xC0) or 0,
// zero past kc.  The Gram kernel turns a byte into a BF16 operand (the byte as
// high byte: -2.0) or into a length mask (from its sign bit).  Built by
// a forward merge.  Postorder positions have
// non-decreasing hi, so along a list of ascending positions a cursor over the
// sample's tips (sorted by rank) only moves forward: it stops at the first tip
// with rank >= hi, and the branch is touched iff the last tip before it has rank
// >= lo.  Thread = sample; block = 256 samples x 64 list entries, transposed
// through LDS into 64-byte row writes.  Entries in [kc, kpad) are zero.
constexpr int kPresSamples = 256, kPresQ = 64;
__global__ __launch_bounds__(256) void k_embed_pres_fp8(
    int64_t n, int64_t k0, int64_t kc, int64_t kpad, const int64_t* __restrict__ row_ptr,
    const int32_t* __restrict__ rank, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const int32_t* __restrict__ list,
    uint8_t* __restrict__ out) {
    // rows of 64 + 16 bytes (80 bytes: 16-byte aligned, rows spread over banks)
    __shared__ __attribute__((aligned(16))) uint8_t tile[kPresSamples][kPresQ + 16];
    __shared__ int32_t qlo[kPresQ], qhi[kPresQ];
    const int tid = threadIdx.x;
    const int64_t sb = int64_t(blockIdx.x) * kPresSamples;
    const int64_t s = sb + tid;
    const int64_t nseg = kpad / kPresQ;
    for (int64_t g = blockIdx.y; g < nseg; g += gridDim.y) {
        const int64_t q0 = g * kPresQ;
        const int nq = kc - q0 <= 0 ? 0 : (kc - q0 < kPresQ ? int(kc - q0) : kPresQ);
        if (tid < nq) {
            const int64_t pos = list ? int64_t(list[k0 + q0 + tid]) : k0 + q0 + tid;
            qlo[tid] = lo[pos];
            qhi[tid] = hi[pos];
        }
        __syncthreads();
        if (s < n) {
            const int64_t a = row_ptr[s], b = row_ptr[s + 1];
            int64_t cur = a;
            int32_t last = -1;
            if (nq > 0) {
                cur = lower_bound_rank(rank, a, b, qhi[0]);
                if (cur > a) last = rank[cur - 1];
            }
            // rank of the tip at the cursor (past the row: larger than any bound), so
            // that a query which does not move the cursor loads nothing
            int32_t nxt = cur < b ? rank[cur] : 0x7fffffff;
            for (int q8 = 0; q8 < kPresQ; q8 += 8) {
                unsigned w[2] = {0u, 0u};
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q8 + u;
                    if (q < nq) {
                        const int32_t h = qhi[q];
                        while (nxt < h) {
                            last = nxt;
                            ++cur;
                            nxt = cur < b ? rank[cur] : 0x7fffffff;
                        }
                        if (last >= qlo[q]) w[u >> 2] |= 0xC0u << (8 * (u & 3));
                    }
                }
                *reinterpret_cast<uint2*>(&tile[tid][q8]) = make_uint2(w[0], w[1]);
            }
        }
        __syncthreads();
        for (int c = tid; c < kPresSamples * (kPresQ / 16); c += 256) {
            const int row = c / (kPresQ / 16), part = c % (kPresQ / 16);
            if (sb + row < n)
                *reinterpret_cast<uint4*>(out + (sb + row) * kpad + q0 + part * 16) =
                    *reinterpret_cast<const uint4*>(&tile[row][part * 16]);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Stripe-band accumulation (vector ALU).
//
// A block owns a band tile: samples i in [i0, i0+128) times stripes s in
// [s0, s0+128); the partner of (s, i) is j = (i+s+1) mod N.  For each branch
// k of the chunk it needs E[k][i] for its 128 samples and E[k][j] for the
// 255 partners.  Thread (ti, ts) keeps an 8x8 register tile: samples
// i0+8ti+a, stripes s0+8ts+b; its partners are the 15 consecutive window
// entries 8ti+8ts+(a+b).  Per branch and thread: 8+15 LDS reads for 64 pair
// updates, each update two VALU ops
//   weighted:   acc += |x_i - x_j|   with x = l * u prescaled in the embedding
//   unweighted: acc += (l * a_i) * a_j  (Gram form, one FMA; 8 extra multiplies)
// Staging: KS branches at a time, double-buffered in LDS and filled by direct
// global->LDS loads (no registers), issued for block b+1 before block b is
// computed.  Column offsets (mod N) are computed once per thread.
// Per-pair sums run over branches in postorder, independent of the tile
// position, so any stripe range reproduces the full run bit for bit.
// ----------------------------------------------------------------------------
template <typename T>
struct BandCfg;
// KS: branches per LDS stage; MS: stripes per thread (tile = 128 x 16*MS)
template <>
struct BandCfg<float> {
    static constexpr int KS = 16, MS = 8;
};
template <>
struct BandCfg<double> {
    static constexpr int KS = 8, MS = 8;
};
template <>
struct BandCfg<uint32_t> {
    static constexpr int KS = 16, MS = 16;
};

// |a - b| + c on unsigned 32-bit integers in one VALU op
__device__ __forceinline__ uint32_t sad_u32(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Hardware hands block b to XCD b mod 8.  Remap so each XCD runs a contiguous
// range of tiles (i-block fastest): neighbouring i-blocks of one stripe block
// share most of their partner window, so those loads hit the XCD's own L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n_tiles) {
    const int64_t x = b & 7, local = b >> 3;
    const int64_t per = n_tiles >> 3, rem = n_tiles & 7;
    return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// Tile l of the band grid (n_iblk sample blocks x n_sblk stripe blocks) in
// patches of 8 x 8 tiles: patches along the sample blocks first, then the next
// row of patches; inside a patch the sample block runs fastest.  With the XCD
// remap above, the blocks an XCD holds at once form about one patch, whose
// sample windows and partner windows overlap (the partner window of (b, t)
// starts at sample block b + t * (stripes per tile) / 128), so they share L2
// lines instead of each streaming its own.
constexpr int64_t kPatch = 8;
__device__ __forceinline__ void band_patch_tile(int64_t l, int64_t n_iblk, int64_t n_sblk,
                                                int64_t* ib, int64_t* sblk) {
    const int64_t ps = l / (kPatch * n_iblk);
    const int64_t rem = l - ps * kPatch * n_iblk;
    const int64_t hs = min(kPatch, n_sblk - ps * kPatch);
    const int64_t pi = rem / (kPatch * hs);
    const int64_t rem2 = rem - pi * kPatch * hs;
    const int64_t wi = min(kPatch, n_iblk - pi * kPatch);
    *ib = pi * kPatch + rem2 % wi;
    *sblk = ps * kPatch + rem2 / wi;
}

// LDS of one band tile of 16*MS stripes: two staging buffers of KS branches.
// With SWZ, rows are stored in 16-byte quads, quad q of a row at position band_swz(q):
// the two low bits are flipped by bits 3 and 4, inside each group of four
// quads.  The fragment reads of a wave start at even quads 2*DW*t (t = 0..15
// for the sample window), which fall on the same banks for t and t+4 (t and
// t+8 with 64 banks) when stored in place; with the flip, the first 8 and all
// 16 of those quads use distinct banks.  The flip never leaves a 64-dword
// segment, so each direct-to-LDS load still fills one segment, its lanes
// taking the permuted source columns.  (Without SWZ, quads stay in place: the
// batch kernel's 256-stripe tiles would need more than 256 VGPRs for the
// permuted reads' offsets, halving their occupancy.)
template <bool SWZ>
__device__ __forceinline__ int band_swz(int q) {
    return SWZ ? q ^ ((((q >> 3) ^ (q >> 4)) & 1) | ((q >> 2) & 2)) : q;
}
template <typename T>
__device__ __forceinline__ T band_from_dw(const uint32_t* d) {
    if constexpr (sizeof(T) == 8) return __hiloint2double(int(d[1]), int(d[0]));
    else if constexpr (std::is_same<T, float>::value) return __uint_as_float(d[0]);
    else return d[0];
}

template <typename T, int KS, int MS = 8>
struct BandLds {
    T wi[2][KS][kBandI];
    T wj[2][KS][kBandI + 16 * MS];
    T wl[2][KS];
};

// One band tile: samples [i0, i0+128) x stripes [s0, s0+16*MS) of a matrix with
// n samples, over the kc branches of node-major E (row stride n).  Thread
// (ti, ts) = (tid % 16, tid / 16) owns the 8 x MS register block of samples
// i0 + 8ti + [0, 8) and stripes s0 + MS*ts + [0, MS); its partners are the
// 8 + MS - 1 consecutive samples from i0 + s0 + 1 + 8ti + MS*ts.
template <typename T, bool W, int KS, int MS = 8, bool SWZ = true>
__device__ __forceinline__ void band_tile(BandLds<T, KS, MS>& L, const T* __restrict__ E,
                                          const T* __restrict__ lenk, int64_t kc, int64_t n,
                                          int64_t sb, int64_t se, int64_t i0, int64_t s0,
                                          int first, T* __restrict__ acc) {
    constexpr int I = kBandI, WJ = kBandI + 16 * MS;
    constexpr int DW = int(sizeof(T) / 4);          // dwords per element
    constexpr int EPS = 64 / DW;                    // elements per 64-dword segment
    constexpr int SEG_I = I / EPS, SEG_J = WJ / EPS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ti = tid & 15, ts = tid >> 4;

    // lane -> the dword of segment p it fills (its quad at band_swz), as
    // (element of the segment, dword of that element)
    auto seg_dword = [&](int p) { return 4 * (band_swz<SWZ>(16 * p + (lane >> 2)) - 16 * p) + (lane & 3); };
    int64_t coli[SEG_I], colj[SEG_J];
#pragma unroll
    for (int p = 0; p < SEG_I; ++p) {
        const int dl = seg_dword(p);
        coli[p] = ((i0 + p * EPS + dl / DW) % n) * DW + dl % DW;
    }
#pragma unroll
    for (int p = 0; p < SEG_J; ++p) {
        const int dl = seg_dword(p);
        colj[p] = ((i0 + s0 + 1 + p * EPS + dl / DW) % n) * DW + dl % DW;
    }
    // this thread's fragment quads: 2*DW from its 8 samples, NQJ from its 7+MS partners
    constexpr int NQI = 2 * DW, NQJ = ((7 + MS) * DW + 3) / 4;
    int oi[NQI], oj[NQJ];
#pragma unroll
    for (int q = 0; q < NQI; ++q) oi[q] = 4 * band_swz<SWZ>(2 * DW * ti + q);
#pragma unroll
    for (int q = 0; q < NQJ; ++q) oj[q] = 4 * band_swz<SWZ>((ti * 8 + ts * MS) * DW / 4 + q);

    auto stage = [&](int buf, int64_t k0) {
#pragma unroll
        for (int kk = wave; kk < KS; kk += 4) {
            const int64_t row = k0 + kk;
            uint32_t* di = reinterpret_cast<uint32_t*>(&L.wi[buf][kk][0]);
            uint32_t* dj = reinterpret_cast<uint32_t*>(&L.wj[buf][kk][0]);
            if (row < kc) {
                const uint32_t* src = reinterpret_cast<const uint32_t*>(E + row * n);
#pragma unroll
                for (int p = 0; p < SEG_I; ++p)
                    __builtin_amdgcn_global_load_lds(src + coli[p], di + p * 64, 4, 0, 0);
#pragma unroll
                for (int p = 0; p < SEG_J; ++p)
                    __builtin_amdgcn_global_load_lds(src + colj[p], dj + p * 64, 4, 0, 0);
            } else {
#pragma unroll
                for (int p = 0; p < SEG_I; ++p) di[p * 64 + lane] = 0u;
#pragma unroll
                for (int p = 0; p < SEG_J; ++p) dj[p * 64 + lane] = 0u;
            }
        }
        if (!W && tid < KS) L.wl[buf][tid] = (k0 + tid < kc) ? lenk[k0 + tid] : T(0);
    };

    T r[8][MS];
#pragma unroll
    for (int b = 0; b < MS; ++b) {
        const int64_t s = s0 + ts * MS + b;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int64_t i = i0 + ti * 8 + a;
            r[a][b] = (!first && s < se && i < n) ? acc[(s - sb) * n + i] : T(0);
        }
    }

    // FP64 tiles: one branch at a time (two in flight would take them past 256
    // VGPRs and halve their occupancy)
    constexpr int UNR = sizeof(T) == 8 ? 1 : 2;
    const int64_t nblk = (kc + KS - 1) / KS;
    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int64_t blk = 0; blk < nblk; ++blk) {
        const int cur = int(blk & 1);
        if (blk + 1 < nblk) stage(cur ^ 1, (blk + 1) * KS);
#pragma unroll UNR
        for (int kk = 0; kk < KS; ++kk) {
            const uint32_t* rwi = reinterpret_cast<const uint32_t*>(&L.wi[cur][kk][0]);
            const uint32_t* rwj = reinterpret_cast<const uint32_t*>(&L.wj[cur][kk][0]);
            uint32_t bi[4 * NQI], bj[4 * NQJ];
#pragma unroll
            for (int q = 0; q < NQI; ++q) *reinterpret_cast<uint4*>(bi + 4 * q) = *reinterpret_cast<const uint4*>(rwi + oi[q]);
#pragma unroll
            for (int q = 0; q < NQJ; ++q) *reinterpret_cast<uint4*>(bj + 4 * q) = *reinterpret_cast<const uint4*>(rwj + oj[q]);
            T xi[8], xj[8 + MS];
#pragma unroll
            for (int a = 0; a < 8; ++a) xi[a] = band_from_dw<T>(bi + a * DW);
#pragma unroll
            for (int c = 0; c < 7 + MS; ++c) xj[c] = band_from_dw<T>(bj + c * DW);
            if constexpr (std::is_same<T, uint32_t>::value) {
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int b = 0; b < MS; ++b) r[a][b] = sad_u32(xi[a], xj[a + b], r[a][b]);
            } else if constexpr (W) {
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int b = 0; b < MS; ++b) r[a][b] += fabs(xi[a] - xj[a + b]);
            } else {
                const T l = L.wl[cur][kk];
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const T li = l * xi[a];
#pragma unroll
                    for (int b = 0; b < MS; ++b) r[a][b] = fma(li, xj[a + b], r[a][b]);
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

#pragma unroll
    for (int b = 0; b < MS; ++b) {
        const int64_t s = s0 + ts * MS + b;
        if (s >= se) continue;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int64_t i = i0 + ti * 8 + a;
            if (i < n) acc[(s - sb) * n + i] = r[a][b];
        }
    }
}

template <typename T, bool W>
__global__ __launch_bounds__(256) void k_band(const T* __restrict__ E,
                                              const T* __restrict__ lenk, int64_t kc,
                                              int64_t n, int64_t sb, int64_t se, int64_t n_iblk,
                                              int first, T* __restrict__ acc) {
    constexpr int KS = BandCfg<T>::KS, MS = BandCfg<T>::MS, TS = 16 * MS;
    __shared__ __attribute__((aligned(16))) BandLds<T, KS, MS> L;
    const int64_t n_sblk = (se - sb + TS - 1) / TS;
    const int64_t n_tiles = n_iblk * n_sblk;
    int64_t ib = 0, sblk = 0;
    band_patch_tile(xcd_tile(blockIdx.x, n_tiles), n_iblk, n_sblk, &ib, &sblk);
    const int64_t i0 = ib * kBandI;
    const int64_t s0 = sb + sblk * TS;
    band_tile<T, W, KS, MS, true>(L, E, lenk, kc, n, sb, se, i0, s0, first, acc);
}

// ----------------------------------------------------------------------------
// Unweighted Gram product on MFMA: G = P diag(l) P^T with P the 0/1 presence
// and l = l_hi + l_lo, both BF16; v_mfma_f32_32x32x16_bf16 accumulates in FP32.
// Block = 8 waves in 2x4, tile 256x256 (wave 128x64 = 4x2 MFMA blocks of 32x32),
// K step 128.  Presence bytes go through LDS as they are (rows of 128 + 16 bytes)
// and become MFMA operands in registers:
// * A (rows i): the byte as the high byte of a BF16 lane, -2.0 where present;
// * B (rows j): the byte's sign bit spread over a BF16 lane, as a mask of the
//   K step's l_hi and l_lo (staged in LDS, read as broadcasts).
// So the MFMAs sum -2 l over the shared branches (exactly twice the negated
// sum in FP32) and the epilogue scales by -1/2.  The contraction is free to
// order K within a step: the MFMA of sub-step s (0..7) takes, from lane group
// g (lanes 32g..32g+31), the positions 64g + 8s + [0, 8), so that one 16-byte
// LDS read serves two sub-steps.  Global loads run one K step ahead of the
// MFMAs, through registers into two LDS stages (one barrier per K step).
// Only upper-triangle tiles (bi <= bj) that hold a pair of the stripe range
// run; each pair i<j of the range is written to its stripe-major slot.
// ----------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bool tile_in_range(int64_t i0, int64_t j0, int64_t n, int64_t sb,
                                              int64_t se) {
    const int64_t S = n / 2;
    const int64_t imax = min(i0 + kGramT, n) - 1;
    const int64_t jmax = min(j0 + kGramT, n) - 1;
    const int64_t dlo = max<int64_t>(1, j0 - imax);
    const int64_t dhi = jmax - i0;
    if (dhi < dlo) return false;
    // partner offset d = j - i; stripe d-1 if d <= S, else n-d-1
    const int64_t a1 = max(dlo, sb + 1), b1 = min(dhi, min(se, S));
    const int64_t a2 = max(dlo, max(n - se, S + 1)), b2 = min(dhi, n - 1 - sb);
    return a1 <= b1 || a2 <= b2;
}

// Block -> tile of the Gram kernel.  The upper-triangle tiles (bi <= bj) are
// numbered super-tile by super-tile: G x G super-tiles, super-row-major, the
// diagonal super-tile first in its super-row, tiles row-major inside.  Blocks are
// dealt to the 8 XCDs round-robin, and XCD x takes the x-th eighth of that order:
// its CUs walk neighbouring super-tiles together, reading each row and column
// panel into the XCD's L2 about once per super-tile, and every XCD gets the same
// number of tiles.  Returns false for slots past the last tile.
constexpr int kGramGroup = 8;

__device__ __forceinline__ bool gram_tile_of(int64_t b, int64_t nblk, int64_t& bi, int64_t& bj) {
    constexpr int64_t G = kGramGroup;
    const int64_t L = nblk * (nblk + 1) / 2;
    const int64_t per = (L + 7) / 8;
    const int64_t k = b >> 3;
    int64_t v = (b & 7) * per + k;
    if (k >= per || v >= L) return false;
    int64_t r0 = 0;                              // first row of the super-row
    for (;;) {
        const int64_t r = min(G, nblk - r0);     // rows of the super-row
        const int64_t cnt = r * (r + 1) / 2 + r * (nblk - r0 - r);
        if (v < cnt) {
            const int64_t diag = r * (r + 1) / 2;
            if (v < diag) {                      // diagonal super-tile: row a holds r - a tiles
                int64_t a = 0;
                while (v >= r - a) {
                    v -= r - a;
                    ++a;
                }
                bi = r0 + a;
                bj = r0 + a + v;
            } else {                             // off-diagonal super-tiles of r x G tiles (the last may be narrower)
                v -= diag;
                const int64_t c0 = r0 + r + (v / (r * G)) * G;   // first column of the super-tile
                const int64_t c = min(G, nblk - c0);
                const int64_t w = v % (r * G);
                bi = r0 + w / c;
                bj = c0 + w % c;
            }
            return true;
        }
        v -= cnt;
        r0 += r;
    }
}

__global__ __launch_bounds__(512, 1) void k_gram_mfma(const uint8_t* __restrict__ P,
                                                      const uint16_t* __restrict__ hiv,
                                                      const uint16_t* __restrict__ lov,
                                                      int64_t kpad, int64_t n, int64_t sb,
                                                      int64_t se, int first,
                                                      float* __restrict__ acc) {
    constexpr int T = kGramT, KT = kGramK, LD = KT + 16;
    static_assert(KT % 32 == 0, "the fragment layout below assumes a K step of 32m");
    int64_t bi, bj;
    if (!gram_tile_of(blockIdx.x, (n + T - 1) / T, bi, bj)) return;
    const int64_t i0 = bi * T, j0 = bj * T;
    if (!tile_in_range(i0, j0, n, sb, se)) return;

    // two LDS stages of the presence bytes of rows i (A) and j (B), and of the
    // step's lengths (l_hi in [0, KT), l_lo in [KT, 2 KT))
    __shared__ __attribute__((aligned(16))) uint8_t As[2][T * LD];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[2][T * LD];
    __shared__ __attribute__((aligned(16))) uint16_t Ls[2][2 * KT];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = wave & 1, wj = wave >> 1;     // wave tile: rows wi*128 + [0,128), cols wj*64 + [0,64)
    const int lg = lane >> 5;                    // lane group: K positions (KT/2)*lg + [0, KT/2) of a step
    floatx16 c[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) c[x][y][r] = 0.0f;

    // staging: row (tid mod 256) of the tile, bytes (KT/2) * (tid / 256) + [0, KT/2)
    // of the step (eight consecutive rows fill all LDS banks: the row pitch is an
    // odd multiple of 16 bytes); and 16 bytes of the step's lengths (every thread
    // loads them, the first KT/4 threads store them)
    const int lrow = tid & (T - 1);
    const int lseg = (tid >> 8) * (KT / 2);
    constexpr int NL = KT / 4;                  // 16-byte pieces of the step's lengths
    const int lq = tid & (NL - 1);
    const uint16_t* lsrc = (lq < NL / 2 ? hiv : lov) + 8 * (lq & (NL / 2 - 1));
    // rows past n read row n-1: their products land in rows/columns >= n, which
    // the epilogue drops
    const int64_t ci = i0 + lrow < n ? i0 + lrow : n - 1;
    const int64_t cj = j0 + lrow < n ? j0 + lrow : n - 1;

    constexpr int NV = KT / 32;                 // 16-byte pieces per staged row half
    static_assert(NV == 4, "named staging registers below");
    struct Regs {
        uint4 a0, a1, a2, a3, b0, b1, b2, b3, l;
    };
    // (Regs move by value: a reference would leave them in memory, which the
    // compiler may place in LDS and wait on at once)
    auto fetch = [&](int64_t k0) -> Regs {
        Regs R;
        const uint4* pa = reinterpret_cast<const uint4*>(P + ci * kpad + k0 + lseg);
        const uint4* pb = reinterpret_cast<const uint4*>(P + cj * kpad + k0 + lseg);
        R.a0 = pa[0];
        R.a1 = pa[1];
        R.a2 = pa[2];
        R.a3 = pa[3];
        R.b0 = pb[0];
        R.b1 = pb[1];
        R.b2 = pb[2];
        R.b3 = pb[3];
        R.l = *reinterpret_cast<const uint4*>(lsrc + k0);
        return R;
    };
    auto stash = [&](const Regs R, int buf) {
        uint4* ad = reinterpret_cast<uint4*>(As[buf] + lrow * LD + lseg);
        uint4* bd = reinterpret_cast<uint4*>(Bs[buf] + lrow * LD + lseg);
        ad[0] = R.a0;
        ad[1] = R.a1;
        ad[2] = R.a2;
        ad[3] = R.a3;
        bd[0] = R.b0;
        bd[1] = R.b1;
        bd[2] = R.b2;
        bd[3] = R.b3;
        if (tid < NL) reinterpret_cast<uint4*>(Ls[buf])[lq] = R.l;
    };
    // v_perm_b32 selectors over {S0, S1} (S1 = bytes 0-3, S0 = bytes 4-7):
    // 12 -> 0x00; 8, 9, 10, 11 -> sign bit of byte 1, 3, 5, 7 spread over a byte
    constexpr unsigned kSelA0 = 0x010C000Cu;   // bytes 0, 1 -> high bytes of two BF16 lanes
    constexpr unsigned kSelA1 = 0x030C020Cu;   // bytes 2, 3
    constexpr unsigned kSelM0 = 0x08080A0Au;   // S0 = x << 8: masks of bytes 0, 1
    constexpr unsigned kSelM1 = 0x09090B0Bu;   // masks of bytes 2, 3
    auto compute = [&](int buf) {
#pragma unroll
        for (int h = 0; h < KT / 32; ++h) {
            // 16 bytes per fragment row: positions (KT/2)*lg + 16*h + [0, 16), i.e.
            // sub-steps 2h and 2h+1
            uint4 ra[4], rb[2];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int row = wi * 128 + x * 32 + (lane & 31);
                ra[x] = *reinterpret_cast<const uint4*>(As[buf] + row * LD + (KT / 2) * lg + 16 * h);
            }
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int col = wj * 64 + y * 32 + (lane & 31);
                rb[y] = *reinterpret_cast<const uint4*>(Bs[buf] + col * LD + (KT / 2) * lg + 16 * h);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int kq = (KT / 2) * lg + 16 * h + 8 * q;
                const uint4 lh = *reinterpret_cast<const uint4*>(Ls[buf] + kq);
                const uint4 ll = *reinterpret_cast<const uint4*>(Ls[buf] + KT + kq);
                const unsigned lhw[4] = {lh.x, lh.y, lh.z, lh.w};
                const unsigned llw[4] = {ll.x, ll.y, ll.z, ll.w};
                bf16x8 fa[4], fh[2], fl[2];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const unsigned u0 = q ? ra[x].z : ra[x].x, u1 = q ? ra[x].w : ra[x].y;
                    unsigned w[4];
                    w[0] = __builtin_amdgcn_perm(0u, u0, kSelA0);
                    w[1] = __builtin_amdgcn_perm(0u, u0, kSelA1);
                    w[2] = __builtin_amdgcn_perm(0u, u1, kSelA0);
                    w[3] = __builtin_amdgcn_perm(0u, u1, kSelA1);
                    __builtin_memcpy(&fa[x], w, sizeof(w));
                }
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const unsigned u0 = q ? rb[y].z : rb[y].x, u1 = q ? rb[y].w : rb[y].y;
                    unsigned m[4], wh[4], wl[4];
                    m[0] = __builtin_amdgcn_perm(u0 << 8, u0, kSelM0);
                    m[1] = __builtin_amdgcn_perm(u0 << 8, u0, kSelM1);
                    m[2] = __builtin_amdgcn_perm(u1 << 8, u1, kSelM0);
                    m[3] = __builtin_amdgcn_perm(u1 << 8, u1, kSelM1);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        wh[e] = m[e] & lhw[e];
                        wl[e] = m[e] & llw[e];
                    }
                    __builtin_memcpy(&fh[y], wh, sizeof(wh));
                    __builtin_memcpy(&fl[y], wl, sizeof(wl));
                }
                // the hi products of all eight blocks, then the lo products, so that
                // no MFMA waits on the one before it
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        c[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fh[y], c[x][y], 0, 0, 0);
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        c[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fl[y], c[x][y], 0, 0, 0);
            }
        }
    };

    // K step t: registers of step t (fetched during step t-1) go to LDS stage
    // t mod 2, the registers are refilled with step t+1, then the MFMAs of step t
    // run.  The stage written at step t was last read by the MFMAs of step t-2,
    // which every wave finished before the barrier of step t-1.  kpad is a
    // multiple of two steps, so both halves of the loop body always run; the
    // fetch past the end re-reads the last step (kept unconditional so that the
    // compiler's wait counts stay exact) and is never stored.
    const int64_t nk = kpad / KT;
    const int64_t klast = kpad - KT;
    Regs R = fetch(0);
    for (int64_t t = 0; t < nk; t += 2) {
        stash(R, 0);
        R = fetch(min((t + 1) * KT, klast));
        __syncthreads();
        compute(0);
        stash(R, 1);
        R = fetch(min((t + 2) * KT, klast));
        __syncthreads();
        compute(1);
    }

    // epilogue: D[i][j] for 32x32 block: lane holds column lane%32 and rows
    // 8*(r/4) + 4*(lane/32) + r%4 for r = 0..15
    const int64_t S = n / 2;
    const bool even = (n & 1) == 0;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + wi * 128 + x * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t j = j0 + wj * 64 + y * 32 + (lane & 31);
                if (!(i < j && j < n)) continue;
                const int64_t d = j - i;
                const float g = -0.5f * c[x][y][r];
                int64_t s, slot;
                if (d <= S) { s = d - 1; slot = i; }
                else { s = n - d - 1; slot = j; }
                if (s < sb || s >= se) continue;
                const int64_t idx = (s - sb) * n + slot;
                acc[idx] = first ? g : acc[idx] + g;
                if (even && d == S) {  // the last stripe of an even N holds the pair twice
                    const int64_t idx2 = (s - sb) * n + j;
                    acc[idx2] = first ? g : acc[idx2] + g;
                }
            }
}

// ----------------------------------------------------------------------------
// Finalize: distance from the accumulator of (s, i), output layout, -d^2/2.
// ----------------------------------------------------------------------------
// With the sparse-aware split (split_m != NULL) the weighted numerator adds the
// exact fixed-point part sigma_i + sigma_j - 2 M_ij (2^-40 units) of the branches
// outside the dense set.
//
// A block takes tiles of 64 stripes x 64 samples.  Distances are computed with
// lanes along samples (coalesced accumulator reads and stripe-major writes);
// for the condensed layout the tile goes through LDS and out in two sweeps:
// pairs (i, i+s+1) with i+s+1 < n sit in condensed row i at column offset s, so
// a run over s is contiguous; wrapped pairs (i+s+1-n, i) sit in row i+s+1-n, so
// a run over i along an anti-diagonal (i+s fixed) is contiguous.  Lane l of
// group g takes diagonal g or g+64 of the tile, so every lane has an element
// and a 64-lane store covers at most two runs.
constexpr int kFinT = 64;

// Inputs of one (stripe, sample) element, loaded ahead of the arithmetic.
template <typename A>
struct FinIn {
    A acc;                         // dense accumulator (unscaled)
    unsigned long long m;          // split: exact pair sum in the split's unit
    unsigned long long sg_i, sg_j; // weighted split: sigma of both samples
    double sc_i, sc_j;             // per-sample scalars
};

// Loads only (no arithmetic on the loaded values, so that the loads of several
// elements stay in flight together).  Indices must be in range.
template <typename A>
__device__ __forceinline__ FinIn<A> final_inputs(const A* __restrict__ acc,
                                                 const double* __restrict__ scal, int64_t n,
                                                 int64_t sb, int64_t s, int64_t i, int64_t j,
                                                 const unsigned long long* __restrict__ sigma) {
    FinIn<A> f;
    f.acc = acc[(s - sb) * n + i];
    f.m = 0ull;   // the split's sum comes from the LDS stage
    f.sg_i = sigma ? sigma[i] : 0ull;
    f.sg_j = sigma ? sigma[j] : 0ull;
    f.sc_i = scal[i];
    f.sc_j = scal[j];
    return f;
}

template <typename A>
__device__ __forceinline__ double final_distance(int kind, const FinIn<A>& f, double acc_scale,
                                                 bool split, double split_unit) {
    double num = double(f.acc) * acc_scale;
    if (split) {
        if (kind == 0) {
            const long long r = (long long)(f.sg_i + f.sg_j - 2ull * f.m);
            num += double(r) * split_unit;
        } else {
            num += double(f.m) * split_unit;
        }
    }
    if (kind == 0) {   // a sum of |x - y| over the sum of x + y: no clamp needed
        const double den = f.sc_i + f.sc_j;
        return den > 0.0 ? num / den : 0.0;
    }
    // Gram form: the differences w_i + w_j - 2G and w_i + w_j - G can round past the
    // ends of [0, 1] (d(a, a) = 0 in exact arithmetic), so the result is clamped
    const double sum = f.sc_i + f.sc_j;
    const double orr = sum - num;
    const double xr = sum - 2.0 * num;
    const double d = orr > 0.0 ? xr / orr : 0.0;
    return fmin(fmax(d, 0.0), 1.0);
}

template <typename A>
__global__ __launch_bounds__(256) void k_finalize(int kind, const A* __restrict__ acc,
                                                  double acc_scale,
                                                  const double* __restrict__ scal, int64_t n,
                                                  int64_t sb, int64_t se, int layout, int out_f32,
                                                  void* __restrict__ out, double* __restrict__ q,
                                                  const unsigned long long* __restrict__ split_m,
                                                  const unsigned long long* __restrict__ sigma,
                                                  double split_unit) {
    // row pitch 66 doubles: the run over s (step 66) has 4-way and the
    // anti-diagonal run (step -65) no LDS bank conflicts
    __shared__ double tile[kFinT][kFinT + 2];
    const int tid = threadIdx.x;
    const int64_t i0 = int64_t(blockIdx.x) * kFinT;
    const bool even = (n & 1) == 0;
    const bool condensed = layout != UF_STRIPES;
    const int64_t n_tiles = (se - sb + kFinT - 1) / kFinT;
    auto put = [&](int64_t idx, double d) {
        if (out_f32) static_cast<float*>(out)[idx] = float(d);
        else static_cast<double*>(out)[idx] = d;
    };
    for (int64_t t = blockIdx.y; t < n_tiles; t += gridDim.y) {
        const int64_t s0 = sb + t * kFinT;
        const int li = tid & 63;
        const int64_t i = i0 + li;
        // the thread's 16 elements in two batches of 8, all loads of a batch in
        // flight before its arithmetic
        // (elements outside the range load from a clamped in-range element and are
        // not stored)
        const int64_t ic = i < n ? i : n - 1;
        if (split_m) {
            // the split's sums are sample-major: stage the tile's 64 rows of 64
            // stripes through LDS with coalesced row reads (each element lands in
            // the cell its distance later takes, read back by the same thread)
            __syncthreads();
            const int64_t sr = se - sb;
            const int cs = tid & 63;
            const int64_t scs = s0 + cs < se ? s0 + cs : se - 1;
#pragma unroll 4
            for (int r = tid >> 6; r < kFinT; r += 4) {
                const int64_t ir = i0 + r < n ? i0 + r : n - 1;
                tile[cs][r] = __longlong_as_double((long long)split_m[ir * sr + (scs - sb)]);
            }
            __syncthreads();
        }
        for (int half = 0; half < 2; ++half) {
            FinIn<A> in[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int ls = (tid >> 6) + 4 * (8 * half + u);
                const int64_t sc = s0 + ls < se ? s0 + ls : se - 1;
                in[u] = final_inputs(acc, scal, n, sb, sc, ic, (ic + sc + 1) % n, sigma);
                if (split_m) in[u].m = (unsigned long long)__double_as_longlong(tile[ls][li]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int ls = (tid >> 6) + 4 * (8 * half + u);
                const int64_t s = s0 + ls;
                if (s >= se || i >= n) continue;
                const double d = final_distance(kind, in[u], acc_scale, split_m != nullptr,
                                                split_unit);
                if (q) q[(s - sb) * n + i] = -0.5 * d * d;
                if (condensed) tile[ls][li] = d;
                else put((s - sb) * n + i, d);
            }
        }
        if (!condensed) continue;
        __syncthreads();
        for (int e = tid; e < kFinT * kFinT; e += 256) {
            const int li = e / kFinT, ls = e % kFinT;
            const int64_t s = s0 + ls, i = i0 + li;
            if (s >= se || i >= n || i + s + 1 >= n) continue;
            put(i * n - i * (i + 1) / 2 + s, tile[ls][li]);
        }
        for (int e = tid; e < kFinT * kFinT; e += 256) {
            const int g = e / kFinT, li = e % kFinT;
            const int ls = (g - li) & (kFinT - 1);
            const int64_t s = s0 + ls, i = i0 + li;
            if (s >= se || i >= n || i + s + 1 < n) continue;
            if (even && s == n / 2 - 1 && i >= n / 2) continue;   // the pair's other copy
            const int64_t jw = i + s + 1 - n;
            put(jw * n - jw * (jw + 1) / 2 + (i - jw - 1), tile[ls][li]);
        }
        __syncthreads();
    }
}

// Row sums, stage 1: part p sums stripes [sb + 256p, sb + 256(p+1)) for sample i,
// taking each distinct pair once: (i, i+s+1) at column i and (i-s-1, i) at
// column i-s-1 (skipped on the duplicated last stripe of an even N).
__global__ __launch_bounds__(256) void k_rowsum_part(const double* __restrict__ q, int64_t n,
                                                     int64_t sb, int64_t se,
                                                     double* __restrict__ part) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t p = blockIdx.y;
    const int64_t a = sb + p * 256, b = min(se, a + 256);
    const bool even = (n & 1) == 0;
    double acc = 0.0;
    for (int64_t s = a; s < b; ++s) {
        const double* row = q + (s - sb) * n;
        acc += row[i];
        if (!(even && s == n / 2 - 1)) {
            int64_t jj = (i - s - 1) % n;
            if (jj < 0) jj += n;
            acc += row[jj];
        }
    }
    part[p * n + i] = acc;
}

__global__ __launch_bounds__(256) void k_rowsum_final(const double* __restrict__ part,
                                                      int64_t n_parts, int64_t n, double scale,
                                                      double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t p = 0; p < n_parts; ++p) acc += part[p * n + i];
    out[i] = acc * scale;
}

__global__ __launch_bounds__(256) void k_grand_mean(const double* __restrict__ rm, int64_t n,
                                                    double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += rm[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / double(n);
}

// ----------------------------------------------------------------------------
// Batches: many tables on one tree.
// ----------------------------------------------------------------------------
// Node-major chunk of every table; global sample g belongs to table tab_of[g].
__global__ __launch_bounds__(256) void k_embed_batch_f32(
    int64_t n_all, int64_t k0, int64_t kc, const BatchTable* __restrict__ tabs,
    const int32_t* __restrict__ tab_of, const int64_t* __restrict__ row_ptr,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ cum,
    const double* __restrict__ total, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const double* __restrict__ len, float* __restrict__ out) {
    constexpr int TK = 256, TS = 64;
    __shared__ float tile[TK][TS + 1];
    const int tid = threadIdx.x;
    const int64_t kb = int64_t(blockIdx.x) * TK;
    const int64_t gb = int64_t(blockIdx.y) * TS;
    const int64_t k = kb + tid;
    const bool kin = k < kc;
    int32_t lk = 0, hk = 0;
    double lv = 0.0;
    if (kin) {
        lk = lo[k0 + k];
        hk = hi[k0 + k];
        lv = len[k0 + k];
    }
    for (int j = 0; j < TS; ++j) {
        const int64_t g = gb + j;
        float v = 0.0f;
        if (kin && g < n_all) {
            const int64_t c = embedded_count(row_ptr, rank, cum, g, lk, hk);
            v = float(lv * (double(c) / total[g]));
        }
        tile[tid][j] = v;
    }
    __syncthreads();
    for (int r = tid / TS; r < TK; r += 256 / TS) {
        const int64_t kk = kb + r;
        const int64_t g = gb + (tid % TS);
        if (kk < kc && g < n_all) {
            const BatchTable t = tabs[tab_of[g]];
            out[t.e_off + kk * t.n + (g - t.off)] = tile[r][tid % TS];
        }
    }
}

// Persistent band kernel: the grid stays resident and pulls (table, tile)
// items from per-XCD queues (block b runs on XCD b mod 8 and drains queue
// b mod 8 first, then steals from the others).  Every queue is finite, so
// every block exits once all queues are exhausted.
template <int KS, int MS>
__global__ __launch_bounds__(256) void k_band_persistent_f32(
    const float* __restrict__ E, const BatchTable* __restrict__ tabs,
    const int2* __restrict__ items, const int64_t* __restrict__ qbeg,
    const int64_t* __restrict__ qend, unsigned* __restrict__ counters, int64_t kc, int first,
    float* __restrict__ acc) {
    __shared__ __attribute__((aligned(16))) BandLds<float, KS, MS> L;
    __shared__ int64_t next_item;
    const int xcd = int(blockIdx.x & 7);
    for (int q = 0; q < 8; ++q) {
        const int queue = (xcd + q) & 7;
        const int64_t end = qend[queue];
        for (;;) {
            if (threadIdx.x == 0) next_item = qbeg[queue] + int64_t(atomicAdd(&counters[queue], 1u));
            __syncthreads();
            const int64_t item = next_item;
            __syncthreads();
            if (item >= end) break;
            const int2 it = items[item];
            const BatchTable t = tabs[it.x];
            const int64_t i0 = (int64_t(it.y) % t.n_iblk) * kBandI;
            const int64_t s0 = (int64_t(it.y) / t.n_iblk) * (16 * MS);
            band_tile<float, true, KS, MS, false>(L, E + t.e_off, nullptr, kc, t.n, 0, t.n / 2, i0, s0,
                                           first, acc + t.acc_off);
        }
    }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

inline unsigned grid_y(int64_t v) { return unsigned(v < 65535 ? (v < 1 ? 1 : v) : 65535); }

}  // namespace

// ============================================================================
// launchers
// ============================================================================
hipError_t sample_scalars(const uf_embedding& e, const int32_t* parent_pos, const int32_t* tip_pos,
                          const double* d64, const double* d32, const double* dbf,
                          hipStream_t st) {
    const unsigned blocks = unsigned((e.n + 3) / 4);
    hipLaunchKernelGGL(k_sample_scalars, dim3(blocks), dim3(256), 0, st, e.n, e.row_ptr, e.rank,
                       e.cum, e.total, parent_pos, e.hi, tip_pos, d64, d32, dbf, e.sw, e.wu,
                       e.wu32, e.wub);
    return hipGetLastError();
}

template <typename T>
static hipError_t embed_nm(const uf_embedding& e, int64_t k0, int64_t kc, int weighted, T* out,
                           hipStream_t st) {
    if (kc <= 0 || e.n <= 0) return hipSuccess;
    constexpr int TS = 256 / int(sizeof(T));
    const int64_t gy = (e.n + TS - 1) / TS;
    if (gy > 65535) return hipErrorInvalidValue;
    dim3 grid(unsigned((kc + 255) / 256), unsigned(gy));
    hipLaunchKernelGGL(k_embed_nm<T>, grid, dim3(256), 0, st, e.n, k0, kc, weighted, e.row_ptr,
                       e.rank, e.cum, e.total, e.lo, e.hi, e.len, out);
    return hipGetLastError();
}

hipError_t embed_node_major_f64(const uf_embedding& e, int64_t k0, int64_t kc, int weighted,
                                double* out, hipStream_t st) {
    return embed_nm<double>(e, k0, kc, weighted, out, st);
}
hipError_t embed_node_major_f32(const uf_embedding& e, int64_t k0, int64_t kc, int weighted,
                                float* out, hipStream_t st) {
    return embed_nm<float>(e, k0, kc, weighted, out, st);
}

hipError_t embed_presence_fp8(const uf_embedding& e, int64_t k0, int64_t kc, int64_t kpad,
                              uint8_t* out, hipStream_t st, const int32_t* list) {
    if (kpad <= 0 || e.n <= 0) return hipSuccess;
    if (kpad % kPresQ != 0) return hipErrorInvalidValue;
    const int64_t gx = (e.n + kPresSamples - 1) / kPresSamples;
    const int64_t gy = std::min<int64_t>(kpad / kPresQ, 65535);
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_embed_pres_fp8, dim3(unsigned(gx), unsigned(gy)), dim3(256), 0, st, e.n,
                       k0, kc, kpad, e.row_ptr, e.rank, e.lo, e.hi, list, out);
    return hipGetLastError();
}

template <typename T>
static hipError_t band(const T* E, const T* lenk, int64_t kc, int64_t n, int64_t sb, int64_t se,
                       int weighted, int first, T* acc, hipStream_t st) {
    if (se <= sb || n <= 0) return hipSuccess;
    constexpr int64_t TS = 16 * BandCfg<T>::MS;
    const int64_t n_iblk = (n + kBandI - 1) / kBandI;
    const int64_t n_tiles = n_iblk * ((se - sb + TS - 1) / TS);
    if (n_tiles > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid{unsigned(n_tiles), 1u, 1u};
    if (weighted)
        hipLaunchKernelGGL((k_band<T, true>), grid, dim3(256), 0, st, E, lenk, kc, n, sb, se,
                           n_iblk, first, acc);
    else
        hipLaunchKernelGGL((k_band<T, false>), grid, dim3(256), 0, st, E, lenk, kc, n, sb, se,
                           n_iblk, first, acc);
    return hipGetLastError();
}

hipError_t band_f64(const double* E, const double* lenk, int64_t kc, int64_t n, int64_t sb,
                    int64_t se, int weighted, int first, double* acc, hipStream_t st) {
    return band<double>(E, lenk, kc, n, sb, se, weighted, first, acc, st);
}
hipError_t band_f32(const float* E, const float* lenk, int64_t kc, int64_t n, int64_t sb,
                    int64_t se, int weighted, int first, float* acc, hipStream_t st) {
    return band<float>(E, lenk, kc, n, sb, se, weighted, first, acc, st);
}

hipError_t band_u32(const uint32_t* E, int64_t kc, int64_t n, int64_t sb, int64_t se, int first,
                    uint32_t* acc, hipStream_t st) {
    if (se <= sb || n <= 0) return hipSuccess;
    constexpr int64_t TS = 16 * BandCfg<uint32_t>::MS;
    const int64_t n_iblk = (n + kBandI - 1) / kBandI;
    const int64_t n_tiles = n_iblk * ((se - sb + TS - 1) / TS);
    if (n_tiles > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid{unsigned(n_tiles), 1u, 1u};
    hipLaunchKernelGGL((k_band<uint32_t, true>), grid, dim3(256), 0, st, E, nullptr, kc, n, sb, se,
                       n_iblk, first, acc);
    return hipGetLastError();
}

hipError_t gram_mfma(const uint8_t* P, const uint16_t* hi, const uint16_t* lo, int64_t kpad,
                     int64_t n, int64_t sb, int64_t se, int first, float* acc, hipStream_t st) {
    if (se <= sb || n <= 0) return hipSuccess;
    const int64_t nblk = (n + kGramT - 1) / kGramT;
    if (nblk > 65535 || kpad <= 0 || (kpad % kGramKPad) != 0) return hipErrorInvalidValue;
    const int64_t blocks = 8 * ((nblk * (nblk + 1) / 2 + 7) / 8);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid{unsigned(blocks), 1u, 1u};
    hipLaunchKernelGGL(k_gram_mfma, grid, dim3(512), 0, st, P, hi, lo, kpad, n, sb, se, first,
                       acc);
    return hipGetLastError();
}

hipError_t finalize(int kind, const void* acc, int acc_type, double acc_scale, const double* scal,
                    int64_t n, int64_t sb, int64_t se, int layout, int out_f32, void* out, double* q,
                    hipStream_t st, const unsigned long long* split_m,
                    const unsigned long long* sigma, double split_unit) {
    if (se <= sb || n <= 0) return hipSuccess;
    const int64_t gx = (n + kFinT - 1) / kFinT;
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(unsigned(gx), grid_y((se - sb + kFinT - 1) / kFinT));
    if (acc_type == kAccF64)
        hipLaunchKernelGGL(k_finalize<double>, grid, dim3(256), 0, st, kind,
                           static_cast<const double*>(acc), acc_scale, scal, n, sb, se, layout,
                           out_f32, out, q, split_m, sigma, split_unit);
    else if (acc_type == kAccU32)
        hipLaunchKernelGGL(k_finalize<uint32_t>, grid, dim3(256), 0, st, kind,
                           static_cast<const uint32_t*>(acc), acc_scale, scal, n, sb, se, layout,
                           out_f32, out, q, split_m, sigma, split_unit);
    else
        hipLaunchKernelGGL(k_finalize<float>, grid, dim3(256), 0, st, kind,
                           static_cast<const float*>(acc), acc_scale, scal, n, sb, se, layout,
                           out_f32, out, q, split_m, sigma, split_unit);
    return hipGetLastError();
}

hipError_t row_sums(const double* q, int64_t n, int64_t sb, int64_t se, double* partial,
                    int64_t n_parts, double scale, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n_parts > 65535) return hipErrorInvalidValue;
    dim3 g1(unsigned((n + 255) / 256), unsigned(n_parts));
    hipLaunchKernelGGL(k_rowsum_part, g1, dim3(256), 0, st, q, n, sb, se, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowsum_final, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, partial,
                       n_parts, n, scale, out);
    return hipGetLastError();
}

hipError_t grand_mean(const double* row_means, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_grand_mean, dim3(1), dim3(256), 0, st, row_means, n, out);
    return hipGetLastError();
}

hipError_t embed_batch_f32(const uf_embedding& e, const BatchTable* tabs, const int32_t* tab_of,
                           int64_t k0, int64_t kc, float* out, hipStream_t st) {
    if (kc <= 0 || e.n <= 0) return hipSuccess;
    const int64_t gy = (e.n + 63) / 64;
    if (gy > 65535) {
        return hipErrorInvalidValue;
    }
    dim3 grid(unsigned((kc + 255) / 256), unsigned(gy));
    hipLaunchKernelGGL(k_embed_batch_f32, grid, dim3(256), 0, st, e.n, k0, kc, tabs, tab_of,
                       e.row_ptr, e.rank, e.cum, e.total, e.lo, e.hi, e.len, out);
    return hipGetLastError();
}

// the persistent kernel for (branches per stage, stripes per tile)
template <int KS, int MS>
static const void* persistent_fn() {
    return reinterpret_cast<const void*>(&k_band_persistent_f32<KS, MS>);
}
static const void* persistent_kernel(int stage_branches, int tile_stripes) {
#define UF_PK(KS_)                                                           \
    if (stage_branches == KS_) {                                             \
        if (tile_stripes == 64) return persistent_fn<KS_, 4>();              \
        if (tile_stripes == 128) return persistent_fn<KS_, 8>();             \
        if (tile_stripes == 256) return persistent_fn<KS_, 16>();            \
    }
    UF_PK(8)
    UF_PK(16)
    UF_PK(32)
#undef UF_PK
    return nullptr;
}

int band_persistent_max_blocks(int stage_branches, int tile_stripes) {
    const void* fn = persistent_kernel(stage_branches, tile_stripes);
    if (!fn) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 256, 0) != hipSuccess) return 0;
    return blocks;
}

hipError_t band_persistent_f32(const float* E, const BatchTable* tabs, const int2* items,
                               const int64_t* qbeg, const int64_t* qend, unsigned* counters,
                               int64_t kc, int first, float* acc, int stage_branches,
                               int tile_stripes, int n_blocks, hipStream_t st) {
    const void* fn = persistent_kernel(stage_branches, tile_stripes);
    if (!fn || n_blocks < 1) return hipErrorInvalidValue;
    void* args[] = {&E, &tabs, &items, &qbeg, &qend, &counters, &kc, &first, &acc};
    const hipError_t e = hipLaunchKernel(fn, dim3(unsigned(n_blocks)), dim3(256), args, 0, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t zero_u32(unsigned* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace ufk
