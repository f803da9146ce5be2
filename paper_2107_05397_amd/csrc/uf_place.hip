// HIP kernels of the learned placement encoder (gfx950):
//
//   k_project          sparse random projection of l*u (fixed-point LDS sums)
//   k_gemm_bf16<..>    BF16 MFMA GEMM, FP32 accumulate, three operand layouts
//                      (forward X W^T, backward-data dY W, weight-grad dY^T X)
//                      with fused bias / ReLU / ReLU-mask epilogues
//   k_colsum_*         bias gradients (fixed-order FP64 column sums)
//   k_pairloss         (||z_a - z_b|| - d)^2 and its gradient
//   k_tripletloss      ranking loss over (anchor, near, far) triples
//   k_adam, k_adam_multi   Adam on FP32 master weights + BF16 copy (one tensor,
//                      or all of an MLP's tensors in one launch)
//   k_sqdist           FP32 pairwise squared distances (kNN)
//   k_topk_rows        exact k smallest per row (radix select, ties by index)
//   k_sparse_*         per-sample lists of (branch, l*u) for nonzero branches
//   k_rerank           exact weighted-normalized distance across two tables
//   k_condensed_block, k_gather_pairs   reads of a condensed matrix
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "uf_internal.h"
#include "uf_place.h"

namespace ufp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);     // round to nearest even (finite inputs)
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ int64_t lower_bound_rank(const int32_t* __restrict__ rank, int64_t a,
                                                    int64_t b, int32_t key) {
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (rank[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a;
}

// count of sample s on the branch covering tip ranks [lo, hi)
__device__ __forceinline__ int64_t count_in(const int64_t* __restrict__ row_ptr,
                                            const int32_t* __restrict__ rank,
                                            const int64_t* __restrict__ cum, int64_t s, int32_t lo,
                                            int32_t hi) {
    const int64_t a = row_ptr[s], b = row_ptr[s + 1];
    const int64_t p1 = lower_bound_rank(rank, a, b, lo);
    const int64_t p2 = lower_bound_rank(rank, p1, b, hi);
    return cum[p2 + s] - cum[p1 + s];
}

// ----------------------------------------------------------------------------
// Nonzero branches of a sample, each exactly once: walking up from the tip of
// entry e, a branch v is reported by e when the previous tip of the row
// (rank[e-1]) lies outside v's subtree, i.e. lo_v > rank[e-1]; the walk stops
// at the first ancestor that also covers the previous tip (reported already).
// ----------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void for_each_branch_of_entry(const Emb& e, int64_t entry,
                                                         int64_t row_start, F&& f) {
    const int32_t r = e.rank[entry];
    const int32_t prev = entry > row_start ? e.rank[entry - 1] : -1;
    int32_t v = e.tip_pos[r];
    while (v < e.root_pos && e.lo[v] > prev) {
        f(v);
        v = e.parent_pos[v];
    }
}

// x[s] = sum_v l_v u_sv * sign/2 at dims: one block per sample, int64 fixed
// point (2^-40) sums in LDS so the result does not depend on atomic order.
__global__ __launch_bounds__(256) void k_project(Emb e, const int32_t* __restrict__ dims,
                                                 const int8_t* __restrict__ signs, int per_node,
                                                 int out_dim, double scale,
                                                 uint16_t* __restrict__ out) {
    extern __shared__ unsigned long long acc[];
    const int64_t s = blockIdx.x;
    for (int d = threadIdx.x; d < out_dim; d += 256) acc[d] = 0ull;
    __syncthreads();
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    const double inv_t = 1.0 / e.total[s];
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256) {
        for_each_branch_of_entry(e, ent, a, [&](int32_t v) {
            const int64_t c = count_in(e.row_ptr, e.rank, e.cum, s, e.lo[v], e.hi[v]);
            const double y = e.len[v] * (double(c) * inv_t) * 0.5 * scale;
            const long long q = llrint(y * 1099511627776.0);   // 2^40
            for (int j = 0; j < per_node; ++j) {
                const long long sq = signs[int64_t(v) * per_node + j] > 0 ? q : -q;
                atomicAdd(&acc[dims[int64_t(v) * per_node + j]], (unsigned long long)sq);
            }
        });
    }
    __syncthreads();
    for (int d = threadIdx.x; d < out_dim; d += 256) {
        const double x = double((long long)acc[d]) * (1.0 / 1099511627776.0);
        out[s * out_dim + d] = f2bf(float(x));
    }
}

// ----------------------------------------------------------------------------
// BF16 GEMM on MFMA: C[m][n] = sum_k A(m, k) B(n, k), FP32 accumulation.
// Layout 0 (row): element (r, k) at P[src(r) * ld + k]   (k contiguous)
// Layout 1 (col): element (r, k) at P[src(k) * ld + r]   (r contiguous)
// src() applies the optional row-index array (a gather of storage rows).
//
// A block computes a BM x BN tile: 128 x 128 or 256 x 128 with 4 waves in 2 x 2
// (a wave owns (BM/2) x 64), or 256 x 256 with 8 waves in 2 x 4 (a wave owns
// 128 x 64), as 32 x 32 blocks of v_mfma_f32_32x32x16_bf16.  The
// K loop steps by 64 through two LDS stages that hold the tile's rows as
// [row][k] with a 144-byte pitch (an odd multiple of 16 bytes, so the 16-byte
// fragment reads of consecutive rows fall on distinct banks).  Row-layout
// operands are staged in 16-byte pieces; column-layout ones in pieces of 4 (k)
// x 8 (rows), transposed in registers on the way into LDS.  The global loads of
// step t+1 are in flight while the MFMAs of step t run, and there is one
// barrier per step: the stage written at step t was last read at step t-2,
// which every wave finished before the barrier of step t-1.
//
// blockIdx.z takes one range of K steps (split K).  With a single range the
// epilogue is applied here; with several, each range writes its raw sums to
// part[z][M][N] and k_gemm_reduce adds the ranges in order and applies the
// epilogue, so the result never depends on the order blocks run in.
// ----------------------------------------------------------------------------
constexpr int kGemmKS = 64;              // K per step
constexpr int kGemmLD = kGemmKS + 8;     // LDS row pitch in bf16 (144 bytes)

template <int EPI>
__device__ __forceinline__ void gemm_store(float v, int64_t i, int64_t j,
                                           const float* __restrict__ bias,
                                           const uint16_t* __restrict__ mask, int64_t ldm,
                                           void* __restrict__ C, int64_t ldc) {
    if (EPI == EPI_F32) {
        static_cast<float*>(C)[i * ldc + j] = v;
    } else if (EPI == EPI_ACC_F32) {
        static_cast<float*>(C)[i * ldc + j] += v;
    } else if (EPI == EPI_BIAS_RELU_BF16) {
        static_cast<uint16_t*>(C)[i * ldc + j] = f2bf(fmaxf(v + bias[j], 0.0f));
    } else if (EPI == EPI_BIAS_F32) {
        static_cast<float*>(C)[i * ldc + j] = v + bias[j];
    } else if (EPI == EPI_MASK_BF16) {
        static_cast<uint16_t*>(C)[i * ldc + j] = mask[i * ldm + j] != 0 ? f2bf(v) : uint16_t(0);
    } else {
        static_cast<uint16_t*>(C)[i * ldc + j] = f2bf(v);
    }
}

// The epilogue on four consecutive columns j..j+3 of row i (j a multiple of 4,
// all four inside the matrix): 16-byte FP32 or 8-byte BF16 accesses, each
// element computed exactly as gemm_store computes it.
template <int EPI>
__device__ __forceinline__ void gemm_store4(float4 v, int64_t i, int64_t j,
                                            const float* __restrict__ bias,
                                            const uint16_t* __restrict__ mask, int64_t ldm,
                                            void* __restrict__ C, int64_t ldc) {
    if (EPI == EPI_F32) {
        *reinterpret_cast<float4*>(static_cast<float*>(C) + i * ldc + j) = v;
    } else if (EPI == EPI_ACC_F32) {
        float4* c = reinterpret_cast<float4*>(static_cast<float*>(C) + i * ldc + j);
        const float4 o = *c;
        *c = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
    } else if (EPI == EPI_BIAS_F32) {
        const float4 b = *reinterpret_cast<const float4*>(bias + j);
        *reinterpret_cast<float4*>(static_cast<float*>(C) + i * ldc + j) =
            make_float4(v.x + b.x, v.y + b.y, v.z + b.z, v.w + b.w);
    } else {
        uint32_t h0, h1, h2, h3;
        if (EPI == EPI_BIAS_RELU_BF16) {
            const float4 b = *reinterpret_cast<const float4*>(bias + j);
            h0 = f2bf(fmaxf(v.x + b.x, 0.0f));
            h1 = f2bf(fmaxf(v.y + b.y, 0.0f));
            h2 = f2bf(fmaxf(v.z + b.z, 0.0f));
            h3 = f2bf(fmaxf(v.w + b.w, 0.0f));
        } else if (EPI == EPI_MASK_BF16) {
            const uint2 mk = *reinterpret_cast<const uint2*>(mask + i * ldm + j);
            h0 = (mk.x & 0xFFFFu) != 0 ? f2bf(v.x) : 0u;
            h1 = (mk.x >> 16) != 0 ? f2bf(v.y) : 0u;
            h2 = (mk.y & 0xFFFFu) != 0 ? f2bf(v.z) : 0u;
            h3 = (mk.y >> 16) != 0 ? f2bf(v.w) : 0u;
        } else {
            h0 = f2bf(v.x);
            h1 = f2bf(v.y);
            h2 = f2bf(v.z);
            h3 = f2bf(v.w);
        }
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(C) + i * ldc + j) =
            make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
    }
}

// One operand's share of a K step in a thread's registers: TR rows of the tile,
// TR/32 uint4 per thread in either layout (row: TR*8 pieces of 16 bytes; col:
// TR*2 pieces of 4 x 16 bytes).
template <int LAY, int TR, int NT = 256>
struct GemmOperand {
    // pieces per thread: row layout TR*8 of 16 bytes, column layout TR*2 of 4 x 16
    static constexpr int NV = TR * 8 / NT;
    static constexpr int NP = LAY == 0 ? NV : TR * 2 / NT;
    static_assert(NP >= 1 && (LAY == 0 ? TR * 8 : TR * 2) % NT == 0, "operand split");
    const uint16_t* P;
    int64_t ld;
    const int32_t* rows;
    int64_t r0, R, K;
    const uint16_t* rowp[LAY == 0 ? NV : 1];              // row layout: source row of each piece
    // column layout with a row gather: the storage rows of the next fetch's k,
    // loaded one fetch ahead so that no fetch waits on its own index loads
    int32_t ix[LAY == 1 ? NP : 1][4];

    __device__ __forceinline__ void load_ix(int64_t k0, int tid) {
        if (K <= 0) return;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int64_t kb = k0 + 4 * ((tid + NT * i) % 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) ix[i][e] = rows[min(kb + e, K - 1)];
        }
    }

    // k_first: the K offset of the first fetch
    __device__ __forceinline__ void init(const uint16_t* P_, int64_t ld_, const int32_t* rows_,
                                         int64_t r0_, int64_t R_, int64_t K_, int tid,
                                         int64_t k_first) {
        P = P_;
        ld = ld_;
        rows = rows_;
        r0 = r0_;
        R = R_;
        K = K_;
        if constexpr (LAY == 1) {
            if (rows) load_ix(k_first, tid);
        }
        if constexpr (LAY == 0) {
            // rows past the end read the last row (always a valid address)
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int64_t gr = min(r0 + ((tid + NT * i) >> 3), R - 1);
                rowp[i] = P + (rows ? int64_t(rows[gr]) : gr) * ld;
            }
        }
    }

    // (staged values travel by value: an array passed by reference is kept in
    // memory, which the compiler may place in LDS)
    struct Regs {
        uint4 v[NV];
    };

    // Every load is issued unconditionally from a clamped, valid address (16-byte
    // vector loads, no branches).  Pieces of rows past R hold copies of the last
    // row: they only reach output rows or columns that are never stored.  Pieces
    // past K are zeroed when they are written to LDS (stash), so no wait on the
    // loads is placed before the MFMAs that overlap them.
    // (k0 advances by one K step per call, except repeats of the last step,
    // whose data is never used)
    __device__ __forceinline__ Regs fetch(int64_t k0, int tid) {
        Regs out;
        uint4* v = out.v;
        if constexpr (LAY == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int p = tid + NT * i;
                const int64_t k = k0 + 8 * (p & 7);
                v[i] = *reinterpret_cast<const uint4*>(rowp[i] + min(k, K - 8));
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int p = tid + NT * i;
                const int64_t rc = min(r0 + 8 * (p / 16), R - 8);
                const int64_t kb = k0 + 4 * (p % 16);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t kcl = min(kb + e, K - 1);
                    const int64_t src = rows ? int64_t(ix[i][e]) : kcl;
                    v[4 * i + e] = *reinterpret_cast<const uint4*>(P + src * ld + rc);
                }
            }
            if (rows) load_ix(k0 + kGemmKS, tid);
        }
        return out;
    }

    static __device__ __forceinline__ uint32_t half_of(const uint4& u, int j) {
        const uint32_t w = j < 2 ? u.x : (j < 4 ? u.y : (j < 6 ? u.z : u.w));
        return (j & 1) ? (w >> 16) : (w & 0xFFFFu);
    }

    // a piece, or zeros (component by component: a select between two uint4
    // objects would be compiled as a select between their addresses, in memory)
    static __device__ __forceinline__ uint4 keep(const uint4& w, bool ok) {
        return make_uint4(ok ? w.x : 0u, ok ? w.y : 0u, ok ? w.z : 0u, ok ? w.w : 0u);
    }

    // the K step at k0 into LDS, its pieces at k >= K as zeros
    __device__ __forceinline__ void stash(const Regs in, uint16_t* __restrict__ S, int tid,
                                          int64_t k0) const {
        const uint4* v = in.v;
        if constexpr (LAY == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int p = tid + NT * i;
                const bool ok = k0 + 8 * (p & 7) < K;
                *reinterpret_cast<uint4*>(S + (p >> 3) * kGemmLD + 8 * (p & 7)) = keep(v[i], ok);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int p = tid + NT * i;
                const int rb = p / 16, kq = p % 16;
                const int64_t kb = k0 + 4 * kq;
                uint4 u[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) u[e] = keep(v[4 * i + e], kb + e < K);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    uint2 w;
                    w.x = half_of(u[0], j) | (half_of(u[1], j) << 16);
                    w.y = half_of(u[2], j) | (half_of(u[3], j) << 16);
                    *reinterpret_cast<uint2*>(S + (8 * rb + j) * kGemmLD + 4 * kq) = w;
                }
            }
        }
    }
};

// Block b runs on XCD b mod 8 and takes the (b / 8)-th tile of that XCD's
// eighth of the tiles in grouped order: bands of gh tile rows, column by column
// inside a band.  An XCD's consecutive tiles then form about a gh x (P / gh)
// rectangle (P tiles per XCD), whose blocks share gh row panels of A and P / gh
// column panels of B in the XCD's L2.
__device__ __forceinline__ void gemm_xcd_tile(int64_t b, int64_t tm, int64_t tn, int64_t gh,
                                              int64_t& mt, int64_t& nt) {
    const int64_t n_tiles = tm * tn;
    const int64_t x = b & 7, local = b >> 3;
    const int64_t per = n_tiles >> 3, rem = n_tiles & 7;
    const int64_t t = x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
    const int64_t band = t / (gh * tn);
    const int64_t r0 = band * gh;
    const int64_t h = min(gh, tm - r0);   // the last band may be shorter
    const int64_t w = t - band * gh * tn;
    nt = w / h;
    mt = r0 + w % h;
}

template <int LA, int LB, int EPI, int BM, int BN, int NT>
__global__ __launch_bounds__(NT, BM * BN >= 32768 ? 1 : 2) void k_gemm_bf16(
    const uint16_t* __restrict__ A, int64_t lda, const int32_t* __restrict__ arow,
    const uint16_t* __restrict__ B, int64_t ldb, const int32_t* __restrict__ brow, int64_t M,
    int64_t N, int64_t K, const float* __restrict__ bias, const uint16_t* __restrict__ mask,
    int64_t ldm, void* __restrict__ C, int64_t ldc, float* __restrict__ part, int64_t gh) {
    // NT/64 waves in 2 x WJ; a wave owns (BM/2) x (BN/WJ) as XB x YB MFMA blocks
    constexpr int WJ = NT / 128;
    constexpr int XB = BM / 64;          // 32-row blocks per wave
    constexpr int YB = BN / (32 * WJ);   // 32-column blocks per wave
    // operand pieces: 128-row halves with 256 threads, whole tiles with 512
    constexpr int TRA = NT == 512 ? BM : 128, TRB = NT == 512 ? BN : 128;
    constexpr int HA = BM / TRA, HB = BN / TRB;
    static_assert(YB >= 1 && HA >= 1 && HA <= 2 && HB >= 1 && HB <= 2, "GEMM tile shape");
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * kGemmLD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * kGemmLD];
    int64_t mt, nt;
    gemm_xcd_tile(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, gh, mt, nt);
    const int64_t m0 = mt * BM, n0 = nt * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave & 1, wj = wave >> 1;

    // this block's range of K steps
    const int64_t nk = (K + kGemmKS - 1) / kGemmKS;
    const int64_t per = (nk + gridDim.z - 1) / gridDim.z;
    const int64_t t0 = int64_t(blockIdx.z) * per;
    const int64_t t1 = min(nk, t0 + per);

    // operands in pieces of at most 16 staged registers per thread (larger
    // arrays would be kept in memory)
    GemmOperand<LA, TRA, NT> oa0, oa1;
    GemmOperand<LB, TRB, NT> ob0, ob1;
    oa0.init(A, lda, arow, m0, M, K, tid, t0 * kGemmKS);
    if constexpr (HA == 2) oa1.init(A, lda, arow, m0 + TRA, M, K, tid, t0 * kGemmKS);
    ob0.init(B, ldb, brow, n0, N, K, tid, t0 * kGemmKS);
    if constexpr (HB == 2) ob1.init(B, ldb, brow, n0 + TRB, N, K, tid, t0 * kGemmKS);

    floatx16 c[XB][YB];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
        for (int y = 0; y < YB; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) c[x][y][r] = 0.0f;

    auto compute = [&](int buf) {
#pragma unroll
        for (int s = 0; s < kGemmKS / 16; ++s) {
            const int kq = 16 * s + 8 * (lane >> 5);
            bf16x8 fa[XB], fb[YB];
#pragma unroll
            for (int x = 0; x < XB; ++x)
                fa[x] = *reinterpret_cast<const bf16x8*>(
                    As[buf] + (wi * (BM / 2) + x * 32 + (lane & 31)) * kGemmLD + kq);
#pragma unroll
            for (int y = 0; y < YB; ++y)
                fb[y] = *reinterpret_cast<const bf16x8*>(
                    Bs[buf] + (wj * (BN / WJ) + y * 32 + (lane & 31)) * kGemmLD + kq);
#pragma unroll
            for (int x = 0; x < XB; ++x)
#pragma unroll
                for (int y = 0; y < YB; ++y)
                    c[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fb[y], c[x][y], 0, 0, 0);
        }
    };

    if (t0 < t1) {
        using OA = GemmOperand<LA, TRA, NT>;
        using OB = GemmOperand<LB, TRB, NT>;
        typename OA::Regs ra0 = oa0.fetch(t0 * kGemmKS, tid), ra1{};
        if constexpr (HA == 2) ra1 = oa1.fetch(t0 * kGemmKS, tid);
        typename OB::Regs rb0 = ob0.fetch(t0 * kGemmKS, tid), rb1{};
        if constexpr (HB == 2) rb1 = ob1.fetch(t0 * kGemmKS, tid);
        auto stash_all = [&](int buf, int64_t k0) {
            oa0.stash(ra0, As[buf], tid, k0);
            if constexpr (HA == 2) oa1.stash(ra1, As[buf] + TRA * kGemmLD, tid, k0);
            ob0.stash(rb0, Bs[buf], tid, k0);
            if constexpr (HB == 2) ob1.stash(rb1, Bs[buf] + TRB * kGemmLD, tid, k0);
        };
        auto fetch_all = [&](int64_t k0) {
            ra0 = oa0.fetch(k0, tid);
            if constexpr (HA == 2) ra1 = oa1.fetch(k0, tid);
            rb0 = ob0.fetch(k0, tid);
            if constexpr (HB == 2) rb1 = ob1.fetch(k0, tid);
        };
        for (int64_t t = t0; t < t1; t += 2) {
            stash_all(0, t * kGemmKS);
            fetch_all(min(t + 1, t1 - 1) * kGemmKS);   // past the end: re-read, unused
            __syncthreads();
            compute(0);
            if (t + 1 < t1) {   // block-uniform
                stash_all(1, (t + 1) * kGemmKS);
                fetch_all(min(t + 2, t1 - 1) * kGemmKS);
                __syncthreads();
                compute(1);
            }
        }
    }

    // Epilogue through LDS.  D of a 32x32 block: lane holds column lane%32, rows
    // 8*(r/4) + 4*(lane/32) + r%4 -- column-wise, so direct stores would be 2 or
    // 4 bytes per lane.  Once every wave has left the K loop the A stages are
    // free: each wave stages one 32-row strip of its sub-tile at a time (32 x
    // 32*YB floats) in an area of its own and reads it back as rows of 4
    // consecutive columns per lane, for 16-byte FP32 (partial sums) or 8-byte
    // BF16 stores.  The area is private to the wave, so wave-scope ordering
    // between its LDS writes and reads suffices.
    __syncthreads();
    constexpr int EW = 32 * YB;          // strip width in columns
    constexpr int EP = EW + 8;           // strip pitch in floats (rows 4 apart on other banks)
    constexpr int CPR = EW / 4;          // 4-column pieces per strip row
    static_assert((NT / 64) * 32 * EP * 4 <= int(sizeof(As)), "epilogue staging");
    float* strip = reinterpret_cast<float*>(&As[0][0]) + wave * (32 * EP);
    const bool split = gridDim.z > 1;
    float* pz = split ? part + int64_t(blockIdx.z) * M * N : nullptr;
    const int64_t ci0 = m0 + wi * (BM / 2), cj0 = n0 + wj * (BN / WJ);
#pragma unroll
    for (int x = 0; x < XB; ++x) {
#pragma unroll
        for (int y = 0; y < YB; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                strip[(8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * EP + 32 * y + (lane & 31)] =
                    c[x][y][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < 32 * CPR / 64; ++q) {
            const int pc = lane + 64 * q;
            const int rr = pc / CPR, cc = pc % CPR;
            const float4 v = *reinterpret_cast<const float4*>(strip + rr * EP + 4 * cc);
            const int64_t i = ci0 + 32 * x + rr, j = cj0 + 4 * cc;
            if (i >= M || j >= N) continue;
            if (split) *reinterpret_cast<float4*>(pz + i * N + j) = v;
            else gemm_store4<EPI>(v, i, j, bias, mask, ldm, C, ldc);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Split-K: the ranges' sums added in range order, then the epilogue; four
// consecutive elements of a row per thread (N is a multiple of 4).
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_reduce(const float* __restrict__ part, int splits,
                                                     int64_t M, int64_t N,
                                                     const float* __restrict__ bias,
                                                     const uint16_t* __restrict__ mask, int64_t ldm,
                                                     void* __restrict__ C, int64_t ldc) {
    const int64_t e = 4 * (int64_t(blockIdx.x) * 256 + threadIdx.x);
    const int64_t MN = M * N;
    if (e >= MN) return;
    float4 v = *reinterpret_cast<const float4*>(part + e);
    for (int z = 1; z < splits; ++z) {
        const float4 w = *reinterpret_cast<const float4*>(part + int64_t(z) * MN + e);
        v = make_float4(v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w);
    }
    const int64_t i = e / N;
    gemm_store4<EPI>(v, i, e - i * N, bias, mask, ldm, C, ldc);
}

// Column sums of a BF16 [rows][cols] matrix (cols a multiple of 8) in FP64, in a
// fixed order.  Block (x, y) takes the G = min(cols/8, 256) groups of 8 columns
// from 8*G*x and rows [y*chunk, (y+1)*chunk): each thread holds one column group
// and strides over the chunk's rows with 256/G others (16-byte loads), then the
// row lanes are added in lane order into part[y][cols].  k_colsum_final adds the
// chunks: 8 lanes per column take every 8th chunk, then are added in lane order.
constexpr int kColsumChunks = 128;
__global__ __launch_bounds__(256) void k_colsum_part(const uint16_t* __restrict__ X, int64_t rows,
                                                     int64_t cols, int64_t chunk,
                                                     double* __restrict__ part) {
    __shared__ double red[256][9];
    const int64_t groups = cols / 8;
    const int G = groups < 256 ? int(groups) : 256;
    const int R = 256 / G;
    const int t = threadIdx.x, cg = t % G, rl = t / G;
    const int64_t grp = int64_t(blockIdx.x) * G + cg;
    const int64_t r0 = int64_t(blockIdx.y) * chunk, r1 = min(rows, r0 + chunk);
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (rl < R && grp < groups) {
        const uint16_t* col = X + 8 * grp;
        for (int64_t r = r0 + rl; r < r1; r += R) {
            const uint4 w = *reinterpret_cast<const uint4*>(col + r * cols);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s[2 * e] += double(__uint_as_float(ws[e] << 16));
                s[2 * e + 1] += double(__uint_as_float(ws[e] & 0xFFFF0000u));
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[t][e] = s[e];
    __syncthreads();
    // column 8*cg' + e' of the block (t' = 8*cg' + e' < 8*G), summed over the R
    // row lanes
    for (int t2 = t; t2 < 8 * G; t2 += 256) {
        const int cg2 = t2 / 8, e2 = t2 % 8;
        const int64_t g2 = int64_t(blockIdx.x) * G + cg2;
        if (g2 < groups) {
            double a = 0.0;
            for (int k = 0; k < R; ++k) a += red[k * G + cg2][e2];
            part[int64_t(blockIdx.y) * cols + 8 * g2 + e2] = a;
        }
    }
}
__global__ __launch_bounds__(256) void k_colsum_final(const double* __restrict__ part, int chunks,
                                                      int64_t cols, float* __restrict__ out) {
    __shared__ double red[8][32];
    const int c = threadIdx.x % 32, ln = threadIdx.x / 32;
    const int64_t j = int64_t(blockIdx.x) * 32 + c;
    double s = 0.0;
    if (j < cols)
        for (int y = ln; y < chunks; y += 8) s += part[int64_t(y) * cols + j];
    red[ln][c] = s;
    __syncthreads();
    if (ln == 0 && j < cols) {
        double a = 0.0;
        for (int k = 0; k < 8; ++k) a += red[k][c];
        out[j] = float(a);
    }
}

// one wave per pair; Z rows [0, P) are the a-ends, [P, 2P) the b-ends
// rel_floor > 0 selects the relative loss ((delta - d) / max(d, rel_floor))^2
__global__ __launch_bounds__(256) void k_pairloss(const float* __restrict__ Z, int64_t P, int D,
                                                  const float* __restrict__ target, float rel_floor,
                                                  uint16_t* __restrict__ dZ,
                                                  float* __restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int64_t p = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (p >= P) return;
    const float* za = Z + p * D;
    const float* zb = Z + (P + p) * D;
    float s = 0.0f;
    for (int d = lane; d < D; d += 64) {
        const float df = za[d] - zb[d];
        s = fmaf(df, df, s);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const float delta = sqrtf(s);
    const float w = rel_floor > 0.0f ? 1.0f / fmaxf(target[p], rel_floor) : 1.0f;
    const float r = (delta - target[p]) * w;
    const float coef = delta > 0.0f ? 2.0f * r * w / delta / float(P) : 0.0f;
    for (int d = lane; d < D; d += 64) {
        const float g = coef * (za[d] - zb[d]);
        dZ[p * D + d] = f2bf(g);
        dZ[(P + p) * D + d] = f2bf(-g);
    }
    if (lane == 0) loss[p] = r * r;
}

// Ranking loss, one wave per triple; Z rows [0, T) are the anchors, [T, 2T) the
// near ends, [2T, 3T) the far ends.  Per triple, with e_p = ||z_a - z_p|| and
// e_n = ||z_a - z_n||:
//   L = alpha ((e_p - d_p)^2 + (e_n - d_n)^2) + lam * tau * softplus((e_p - e_n) / tau)
// and dZ receives dL/dz / T for the mean over triples.
__global__ __launch_bounds__(256) void k_tripletloss(const float* __restrict__ Z, int64_t T, int D,
                                                     const float* __restrict__ d_near,
                                                     const float* __restrict__ d_far, float alpha,
                                                     float lam, float tau,
                                                     uint16_t* __restrict__ dZ,
                                                     float* __restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= T) return;
    const float* za = Z + t * D;
    const float* zp = Z + (T + t) * D;
    const float* zn = Z + (2 * T + t) * D;
    float sp = 0.0f, sn = 0.0f;
    for (int d = lane; d < D; d += 64) {
        const float a = za[d];
        const float dp = a - zp[d], dn = a - zn[d];
        sp = fmaf(dp, dp, sp);
        sn = fmaf(dn, dn, sn);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sp += __shfl_xor(sp, off, 64);
        sn += __shfl_xor(sn, off, 64);
    }
    const float ep = sqrtf(sp), en = sqrtf(sn);
    const float s = (ep - en) / tau;
    const float e = expf(-fabsf(s));                           // in (0, 1]
    const float sig = s >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
    const float rp = ep - d_near[t], rn = en - d_far[t];
    const float inv_t = 1.0f / float(T);
    const float gp = (2.0f * alpha * rp + lam * sig) * inv_t;
    const float gn = (2.0f * alpha * rn - lam * sig) * inv_t;
    const float cp = ep > 0.0f ? gp / ep : 0.0f;
    const float cn = en > 0.0f ? gn / en : 0.0f;
    for (int d = lane; d < D; d += 64) {
        const float a = za[d];
        const float vp = cp * (a - zp[d]), vn = cn * (a - zn[d]);
        dZ[t * D + d] = f2bf(vp + vn);
        dZ[(T + t) * D + d] = f2bf(-vp);
        dZ[(2 * T + t) * D + d] = f2bf(-vn);
    }
    if (lane == 0) loss[t] = alpha * (rp * rp + rn * rn) + lam * tau * (fmaxf(s, 0.0f) + log1pf(e));
}

__global__ __launch_bounds__(256) void k_mean(const float* __restrict__ x, int64_t n,
                                              float* __restrict__ out) {
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) a += x[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = float(red[0] / double(n > 0 ? n : 1));
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2, float wd,
                                              uint16_t* __restrict__ pbf) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    // decoupled weight decay (AdamW): wd = 0 gives plain Adam
    const float pi = p[i] - lr * ((mi / bc1) / (sqrtf(vi / bc2) + eps) + wd * p[i]);
    p[i] = pi;
    if (pbf) pbf[i] = f2bf(pi);
}

// Adam over several tensors in one launch: thread t of the launch takes four
// consecutive elements of the tensor whose range of 4-element groups holds t
// (16-byte accesses where the tensor allows them); each element is updated
// exactly as k_adam updates it.
__device__ __forceinline__ float adam_elem(float& p, float g, float& m, float& v, float lr,
                                           float b1, float b2, float eps, float bc1, float bc2,
                                           float wd) {
    const float mi = b1 * m + (1.0f - b1) * g;
    const float vi = b2 * v + (1.0f - b2) * g * g;
    m = mi;
    v = vi;
    p = p - lr * ((mi / bc1) / (sqrtf(vi / bc2) + eps) + wd * p);
    return p;
}
__global__ __launch_bounds__(256) void k_adam_multi(AdamBatch ab, float lr, float b1, float b2,
                                                    float eps, float bc1, float bc2) {
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= ab.start[ab.count]) return;
    int k = 0;
    while (q >= ab.start[k + 1]) ++k;
    const AdamTensor& t = ab.t[k];
    const int64_t i0 = 4 * (q - ab.start[k]);
    if (t.vec) {   // n % 4 == 0, 16-byte aligned FP32 arrays, 8-byte aligned BF16 copy
        float4 p = *reinterpret_cast<const float4*>(t.p + i0);
        const float4 g = *reinterpret_cast<const float4*>(t.g + i0);
        float4 m = *reinterpret_cast<const float4*>(t.m + i0);
        float4 v = *reinterpret_cast<const float4*>(t.v + i0);
        adam_elem(p.x, g.x, m.x, v.x, lr, b1, b2, eps, bc1, bc2, t.wd);
        adam_elem(p.y, g.y, m.y, v.y, lr, b1, b2, eps, bc1, bc2, t.wd);
        adam_elem(p.z, g.z, m.z, v.z, lr, b1, b2, eps, bc1, bc2, t.wd);
        adam_elem(p.w, g.w, m.w, v.w, lr, b1, b2, eps, bc1, bc2, t.wd);
        *reinterpret_cast<float4*>(t.p + i0) = p;
        *reinterpret_cast<float4*>(t.m + i0) = m;
        *reinterpret_cast<float4*>(t.v + i0) = v;
        if (t.pbf)
            *reinterpret_cast<uint2*>(t.pbf + i0) =
                make_uint2(f2bf(p.x) | (uint32_t(f2bf(p.y)) << 16), f2bf(p.z) | (uint32_t(f2bf(p.w)) << 16));
        return;
    }
    const int64_t cnt = min(int64_t(4), t.n - i0);
    for (int64_t e = 0; e < cnt; ++e) {
        const int64_t i = i0 + e;
        float p = t.p[i], m = t.m[i], v = t.v[i];
        adam_elem(p, t.g[i], m, v, lr, b1, b2, eps, bc1, bc2, t.wd);
        t.m[i] = m;
        t.v[i] = v;
        t.p[i] = p;
        if (t.pbf) t.pbf[i] = f2bf(p);
    }
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* __restrict__ x, int64_t n,
                                                     uint16_t* __restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// out[i][j] = sum_d (a_i[d] - b_j[d])^2, d in increasing order (one fused
// multiply-add per d).  128 x 128 tiles, 8 x 8 per thread; the tile's rows go
// through LDS 16 dimensions at a time as [d][row], so a thread reads its eight
// rows of A and of B as two 16-byte loads each.
constexpr int kSqT = 128, kSqD = 16, kSqP = kSqT + 4;
__global__ __launch_bounds__(256) void k_sqdist(const float* __restrict__ A, int64_t na,
                                                const float* __restrict__ B, int64_t nb, int64_t D,
                                                float* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) float as[kSqD][kSqP];
    __shared__ __attribute__((aligned(16))) float bs[kSqD][kSqP];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t i0 = int64_t(blockIdx.y) * kSqT, j0 = int64_t(blockIdx.x) * kSqT;
    float acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int w = 0; w < 8; ++w) acc[u][w] = 0.0f;
    for (int64_t d0 = 0; d0 < D; d0 += kSqD) {
        __syncthreads();
        for (int t = threadIdx.x; t < kSqT * kSqD; t += 256) {
            const int r = t / kSqD, dd = t % kSqD;
            as[dd][r] = (i0 + r < na && d0 + dd < D) ? A[(i0 + r) * D + d0 + dd] : 0.0f;
            bs[dd][r] = (j0 + r < nb && d0 + dd < D) ? B[(j0 + r) * D + d0 + dd] : 0.0f;
        }
        __syncthreads();
        const int dn = int(min<int64_t>(kSqD, D - d0));
        for (int dd = 0; dd < dn; ++dd) {
            const float4 a0 = *reinterpret_cast<const float4*>(&as[dd][ty * 8]);
            const float4 a1 = *reinterpret_cast<const float4*>(&as[dd][ty * 8 + 4]);
            const float4 b0 = *reinterpret_cast<const float4*>(&bs[dd][tx * 8]);
            const float4 b1 = *reinterpret_cast<const float4*>(&bs[dd][tx * 8 + 4]);
            const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const float b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const float df = a[u] - b[w];
                    acc[u][w] = fmaf(df, df, acc[u][w]);
                }
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const int64_t i = i0 + ty * 8 + u, j = j0 + tx * 8 + w;
            if (i < na && j < nb) out[i * nb + j] = acc[u][w];
        }
}

// ----------------------------------------------------------------------------
// k smallest of each row (values >= 0), ties by the smaller column: radix
// select on the FP32 bit pattern (monotone for non-negative floats) in four
// 8-bit passes, then collect below-threshold entries plus the first equal
// ones in column order, then sort the k pairs (bits, column) in LDS.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_topk_rows(const float* __restrict__ vals, int64_t cols,
                                                   int k, int32_t* __restrict__ idx_out,
                                                   float* __restrict__ val_out) {
    __shared__ unsigned hist[256];
    __shared__ unsigned s_prefix, s_mask, s_remaining, s_nless, s_neq;
    __shared__ unsigned cb[kTopkMax];
    __shared__ int ci[kTopkMax];
    __shared__ unsigned wave_cnt[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float* v = vals + int64_t(blockIdx.x) * cols;
    if (tid == 0) {
        s_prefix = 0;
        s_mask = 0;
        s_remaining = unsigned(k);
        s_nless = 0;
        s_neq = 0;
    }
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        const unsigned prefix = s_prefix, mask = s_mask;
        for (int64_t c = tid; c < cols; c += 256) {
            const unsigned bits = __float_as_uint(v[c]);
            if ((bits & mask) == prefix) atomicAdd(&hist[(bits >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            unsigned cum = 0, rem = s_remaining;
            int d = 0;
            for (; d < 256; ++d) {
                if (cum + hist[d] >= rem) break;
                cum += hist[d];
            }
            s_remaining = rem - cum;
            s_prefix = prefix | (unsigned(d) << shift);
            s_mask = mask | (255u << shift);
        }
        __syncthreads();
    }
    const unsigned thr = s_prefix;
    const unsigned take_eq = s_remaining;            // equal entries to keep
    const unsigned n_less = unsigned(k) - take_eq;
    // entries strictly below the threshold (any order; sorted below)
    for (int64_t c = tid; c < cols; c += 256) {
        const unsigned bits = __float_as_uint(v[c]);
        if (bits < thr) {
            const unsigned slot = atomicAdd(&s_nless, 1u);
            cb[slot] = bits;
            ci[slot] = int(c);
        }
    }
    __syncthreads();
    // equal entries: the first take_eq in column order
    for (int64_t base = 0; base < cols; base += 256) {
        if (s_neq >= take_eq) break;
        const int64_t c = base + tid;
        const bool eq = c < cols && __float_as_uint(v[c]) == thr;
        const unsigned long long bal = __ballot(eq);
        if (lane == 0) wave_cnt[wave] = unsigned(__popcll(bal));
        __syncthreads();
        unsigned before = s_neq;
        for (int w = 0; w < wave; ++w) before += wave_cnt[w];
        before += unsigned(__popcll(bal & ((1ull << lane) - 1ull)));
        if (eq && before < take_eq) {
            cb[n_less + before] = thr;
            ci[n_less + before] = int(c);
        }
        __syncthreads();
        if (tid == 0) s_neq += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        __syncthreads();
    }
    // pad to kTopkMax and bitonic-sort (bits, column)
    for (int t = tid; t < kTopkMax; t += 256)
        if (t >= k) {
            cb[t] = 0xFFFFFFFFu;
            ci[t] = 0x7FFFFFFF;
        }
    __syncthreads();
    for (int size = 2; size <= kTopkMax; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < kTopkMax; t += 256) {
                const int partner = t ^ stride;
                if (partner > t) {
                    const bool up = (t & size) == 0;
                    const bool gt = cb[t] > cb[partner] || (cb[t] == cb[partner] && ci[t] > ci[partner]);
                    if (gt == up) {
                        const unsigned tb = cb[t];
                        cb[t] = cb[partner];
                        cb[partner] = tb;
                        const int tc = ci[t];
                        ci[t] = ci[partner];
                        ci[partner] = tc;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = tid; t < k; t += 256) {
        idx_out[int64_t(blockIdx.x) * k + t] = ci[t];
        if (val_out) val_out[int64_t(blockIdx.x) * k + t] = __uint_as_float(cb[t]);
    }
}

// ----------------------------------------------------------------------------
// Sparse per-sample branch lists (position, l*u in FP64)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sparse_count(Emb e, int64_t* __restrict__ cnt) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256) {
        int64_t c = 0;
        for_each_branch_of_entry(e, ent, a, [&](int32_t) { ++c; });
        cnt[ent] = c;
    }
}

__global__ __launch_bounds__(256) void k_sparse_fill(Emb e, const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ pos,
                                                     double* __restrict__ val) {
    const int64_t s = blockIdx.x;
    const int64_t a = e.row_ptr[s], b = e.row_ptr[s + 1];
    const double inv_t = 1.0 / e.total[s];
    for (int64_t ent = a + threadIdx.x; ent < b; ent += 256) {
        int64_t o = off[ent];
        for_each_branch_of_entry(e, ent, a, [&](int32_t v) {
            const int64_t c = count_in(e.row_ptr, e.rank, e.cum, s, e.lo[v], e.hi[v]);
            pos[o] = v;
            val[o] = e.len[v] * (double(c) * inv_t);
            ++o;
        });
    }
}

__global__ __launch_bounds__(256) void k_rerank(SparseView q, SparseView rf,
                                                const int32_t* __restrict__ qids,
                                                const int32_t* __restrict__ cand, int64_t nq,
                                                int kc, int64_t nb, double* __restrict__ scratch,
                                                double* __restrict__ out) {
    __shared__ double red[256];
    double* row = scratch + int64_t(blockIdx.x) * nb;
    for (int64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int64_t qs = qids[qi];
        const int64_t qa = q.off[qs], qb = q.off[qs + 1];
        for (int64_t t = qa + threadIdx.x; t < qb; t += 256) row[q.pos[t]] = q.val[t];
        __syncthreads();
        for (int c = 0; c < kc; ++c) {
            const int64_t r = cand[qi * kc + c];
            const int64_t ra = rf.off[r], rb = rf.off[r + 1];
            double acc = 0.0;
            for (int64_t t = ra + threadIdx.x; t < rb; t += 256) acc += fmin(row[rf.pos[t]], rf.val[t]);
            red[threadIdx.x] = acc;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                const double den = q.s[qs] + rf.s[r];
                double d = den > 0.0 ? (den - 2.0 * red[0]) / den : 0.0;
                out[qi * kc + c] = fmin(fmax(d, 0.0), 1.0);
            }
            __syncthreads();
        }
        for (int64_t t = qa + threadIdx.x; t < qb; t += 256) row[q.pos[t]] = 0.0;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename V>
__device__ __forceinline__ float cond_at(const V* __restrict__ c, int64_t n, int64_t i, int64_t j) {
    if (i == j) return __builtin_inff();
    const int64_t a = i < j ? i : j, b = i < j ? j : i;
    return float(c[a * n - a * (a + 1) / 2 + (b - a - 1)]);
}

template <typename V>
__global__ __launch_bounds__(256) void k_condensed_block(const V* __restrict__ c, int64_t n,
                                                         int64_t row_off, int64_t n_rows,
                                                         int64_t col_off, int64_t n_cols,
                                                         float* __restrict__ out) {
    const int64_t r = blockIdx.y;
    for (int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x; j < n_cols; j += int64_t(gridDim.x) * 256)
        out[r * n_cols + j] = cond_at(c, n, row_off + r, col_off + j);
}

template <typename V>
__global__ __launch_bounds__(256) void k_gather_pairs(const V* __restrict__ c, int64_t n,
                                                      const int32_t* __restrict__ a,
                                                      const int32_t* __restrict__ b, int64_t cnt,
                                                      float* __restrict__ out) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= cnt) return;
    const float v = cond_at(c, n, a[p], b[p]);
    out[p] = a[p] == b[p] ? 0.0f : v;
}

}  // namespace

// ============================================================================
// launchers
// ============================================================================
hipError_t project(const Emb& e, const int32_t* dims, const int8_t* signs, int per_node,
                   int out_dim, double scale, uint16_t* out, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    const size_t lds = size_t(out_dim) * 8;
    hipLaunchKernelGGL(k_project, dim3(unsigned(e.n)), dim3(256), lds, st, e, dims, signs,
                       per_node, out_dim, scale, out);
    return hipGetLastError();
}

// Launch plan of one GEMM: 256 x 256 tiles when both sides have at least 256
// rows (each wave then runs 64 MFMAs per K step between barriers) and K has
// more than four steps or the tiles fill the CUs; else 256 x 128 while those
// still give every CU a block; else 128 x 128 (two blocks per CU).  K is split into s ranges (s a power of two, every range at least
// four K steps, the partial sums within part_elems floats) for the s of least
// estimated time: rounds of blocks over the CUs' slots times the K steps per
// range, plus, for s > 1, writing and re-reading the s partial matrices.
hipError_t gemm_bf16(int la, int lb, int epi, const uint16_t* A, int64_t lda, const int32_t* arow,
                     const uint16_t* B, int64_t ldb, const int32_t* brow, int64_t M, int64_t N,
                     int64_t K, const float* bias, const uint16_t* mask, int64_t ldm, void* C,
                     int64_t ldc, float* part, int64_t part_elems, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K < 0) return hipErrorInvalidValue;
    // the 16-byte loads: row layout reads 8 consecutive k, column layout 8
    // consecutive rows, from 16-byte aligned storage rows
    auto aligned = [](const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
    if (!aligned(A, 16) || !aligned(B, 16) || lda % 8 || ldb % 8) return hipErrorInvalidValue;
    if ((la == 0 ? K : M) % 8 || (lb == 0 ? K : N) % 8) return hipErrorInvalidValue;
    // the epilogue writes 4 consecutive columns: 16-byte FP32 or 8-byte BF16
    // stores, 16-byte bias and 8-byte mask reads
    const bool f32_out = epi == EPI_F32 || epi == EPI_ACC_F32 || epi == EPI_BIAS_F32;
    if (N % 4 || ldc % 4 || !aligned(C, f32_out ? 16 : 8)) return hipErrorInvalidValue;
    if ((epi == EPI_BIAS_RELU_BF16 || epi == EPI_BIAS_F32) && !aligned(bias, 16))
        return hipErrorInvalidValue;
    if (epi == EPI_MASK_BF16 && (ldm % 4 || !aligned(mask, 8))) return hipErrorInvalidValue;
    if (part && !aligned(part, 16)) return hipErrorInvalidValue;
    const int64_t nk = (K + kGemmKS - 1) / kGemmKS;
    int bm = 128, bn = 128;
    // (with at most four K steps, 256 x 256 tiles would leave CUs idle through
    // the epilogue when they do not fill every CU)
    if (M >= 256 && N >= 256 && (nk > 4 || (M / 256) * (N / 256) >= 256)) bm = bn = 256;
    else if (M >= 256 && (M + 255) / 256 * ((N + 127) / 128) >= 256) bm = 256;
    const int64_t tn = (N + bn - 1) / bn;
    const int64_t tm = (M + bm - 1) / bm;
    const int64_t slots = bm * bn >= 32768 ? 256 : 512;   // blocks resident at once (LDS)
    // Measured on MI355X: a K step of a block takes ~2.3 us at 256 x 256 (~2 us
    // smaller); a block's epilogue stores its tile at ~40 GB/s (4-byte partial
    // sums, or the output's width); the reduction reads the s partial matrices
    // and writes the output at ~6 TB/s.
    const double t_step = bm * bn >= 65536 ? 2.3e-6 : 2.0e-6;
    const double out_b = f32_out ? 4.0 : 2.0;
    auto cost = [&](int64_t s) {
        const int64_t rounds = (tm * tn * s + slots - 1) / slots;
        const double epi = double(bm * bn) * (s > 1 ? 4.0 : out_b) / 40.0e9;
        const double t = double(rounds) * (double((nk + s - 1) / s) * t_step + epi);
        return s > 1 ? t + double(M * N) * (4.0 * double(s) + out_b) / 6.0e12 : t;
    };
    int64_t splits = 1;
    double best = cost(1);
    for (int64_t s = 2; part && nk / s >= 4 && s * M * N <= part_elems; s *= 2)
        if (cost(s) < best) {
            best = cost(s);
            splits = s;
        }
    if (tm * tn > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid{unsigned(tm * tn), 1u, unsigned(splits)};
    // band height of the tile order: the divisor of an XCD's share P nearest
    // sqrt(P), at most tm
    const int64_t per_xcd = (tm * tn + 7) / 8;
    int64_t gh = 1;
    for (int64_t h = 1; h <= std::min(tm, per_xcd); ++h)
        if (per_xcd % h == 0 && std::abs(double(h) - std::sqrt(double(per_xcd))) <
                                    std::abs(double(gh) - std::sqrt(double(per_xcd))))
            gh = h;
    bool launched = false;
#define UF_GEMM_T(LA_, LB_, EPI_, BM_, BN_, NT_)                                                \
    hipLaunchKernelGGL((k_gemm_bf16<LA_, LB_, EPI_, BM_, BN_, NT_>), grid, dim3(NT_), 0, st, A,  \
                       lda, arow, B, ldb, brow, M, N, K, bias, mask, ldm, C, ldc, part, gh)
#define UF_GEMM(LA_, LB_, EPI_)                                                                  \
    if (!launched && la == LA_ && lb == LB_ && epi == EPI_) {                                    \
        if (bn == 256)                                                                           \
            UF_GEMM_T(LA_, LB_, EPI_, 256, 256, 512);                                            \
        else if (bm == 256)                                                                      \
            UF_GEMM_T(LA_, LB_, EPI_, 256, 128, 256);                                            \
        else                                                                                     \
            UF_GEMM_T(LA_, LB_, EPI_, 128, 128, 256);                                            \
        launched = true;                                                                         \
    }
    UF_GEMM(0, 0, EPI_BIAS_RELU_BF16)
    UF_GEMM(0, 0, EPI_BIAS_F32)
    UF_GEMM(0, 0, EPI_F32)
    UF_GEMM(0, 0, EPI_ACC_F32)
    UF_GEMM(0, 1, EPI_MASK_BF16)
    UF_GEMM(0, 1, EPI_F32)
    UF_GEMM(1, 1, EPI_F32)
#undef UF_GEMM
#undef UF_GEMM_T
    if (!launched) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const dim3 rg{unsigned((M * N / 4 + 255) / 256)};
    switch (epi) {
        case EPI_BIAS_RELU_BF16:
            hipLaunchKernelGGL(k_gemm_reduce<EPI_BIAS_RELU_BF16>, rg, dim3(256), 0, st, part,
                               int(splits), M, N, bias, mask, ldm, C, ldc);
            break;
        case EPI_BIAS_F32:
            hipLaunchKernelGGL(k_gemm_reduce<EPI_BIAS_F32>, rg, dim3(256), 0, st, part, int(splits),
                               M, N, bias, mask, ldm, C, ldc);
            break;
        case EPI_ACC_F32:
            hipLaunchKernelGGL(k_gemm_reduce<EPI_ACC_F32>, rg, dim3(256), 0, st, part, int(splits),
                               M, N, bias, mask, ldm, C, ldc);
            break;
        case EPI_MASK_BF16:
            hipLaunchKernelGGL(k_gemm_reduce<EPI_MASK_BF16>, rg, dim3(256), 0, st, part,
                               int(splits), M, N, bias, mask, ldm, C, ldc);
            break;
        default:
            hipLaunchKernelGGL(k_gemm_reduce<EPI_F32>, rg, dim3(256), 0, st, part, int(splits), M, N,
                               bias, mask, ldm, C, ldc);
    }
    return hipGetLastError();
}

hipError_t colsum_bf16(const uint16_t* X, int64_t rows, int64_t cols, double* part,
                       int64_t part_elems, float* out, hipStream_t st) {
    if (cols <= 0) return hipSuccess;
    if (rows < 0 || !part || part_elems < cols || cols % 8 ||
        (reinterpret_cast<uintptr_t>(X) & 15u))
        return hipErrorInvalidValue;
    const int64_t groups = cols / 8;
    const int64_t G = groups < 256 ? groups : 256;
    const int64_t gx = (groups + G - 1) / G;
    // about kColsumChunks chunks of at least 16 rows, as far as part holds them
    int64_t chunks = std::min<int64_t>(kColsumChunks, std::max<int64_t>(rows / 16, 1));
    while (chunks > 1 && chunks * cols > part_elems) chunks /= 2;
    const int64_t chunk = std::max<int64_t>((rows + chunks - 1) / chunks, 1);
    chunks = std::max<int64_t>((rows + chunk - 1) / chunk, 1);
    if (gx > 0x7fffffff || chunks > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colsum_part, dim3(unsigned(gx), unsigned(chunks)), dim3(256), 0, st, X,
                       rows, cols, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum_final, dim3(unsigned((cols + 31) / 32)), dim3(256), 0, st, part,
                       int(chunks), cols, out);
    return hipGetLastError();
}

hipError_t pairloss(const float* Z, int64_t P, int D, const float* target, float rel_floor,
                    uint16_t* dZ, float* loss_per_pair, float* loss_mean, hipStream_t st) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairloss, dim3(unsigned((P + 3) / 4)), dim3(256), 0, st, Z, P, D, target,
                       rel_floor, dZ, loss_per_pair);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, loss_per_pair, P, loss_mean);
    return hipGetLastError();
}

hipError_t tripletloss(const float* Z, int64_t T, int D, const float* d_near, const float* d_far,
                       float alpha, float lam, float tau, uint16_t* dZ, float* loss_per_triple,
                       float* loss_mean, hipStream_t st) {
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tripletloss, dim3(unsigned((T + 3) / 4)), dim3(256), 0, st, Z, T, D, d_near,
                       d_far, alpha, lam, tau, dZ, loss_per_triple);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, loss_per_triple, T, loss_mean);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, float wd, uint16_t* pbf, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr,
                       b1, b2, eps, bc1, bc2, wd, pbf);
    return hipGetLastError();
}

hipError_t adam_multi(const AdamTensor* ts, int count, float lr, float b1, float b2, float eps,
                      float bc1, float bc2, hipStream_t st) {
    if (count < 0 || count > kAdamMaxTensors) return hipErrorInvalidValue;
    AdamBatch ab{};
    ab.count = count;
    ab.start[0] = 0;
    auto al = [](const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
    for (int k = 0; k < count; ++k) {
        if (ts[k].n < 0) return hipErrorInvalidValue;
        ab.t[k] = ts[k];
        ab.t[k].vec = ts[k].n % 4 == 0 && al(ts[k].p, 16) && al(ts[k].g, 16) && al(ts[k].m, 16) &&
                      al(ts[k].v, 16) && al(ts[k].pbf, 8);
        ab.start[k + 1] = ab.start[k] + (ts[k].n + 3) / 4;
    }
    const int64_t groups = ab.start[count];
    if (groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam_multi, dim3(unsigned((groups + 255) / 256)), dim3(256), 0, st, ab, lr,
                       b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t f32_to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}

hipError_t sqdist(const float* A, int64_t na, const float* B, int64_t nb, int64_t D, float* out,
                  hipStream_t st) {
    if (na <= 0 || nb <= 0) return hipSuccess;
    if ((na + kSqT - 1) / kSqT > 65535 || (nb + kSqT - 1) / kSqT > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sqdist, dim3(unsigned((nb + kSqT - 1) / kSqT), unsigned((na + kSqT - 1) / kSqT)),
                       dim3(256), 0, st, A, na, B, nb, D, out);
    return hipGetLastError();
}

hipError_t topk_rows(const float* vals, int64_t rows, int64_t cols, int k, int32_t* idx,
                     float* val, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (k < 1 || k > kTopkMax || cols < k || rows > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_topk_rows, dim3(unsigned(rows)), dim3(256), 0, st, vals, cols, k, idx, val);
    return hipGetLastError();
}

hipError_t sparse_count(const Emb& e, int64_t* cnt, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_count, dim3(unsigned(e.n)), dim3(256), 0, st, e, cnt);
    return hipGetLastError();
}

hipError_t sparse_fill(const Emb& e, const int64_t* off, int32_t* pos, double* val, hipStream_t st) {
    if (e.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_fill, dim3(unsigned(e.n)), dim3(256), 0, st, e, off, pos, val);
    return hipGetLastError();
}

hipError_t rerank(const SparseView& q, const SparseView& r, const int32_t* qids,
                  const int32_t* cand, int64_t nq, int kc, int64_t nb, double* scratch,
                  int64_t n_rows, double* out, hipStream_t st) {
    if (nq <= 0 || kc <= 0) return hipSuccess;
    const int64_t grid = nq < n_rows ? nq : n_rows;
    hipLaunchKernelGGL(k_rerank, dim3(unsigned(grid)), dim3(256), 0, st, q, r, qids, cand, nq, kc,
                       nb, scratch, out);
    return hipGetLastError();
}

hipError_t zero_f64(double* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t condensed_block(const void* c, int is_f32, int64_t n, int64_t row_off, int64_t n_rows,
                           int64_t col_off, int64_t n_cols, float* out, hipStream_t st) {
    if (n_rows <= 0 || n_cols <= 0) return hipSuccess;
    if (n_rows > 65535) return hipErrorInvalidValue;
    const int64_t gx = (n_cols + 255) / 256 < 64 ? (n_cols + 255) / 256 : 64;
    if (is_f32)
        hipLaunchKernelGGL(k_condensed_block<float>, dim3(unsigned(gx), unsigned(n_rows)), dim3(256),
                           0, st, static_cast<const float*>(c), n, row_off, n_rows, col_off, n_cols, out);
    else
        hipLaunchKernelGGL(k_condensed_block<double>, dim3(unsigned(gx), unsigned(n_rows)), dim3(256),
                           0, st, static_cast<const double*>(c), n, row_off, n_rows, col_off, n_cols, out);
    return hipGetLastError();
}

hipError_t gather_pairs(const void* c, int is_f32, int64_t n, const int32_t* a, const int32_t* b,
                        int64_t cnt, float* out, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    if (is_f32)
        hipLaunchKernelGGL(k_gather_pairs<float>, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, st,
                           static_cast<const float*>(c), n, a, b, cnt, out);
    else
        hipLaunchKernelGGL(k_gather_pairs<double>, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, st,
                           static_cast<const double*>(c), n, a, b, cnt, out);
    return hipGetLastError();
}

}  // namespace ufp
