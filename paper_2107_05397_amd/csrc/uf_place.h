// Internal declarations of the placement-encoder kernels (uf_place.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ufp {

constexpr int kTopkMax = 128;   // largest k of the top-k kernel
enum { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_BIAS_F32 = 2, EPI_MASK_BF16 = 3, EPI_BF16 = 4,
       EPI_ACC_F32 = 5 };

// Device view of an embedding's table and tree arrays (passed by value).
struct Emb {
    int64_t n;
    const int64_t* row_ptr;
    const int32_t* rank;
    const int64_t* cum;
    const double* total;
    const int32_t* lo;
    const int32_t* hi;
    const double* len;
    const int32_t* parent_pos;
    const int32_t* tip_pos;
    int32_t root_pos;
};

// Per-sample lists of nonzero branches: sample s owns [off[s], off[s+1]).
struct SparseView {
    const int64_t* off;
    const int32_t* pos;
    const double* val;   // l_v * u_sv
    const double* s;     // per-sample sum_v l_v u_sv
};

hipError_t project(const Emb& e, const int32_t* dims, const int8_t* signs, int per_node,
                   int out_dim, double scale, uint16_t* out, hipStream_t st);
// la/lb: 0 = row layout (k contiguous), 1 = column layout (row index contiguous).
// part: device FP32 scratch of part_elems floats for split-K partial sums
// (nullable: no split; 16-byte aligned).  Requires 16-byte aligned A and B, lda
// and ldb multiples of 8, the contiguous extent of each operand (K for the row
// layout, M or N for the column layout) a multiple of 8, and for the epilogue's
// 4-column stores N and ldc multiples of 4, C 16-byte (FP32 outputs) or 8-byte
// (BF16) aligned, bias 16-byte aligned, mask 8-byte aligned with ldm a multiple
// of 4.  Other arguments give hipErrorInvalidValue.
hipError_t gemm_bf16(int la, int lb, int epi, const uint16_t* A, int64_t lda, const int32_t* arow,
                     const uint16_t* B, int64_t ldb, const int32_t* brow, int64_t M, int64_t N,
                     int64_t K, const float* bias, const uint16_t* mask, int64_t ldm, void* C,
                     int64_t ldc, float* part, int64_t part_elems, hipStream_t st);
// Column sums of a BF16 [rows][cols] matrix in FP64, fixed order; part: device
// FP64 scratch of part_elems (>= cols) doubles.  cols a multiple of 8 and X
// 16-byte aligned (16-byte loads), else hipErrorInvalidValue.
hipError_t colsum_bf16(const uint16_t* X, int64_t rows, int64_t cols, double* part,
                       int64_t part_elems, float* out, hipStream_t st);
hipError_t pairloss(const float* Z, int64_t P, int D, const float* target, float rel_floor,
                    uint16_t* dZ, float* loss_per_pair, float* loss_mean, hipStream_t st);
// Ranking loss over T triples (rows: anchors, near ends, far ends of Z [3T][D]).
hipError_t tripletloss(const float* Z, int64_t T, int D, const float* d_near, const float* d_far,
                       float alpha, float lam, float tau, uint16_t* dZ, float* loss_per_triple,
                       float* loss_mean, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, float wd, uint16_t* pbf, hipStream_t st);
// Adam / AdamW over up to kAdamMaxTensors tensors in one launch (per tensor: FP32
// parameters p, gradient g, moments m and v, n elements, decoupled weight decay wd,
// optional BF16 copy pbf).
constexpr int kAdamMaxTensors = 20;
struct AdamTensor {
    float* p;
    const float* g;
    float* m;
    float* v;
    uint16_t* pbf;
    int64_t n;
    float wd;
    bool vec;   // set by adam_multi: 16-byte accesses allowed
};
struct AdamBatch {
    AdamTensor t[kAdamMaxTensors];
    int64_t start[kAdamMaxTensors + 1];   // first 4-element group of each tensor
    int count;
};
hipError_t adam_multi(const AdamTensor* ts, int count, float lr, float b1, float b2, float eps,
                      float bc1, float bc2, hipStream_t st);
hipError_t f32_to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st);
hipError_t sqdist(const float* A, int64_t na, const float* B, int64_t nb, int64_t D, float* out,
                  hipStream_t st);
hipError_t topk_rows(const float* vals, int64_t rows, int64_t cols, int k, int32_t* idx,
                     float* val, hipStream_t st);
hipError_t sparse_count(const Emb& e, int64_t* cnt, hipStream_t st);
hipError_t sparse_fill(const Emb& e, const int64_t* off, int32_t* pos, double* val, hipStream_t st);
hipError_t rerank(const SparseView& q, const SparseView& r, const int32_t* qids,
                  const int32_t* cand, int64_t nq, int kc, int64_t nb, double* scratch,
                  int64_t n_rows, double* out, hipStream_t st);
hipError_t zero_f64(double* p, int64_t n, hipStream_t st);
hipError_t condensed_block(const void* c, int is_f32, int64_t n, int64_t row_off, int64_t n_rows,
                           int64_t col_off, int64_t n_cols, float* out, hipStream_t st);
hipError_t gather_pairs(const void* c, int is_f32, int64_t n, const int32_t* a, const int32_t* b,
                        int64_t cnt, float* out, hipStream_t st);

}  // namespace ufp
