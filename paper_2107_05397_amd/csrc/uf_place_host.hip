// Host side of the learned placement encoder: the C ABI of uf.h's placement
// section (projection, MLP training and inference, kNN, exact re-rank).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "uf_internal.h"
#include "uf_place.h"

using ufh::check_device;
using ufh::fail;
using ufh::hip_fail;

#define UF_HIP(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hip_fail(e_, #call);       \
    } while (0)

namespace {

template <class F>
uf_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(UF_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(UF_ERR_ARG, "unexpected error");
    }
}

ufp::Emb view(const uf_embedding& e) {
    ufp::Emb v;
    v.n = e.n;
    v.row_ptr = e.row_ptr;
    v.rank = e.rank;
    v.cum = e.cum;
    v.total = e.total;
    v.lo = e.lo;
    v.hi = e.hi;
    v.len = e.len;
    v.parent_pos = e.parent_pos;
    v.tip_pos = e.tip_pos;
    v.root_pos = int32_t(e.nb);
    return v;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct uf_mlp {
    int64_t L = 0;                    // layers
    std::vector<int64_t> dims;        // L + 1
    int64_t max_rows = 0;
    void* arena = nullptr;
    std::vector<float*> W, b, gW, gb, mW, vW, mb, vb;
    std::vector<uint16_t*> Wbf;
    std::vector<uint16_t*> H;         // hidden activations, layers 1..L-1 (index l)
    std::vector<uint16_t*> dA;        // gradients w.r.t. hidden activations
    float* Z = nullptr;               // [max_rows][dims[L]]
    uint16_t* dZ = nullptr;
    float* loss_pp = nullptr;
    int32_t* rows = nullptr;          // [max_rows]
    float* part = nullptr;            // split-K partial sums / column-sum chunks
    int64_t part_elems = 0;           // floats in part
    // optional linear path z += S x (S: [dims[L]][dims[0]])
    bool skip = false;
    float *S = nullptr, *gS = nullptr, *mS = nullptr, *vS = nullptr;
    uint16_t* Sbf = nullptr;
    ~uf_mlp() {
        if (arena) (void)hipFree(arena);
    }
};

struct uf_sparse {
    int64_t n = 0, nb = 0, nnz = 0;
    void* arena = nullptr;
    int64_t* off = nullptr;
    int32_t* pos = nullptr;
    double* val = nullptr;
    double* s = nullptr;
    ~uf_sparse() {
        if (arena) (void)hipFree(arena);
    }
    ufp::SparseView view() const { return ufp::SparseView{off, pos, val, s}; }
};

extern "C" {

// ------------------------------------------------------------------ projection
uf_status uf_project(const uf_tree* tree, const uf_embedding* emb, const int32_t* dims,
                     const int8_t* signs, int64_t per_node, int64_t out_dim, double scale,
                     void* out_bf16,
                     void* stream) {
    return guarded([&]() -> uf_status {
        if (!tree || !emb || !dims || !signs || !out_bf16) return fail(UF_ERR_ARG, "NULL argument");
        if (per_node < 1 || per_node > 16 || out_dim < 1 || out_dim > 8192)
            return fail(UF_ERR_ARG, "per_node must be 1..16 and out_dim 1..8192");
        if (tree->n_nodes - 1 != emb->nb) return fail(UF_ERR_ARG, "embedding was built on another tree");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        const int64_t m = tree->n_nodes;
        // re-index (node id -> postorder position); the root's row is never read
        std::vector<int32_t> pd(size_t(m * per_node));
        std::vector<int8_t> ps(size_t(m * per_node));
        for (int64_t k = 0; k < m; ++k) {
            const int64_t v = tree->node_at[k];
            for (int64_t j = 0; j < per_node; ++j) {
                const int32_t d = dims[v * per_node + j];
                if (d < 0 || d >= out_dim) return fail(UF_ERR_ARG, "projection dim out of range");
                pd[size_t(k * per_node + j)] = d;
                ps[size_t(k * per_node + j)] = signs[v * per_node + j];
            }
        }
        void* buf = nullptr;
        const size_t bd = align256(pd.size() * 4);
        if (hipMalloc(&buf, bd + ps.size() + 256) != hipSuccess) return fail(UF_ERR_NOMEM, "projection");
        std::unique_ptr<void, void (*)(void*)> g(buf, [](void* p) { (void)hipFree(p); });
        int32_t* ddims = static_cast<int32_t*>(buf);
        int8_t* dsigns = reinterpret_cast<int8_t*>(static_cast<char*>(buf) + bd);
        UF_HIP(hipMemcpy(ddims, pd.data(), pd.size() * 4, hipMemcpyHostToDevice));
        UF_HIP(hipMemcpy(dsigns, ps.data(), ps.size(), hipMemcpyHostToDevice));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (!(scale > 0.0) || !std::isfinite(scale)) return fail(UF_ERR_ARG, "scale must be positive");
        UF_HIP(ufp::project(view(*emb), ddims, dsigns, int(per_node), int(out_dim), scale,
                            static_cast<uint16_t*>(out_bf16), s));
        UF_HIP(hipStreamSynchronize(s));   // the index buffers are freed on return
        return UF_OK;
    });
}

// ------------------------------------------------------------------ MLP
uf_status uf_mlp_create(int64_t n_layers, const int64_t* dims, int64_t max_rows, int skip,
                        uf_mlp** out) {
    return guarded([&]() -> uf_status {
        if (!out || !dims || n_layers < 1 || n_layers > 8 || max_rows < 2)
            return fail(UF_ERR_ARG, "need 1..8 layers, dims and max_rows >= 2");
        *out = nullptr;
        for (int64_t l = 0; l <= n_layers; ++l)
            if (dims[l] < 32 || dims[l] % 32 != 0 || dims[l] > 65536)
                return fail(UF_ERR_ARG, "every width must be a positive multiple of 32");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        auto m = new uf_mlp();
        std::unique_ptr<uf_mlp> guard(m);
        m->L = n_layers;
        m->dims.assign(dims, dims + n_layers + 1);
        m->max_rows = max_rows;
        size_t total = 0;
        std::vector<size_t> offs;
        auto take = [&](size_t bytes) {
            offs.push_back(total);
            total += align256(bytes);
        };
        for (int64_t l = 0; l < n_layers; ++l) {
            const size_t nw = size_t(dims[l + 1] * dims[l]), nbias = size_t(dims[l + 1]);
            take(nw * 4); take(nbias * 4); take(nw * 4); take(nbias * 4);   // W b gW gb
            take(nw * 4); take(nw * 4); take(nbias * 4); take(nbias * 4);   // mW vW mb vb
            take(nw * 2);                                                    // Wbf
        }
        for (int64_t l = 1; l < n_layers; ++l) {
            take(size_t(max_rows * dims[l]) * 2);   // H
            take(size_t(max_rows * dims[l]) * 2);   // dA
        }
        take(size_t(max_rows * dims[n_layers]) * 4);   // Z
        take(size_t(max_rows * dims[n_layers]) * 2);   // dZ
        take(size_t(max_rows) * 4);                    // loss per pair
        take(size_t(max_rows) * 4);                    // rows
        const int64_t part_elems = int64_t(32) << 20;  // 128 MiB of GEMM / column-sum scratch
        take(size_t(part_elems) * 4);                  // part
        m->skip = skip != 0;
        const size_t ns = m->skip ? size_t(dims[n_layers] * dims[0]) : 0;
        take(ns * 4); take(ns * 4); take(ns * 4); take(ns * 4); take(ns * 2);   // S gS mS vS Sbf
        if (hipMalloc(&m->arena, total + 256) != hipSuccess) return fail(UF_ERR_NOMEM, "MLP buffers");
        UF_HIP(hipMemset(m->arena, 0, total));
        char* base = static_cast<char*>(m->arena);
        size_t k = 0;
        for (int64_t l = 0; l < n_layers; ++l) {
            m->W.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->b.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->gW.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->gb.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->mW.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->vW.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->mb.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->vb.push_back(reinterpret_cast<float*>(base + offs[k++]));
            m->Wbf.push_back(reinterpret_cast<uint16_t*>(base + offs[k++]));
        }
        m->H.assign(size_t(n_layers), nullptr);
        m->dA.assign(size_t(n_layers), nullptr);
        for (int64_t l = 1; l < n_layers; ++l) {
            m->H[size_t(l)] = reinterpret_cast<uint16_t*>(base + offs[k++]);
            m->dA[size_t(l)] = reinterpret_cast<uint16_t*>(base + offs[k++]);
        }
        m->Z = reinterpret_cast<float*>(base + offs[k++]);
        m->dZ = reinterpret_cast<uint16_t*>(base + offs[k++]);
        m->loss_pp = reinterpret_cast<float*>(base + offs[k++]);
        m->rows = reinterpret_cast<int32_t*>(base + offs[k++]);
        m->part = reinterpret_cast<float*>(base + offs[k++]);
        m->part_elems = part_elems;
        if (m->skip) {
            m->S = reinterpret_cast<float*>(base + offs[k]);
            m->gS = reinterpret_cast<float*>(base + offs[k + 1]);
            m->mS = reinterpret_cast<float*>(base + offs[k + 2]);
            m->vS = reinterpret_cast<float*>(base + offs[k + 3]);
            m->Sbf = reinterpret_cast<uint16_t*>(base + offs[k + 4]);
        }
        *out = guard.release();
        return UF_OK;
    });
}

uf_status uf_mlp_set(uf_mlp* m, int64_t layer, const float* w, const float* b, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || layer < 0 || layer > m->L || (layer == m->L && !m->skip))
            return fail(UF_ERR_ARG, "bad MLP or layer");
        hipStream_t s = static_cast<hipStream_t>(stream);
        // work already queued on the stream may still read the parameters
        UF_HIP(hipStreamSynchronize(s));
        if (layer == m->L) {   // the linear path S
            const size_t ns = size_t(m->dims[m->L] * m->dims[0]);
            if (w) {
                UF_HIP(hipMemcpyAsync(m->S, w, ns * 4, hipMemcpyHostToDevice, s));
                UF_HIP(ufp::f32_to_bf16(m->S, int64_t(ns), m->Sbf, s));
            }
            UF_HIP(hipStreamSynchronize(s));
            return UF_OK;
        }
        const size_t nw = size_t(m->dims[layer + 1] * m->dims[layer]), nb = size_t(m->dims[layer + 1]);
        if (w) {
            UF_HIP(hipMemcpyAsync(m->W[layer], w, nw * 4, hipMemcpyHostToDevice, s));
            UF_HIP(ufp::f32_to_bf16(m->W[layer], int64_t(nw), m->Wbf[layer], s));
        }
        if (b) UF_HIP(hipMemcpyAsync(m->b[layer], b, nb * 4, hipMemcpyHostToDevice, s));
        UF_HIP(hipStreamSynchronize(s));   // the host arrays may be freed on return
        return UF_OK;
    });
}

uf_status uf_mlp_get(const uf_mlp* m, int64_t layer, int what, float* w, float* b, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || layer < 0 || layer > m->L || (layer == m->L && !m->skip) || what < 0 || what > 3)
            return fail(UF_ERR_ARG, "bad MLP, layer or selector");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (layer == m->L) {
            const size_t ns = size_t(m->dims[m->L] * m->dims[0]);
            const float* ss[4] = {m->S, m->gS, m->mS, m->vS};
            if (w) UF_HIP(hipMemcpyAsync(w, ss[what], ns * 4, hipMemcpyDeviceToHost, s));
            UF_HIP(hipStreamSynchronize(s));
            return UF_OK;
        }
        const size_t nw = size_t(m->dims[layer + 1] * m->dims[layer]), nb = size_t(m->dims[layer + 1]);
        const float* sw[4] = {m->W[layer], m->gW[layer], m->mW[layer], m->vW[layer]};
        const float* sb[4] = {m->b[layer], m->gb[layer], m->mb[layer], m->vb[layer]};
        if (w) UF_HIP(hipMemcpyAsync(w, sw[what], nw * 4, hipMemcpyDeviceToHost, s));
        if (b) UF_HIP(hipMemcpyAsync(b, sb[what], nb * 4, hipMemcpyDeviceToHost, s));
        UF_HIP(hipStreamSynchronize(s));
        return UF_OK;
    });
}

namespace {
// One GEMM of the MLP with its split-K scratch, timed as "encoder_gemm" while
// profiling is enabled.
hipError_t mlp_gemm(const uf_mlp* m, int la, int lb, int epi, const uint16_t* A, int64_t lda,
                    const int32_t* arow, const uint16_t* B, int64_t ldb, const int32_t* brow,
                    int64_t M, int64_t N, int64_t K, const float* bias, const uint16_t* mask,
                    int64_t ldm, void* C, int64_t ldc, hipStream_t s) {
    ufh::ProfGuard pg("encoder_gemm", s);
    return ufp::gemm_bf16(la, lb, epi, A, lda, arow, B, ldb, brow, M, N, K, bias, mask, ldm, C, ldc,
                          m->part, m->part_elems, s);
}

uf_status mlp_forward(uf_mlp* m, const uint16_t* x, int64_t ldx, const int32_t* rows, int64_t n,
                      float* z, hipStream_t s) {
    const uint16_t* in = x;
    int64_t ld = ldx;
    const int32_t* r = rows;
    for (int64_t l = 0; l < m->L; ++l) {
        const int64_t din = m->dims[l], dout = m->dims[l + 1];
        if (l < m->L - 1) {
            UF_HIP(mlp_gemm(m, 0, 0, ufp::EPI_BIAS_RELU_BF16, in, ld, r, m->Wbf[l], din, nullptr, n,
                            dout, din, m->b[l], nullptr, 0, m->H[l + 1], dout, s));
            in = m->H[l + 1];
            ld = dout;
            r = nullptr;
        } else {
            UF_HIP(mlp_gemm(m, 0, 0, ufp::EPI_BIAS_F32, in, ld, r, m->Wbf[l], din, nullptr, n, dout,
                            din, m->b[l], nullptr, 0, z, dout, s));
        }
    }
    if (m->skip)   // z += x S^T
        UF_HIP(mlp_gemm(m, 0, 0, ufp::EPI_ACC_F32, x, ldx, rows, m->Sbf, m->dims[0], nullptr, n,
                        m->dims[m->L], m->dims[0], nullptr, nullptr, 0, z, m->dims[m->L], s));
    return UF_OK;
}
}  // namespace

uf_status uf_mlp_forward(uf_mlp* m, const void* x_bf16, int64_t ldx, const int32_t* rows, int64_t n,
                         float* z, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || !x_bf16 || !z || n < 0) return fail(UF_ERR_ARG, "NULL argument");
        if (ldx < m->dims[0] || ldx % 8 != 0) return fail(UF_ERR_ARG, "ldx must be >= d0 and a multiple of 8");
        if (n > m->max_rows) return fail(UF_ERR_ARG, "more rows than max_rows");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        return mlp_forward(m, static_cast<const uint16_t*>(x_bf16), ldx, rows, n, z,
                           static_cast<hipStream_t>(stream));
    });
}

namespace {
// Gradients of every parameter from dZ (BF16 [n][dL]) for the n rows of the
// preceding forward pass (x, ldx, rows as given to it; its hidden activations are
// still held in m->H).
uf_status mlp_backward(uf_mlp* m, const uint16_t* x, int64_t ldx, const int32_t* rows, int64_t n,
                       const uint16_t* dz, hipStream_t s) {
    const int64_t L = m->L;
    if (m->skip)   // dS = dZ^T x
        UF_HIP(mlp_gemm(m, 1, 1, ufp::EPI_F32, dz, m->dims[L], nullptr, x, ldx, rows,
                        m->dims[L], m->dims[0], n, nullptr, nullptr, 0, m->gS, m->dims[0], s));
    const uint16_t* g = dz;
    for (int64_t l = L - 1; l >= 0; --l) {
        const int64_t din = m->dims[l], dout = m->dims[l + 1];
        // dW_l = g^T h_{l}: A = g (column layout), B = input of layer l (column layout)
        const uint16_t* hin = l == 0 ? x : m->H[l];
        const int64_t ldh = l == 0 ? ldx : din;
        UF_HIP(mlp_gemm(m, 1, 1, ufp::EPI_F32, g, dout, nullptr, hin, ldh, l == 0 ? rows : nullptr,
                        dout, din, n, nullptr, nullptr, 0, m->gW[l], din, s));
        {
            ufh::ProfGuard pc("encoder_colsum", s);
            UF_HIP(ufp::colsum_bf16(g, n, dout, reinterpret_cast<double*>(m->part),
                                    m->part_elems / 2, m->gb[l], s));
        }
        if (l > 0) {
            // dA_l = (g W_l) * [h_l > 0]: A = g (row), B = W_l (column layout)
            UF_HIP(mlp_gemm(m, 0, 1, ufp::EPI_MASK_BF16, g, dout, nullptr, m->Wbf[l], din, nullptr,
                            n, din, dout, nullptr, m->H[l], din, m->dA[l], din, s));
            g = m->dA[l];
        }
    }
    return UF_OK;
}
}  // namespace

uf_status uf_mlp_backward(uf_mlp* m, const void* x_bf16, int64_t ldx, const int32_t* rows,
                          int64_t n, const void* dz_bf16, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || !x_bf16 || !dz_bf16 || n < 1) return fail(UF_ERR_ARG, "NULL argument or no rows");
        if (n > m->max_rows) return fail(UF_ERR_ARG, "more rows than max_rows");
        if (ldx < m->dims[0] || ldx % 8 != 0) return fail(UF_ERR_ARG, "ldx must be >= d0 and a multiple of 8");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        return mlp_backward(m, static_cast<const uint16_t*>(x_bf16), ldx, rows, n,
                            static_cast<const uint16_t*>(dz_bf16), static_cast<hipStream_t>(stream));
    });
}

uf_status uf_mlp_loss_grad(uf_mlp* m, const void* x_bf16, int64_t ldx, const int32_t* pair_a,
                           const int32_t* pair_b, const float* target, int64_t n_pairs,
                           float rel_floor, float* loss, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || !x_bf16 || !pair_a || !pair_b || !target || !loss || n_pairs < 1)
            return fail(UF_ERR_ARG, "NULL argument or no pairs");
        if (2 * n_pairs > m->max_rows) return fail(UF_ERR_ARG, "2 * n_pairs exceeds max_rows");
        if (ldx < m->dims[0] || ldx % 8 != 0) return fail(UF_ERR_ARG, "ldx must be >= d0 and a multiple of 8");
        if (!(rel_floor >= 0.0f)) return fail(UF_ERR_ARG, "rel_floor must be >= 0");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint16_t* x = static_cast<const uint16_t*>(x_bf16);
        const int64_t R = 2 * n_pairs, L = m->L;
        UF_HIP(hipMemcpyAsync(m->rows, pair_a, size_t(n_pairs) * 4, hipMemcpyDeviceToDevice, s));
        UF_HIP(hipMemcpyAsync(m->rows + n_pairs, pair_b, size_t(n_pairs) * 4, hipMemcpyDeviceToDevice, s));
        st = mlp_forward(m, x, ldx, m->rows, R, m->Z, s);
        if (st != UF_OK) return st;
        {
            ufh::ProfGuard pl("encoder_loss", s);
            UF_HIP(ufp::pairloss(m->Z, n_pairs, int(m->dims[L]), target, rel_floor, m->dZ,
                                 m->loss_pp, loss, s));
        }
        return mlp_backward(m, x, ldx, m->rows, R, m->dZ, s);
    });
}

uf_status uf_mlp_triplet_loss_grad(uf_mlp* m, const void* x_bf16, int64_t ldx,
                                   const int32_t* anchor, const int32_t* near, const int32_t* far,
                                   const float* d_near, const float* d_far, int64_t n_triples,
                                   float dist_weight, float rank_weight, float tau, float* loss,
                                   void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || !x_bf16 || !anchor || !near || !far || !d_near || !d_far || !loss ||
            n_triples < 1)
            return fail(UF_ERR_ARG, "NULL argument or no triples");
        if (3 * n_triples > m->max_rows) return fail(UF_ERR_ARG, "3 * n_triples exceeds max_rows");
        if (ldx < m->dims[0] || ldx % 8 != 0) return fail(UF_ERR_ARG, "ldx must be >= d0 and a multiple of 8");
        if (!(dist_weight >= 0.0f) || !(rank_weight >= 0.0f) || !(tau > 0.0f))
            return fail(UF_ERR_ARG, "need dist_weight >= 0, rank_weight >= 0 and tau > 0");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint16_t* x = static_cast<const uint16_t*>(x_bf16);
        const int64_t T = n_triples, R = 3 * T, L = m->L;
        UF_HIP(hipMemcpyAsync(m->rows, anchor, size_t(T) * 4, hipMemcpyDeviceToDevice, s));
        UF_HIP(hipMemcpyAsync(m->rows + T, near, size_t(T) * 4, hipMemcpyDeviceToDevice, s));
        UF_HIP(hipMemcpyAsync(m->rows + 2 * T, far, size_t(T) * 4, hipMemcpyDeviceToDevice, s));
        st = mlp_forward(m, x, ldx, m->rows, R, m->Z, s);
        if (st != UF_OK) return st;
        {
            ufh::ProfGuard pl("encoder_loss", s);
            UF_HIP(ufp::tripletloss(m->Z, T, int(m->dims[L]), d_near, d_far, dist_weight, rank_weight,
                                    tau, m->dZ, m->loss_pp, loss, s));
        }
        return mlp_backward(m, x, ldx, m->rows, R, m->dZ, s);
    });
}

uf_status uf_mlp_adam(uf_mlp* m, float lr, float beta1, float beta2, float eps,
                      float weight_decay, int64_t step, void* stream) {
    return guarded([&]() -> uf_status {
        if (!m || step < 1 || !(weight_decay >= 0.0f)) return fail(UF_ERR_ARG, "bad MLP, step or decay");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const float bc1 = float(1.0 - std::pow(double(beta1), double(step)));
        const float bc2 = float(1.0 - std::pow(double(beta2), double(step)));
        ufh::ProfGuard pa("encoder_adam", s);
        // every weight, bias and the linear path in one launch
        std::vector<ufp::AdamTensor> ts;
        for (int64_t l = 0; l < m->L; ++l) {
            ts.push_back({m->W[l], m->gW[l], m->mW[l], m->vW[l], m->Wbf[l],
                          m->dims[l + 1] * m->dims[l], weight_decay});
            ts.push_back({m->b[l], m->gb[l], m->mb[l], m->vb[l], nullptr, m->dims[l + 1], 0.0f});
        }
        if (m->skip)
            ts.push_back({m->S, m->gS, m->mS, m->vS, m->Sbf, m->dims[m->L] * m->dims[0], weight_decay});
        UF_HIP(ufp::adam_multi(ts.data(), int(ts.size()), lr, beta1, beta2, eps, bc1, bc2, s));
        return UF_OK;
    });
}

uf_status uf_adam_step(uf_mlp* m, float lr, float beta1, float beta2, float eps, int64_t step,
                       void* stream) {
    return uf_mlp_adam(m, lr, beta1, beta2, eps, 0.0f, step, stream);
}

void uf_free_mlp(uf_mlp* m) { delete m; }

// ------------------------------------------------------------------ kNN helpers
uf_status uf_sqdist(const float* a, int64_t na, const float* b, int64_t nb, int64_t dim, float* out,
                    void* stream) {
    return guarded([&]() -> uf_status {
        if (!a || !b || !out || na < 0 || nb < 0 || dim < 1) return fail(UF_ERR_ARG, "bad argument");
        UF_HIP(ufp::sqdist(a, na, b, nb, dim, out, static_cast<hipStream_t>(stream)));
        return UF_OK;
    });
}

uf_status uf_topk_rows(const float* values, int64_t rows, int64_t cols, int64_t k, int32_t* idx,
                       float* vals, void* stream) {
    return guarded([&]() -> uf_status {
        if (!values || !idx || rows < 0) return fail(UF_ERR_ARG, "bad argument");
        if (k < 1 || k > ufp::kTopkMax || cols < k) return fail(UF_ERR_ARG, "need 1 <= k <= 128 and k <= cols");
        UF_HIP(ufp::topk_rows(values, rows, cols, int(k), idx, vals, static_cast<hipStream_t>(stream)));
        return UF_OK;
    });
}

uf_status uf_condensed_block(const void* cond, uf_out_dtype dtype, int64_t n, int64_t row_off,
                             int64_t n_rows, int64_t col_off, int64_t n_cols, float* out,
                             void* stream) {
    return guarded([&]() -> uf_status {
        if (!cond || !out) return fail(UF_ERR_ARG, "NULL argument");
        if (row_off < 0 || col_off < 0 || n_rows < 0 || n_cols < 0 || row_off + n_rows > n ||
            col_off + n_cols > n)
            return fail(UF_ERR_RANGE, "block outside the matrix");
        UF_HIP(ufp::condensed_block(cond, dtype == UF_OUT_F32, n, row_off, n_rows, col_off, n_cols, out,
                                    static_cast<hipStream_t>(stream)));
        return UF_OK;
    });
}

uf_status uf_gather_pairs(const void* cond, uf_out_dtype dtype, int64_t n, const int32_t* a,
                          const int32_t* b, int64_t count, float* out, void* stream) {
    return guarded([&]() -> uf_status {
        if (!cond || !a || !b || !out || count < 0) return fail(UF_ERR_ARG, "bad argument");
        UF_HIP(ufp::gather_pairs(cond, dtype == UF_OUT_F32, n, a, b, count, out,
                                 static_cast<hipStream_t>(stream)));
        return UF_OK;
    });
}

// ------------------------------------------------------------------ sparse lists + re-rank
uf_status uf_sparse_build(const uf_embedding* emb, void* stream, uf_sparse** out) {
    return guarded([&]() -> uf_status {
        if (!emb || !out) return fail(UF_ERR_ARG, "NULL argument");
        *out = nullptr;
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int64_t n = emb->n, nnz = emb->nnz;
        int64_t* cnt = nullptr;
        if (hipMalloc(&cnt, size_t(std::max<int64_t>(nnz, 1)) * 8) != hipSuccess)
            return fail(UF_ERR_NOMEM, "sparse counts");
        std::unique_ptr<void, void (*)(void*)> gc(cnt, [](void* p) { (void)hipFree(p); });
        UF_HIP(ufp::sparse_count(view(*emb), cnt, s));
        std::vector<int64_t> hc(size_t(std::max<int64_t>(nnz, 1)), 0), rp(size_t(n + 1));
        UF_HIP(hipStreamSynchronize(s));
        if (nnz) UF_HIP(hipMemcpy(hc.data(), cnt, size_t(nnz) * 8, hipMemcpyDeviceToHost));
        UF_HIP(hipMemcpy(rp.data(), emb->row_ptr, size_t(n + 1) * 8, hipMemcpyDeviceToHost));
        std::vector<int64_t> eoff(size_t(std::max<int64_t>(nnz, 1)));
        int64_t run = 0;
        for (int64_t e = 0; e < nnz; ++e) {
            eoff[size_t(e)] = run;
            run += hc[size_t(e)];
        }
        std::vector<int64_t> soff(size_t(n + 1));
        for (int64_t i = 0; i < n; ++i) soff[size_t(i)] = rp[size_t(i)] < nnz ? eoff[size_t(rp[size_t(i)])] : run;
        soff[size_t(n)] = run;
        auto sp = new uf_sparse();
        std::unique_ptr<uf_sparse> guard(sp);
        sp->n = n;
        sp->nb = emb->nb;
        sp->nnz = run;
        const size_t o_off = 0, o_pos = align256(size_t(n + 1) * 8);
        const size_t o_val = o_pos + align256(size_t(std::max<int64_t>(run, 1)) * 4);
        const size_t o_s = o_val + align256(size_t(std::max<int64_t>(run, 1)) * 8);
        const size_t tot = o_s + align256(size_t(std::max<int64_t>(n, 1)) * 8);
        if (hipMalloc(&sp->arena, tot) != hipSuccess) return fail(UF_ERR_NOMEM, "sparse lists");
        char* base = static_cast<char*>(sp->arena);
        sp->off = reinterpret_cast<int64_t*>(base + o_off);
        sp->pos = reinterpret_cast<int32_t*>(base + o_pos);
        sp->val = reinterpret_cast<double*>(base + o_val);
        sp->s = reinterpret_cast<double*>(base + o_s);
        UF_HIP(hipMemcpy(sp->off, soff.data(), size_t(n + 1) * 8, hipMemcpyHostToDevice));
        UF_HIP(hipMemcpy(cnt, eoff.data(), size_t(std::max<int64_t>(nnz, 1)) * 8, hipMemcpyHostToDevice));
        UF_HIP(ufp::sparse_fill(view(*emb), cnt, sp->pos, sp->val, s));
        if (n) UF_HIP(hipMemcpyAsync(sp->s, emb->sw, size_t(n) * 8, hipMemcpyDeviceToDevice, s));
        UF_HIP(hipStreamSynchronize(s));
        *out = guard.release();
        return UF_OK;
    });
}

int64_t uf_sparse_nnz(const uf_sparse* sp) { return sp ? sp->nnz : -1; }
void uf_free_sparse(uf_sparse* sp) { delete sp; }

static int64_t rerank_rows(int64_t n_queries) { return std::min<int64_t>(std::max<int64_t>(n_queries, 1), 1024); }

uf_status uf_rerank_workspace_size(const uf_sparse* q, int64_t n_queries, size_t* bytes) {
    if (!q || !bytes || n_queries < 0) return fail(UF_ERR_ARG, "bad argument");
    *bytes = size_t(rerank_rows(n_queries)) * size_t(std::max<int64_t>(q->nb, 1)) * 8 + 256;
    return UF_OK;
}

uf_status uf_dm_rerank_weighted_normalized(const uf_sparse* queries, const uf_sparse* refs,
                                           const int32_t* query_ids, const int32_t* cand,
                                           int64_t n_queries, int64_t k, double* out, void* ws,
                                           size_t ws_bytes, void* stream) {
    return guarded([&]() -> uf_status {
        if (!queries || !refs || !query_ids || !cand || !out || n_queries < 0 || k < 1)
            return fail(UF_ERR_ARG, "bad argument");
        if (queries->nb != refs->nb) return fail(UF_ERR_ARG, "query and reference trees differ");
        size_t need = 0;
        uf_rerank_workspace_size(queries, n_queries, &need);
        if (!ws || ws_bytes < need) return fail(UF_ERR_WORKSPACE, "re-rank workspace too small");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        double* scratch = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
        const int64_t rows = rerank_rows(n_queries);
        UF_HIP(ufp::zero_f64(scratch, rows * queries->nb, s));
        UF_HIP(ufp::rerank(queries->view(), refs->view(), query_ids, cand, n_queries, int(k),
                           queries->nb, scratch, rows, out, s));
        return UF_OK;
    });
}

uf_status uf_dm_pairs_weighted_normalized(const uf_sparse* a, const uf_sparse* b,
                                          const int32_t* pairs, int64_t n_pairs, double* out,
                                          void* ws, size_t ws_bytes, void* stream) {
    // pair p is (a[pairs[p]], b[pairs[n_pairs + p]]): the re-rank with one candidate each
    if (!pairs || n_pairs < 0) return fail(UF_ERR_ARG, "bad pair list");
    if (n_pairs == 0) return UF_OK;
    return uf_dm_rerank_weighted_normalized(a, b, pairs, pairs + n_pairs, n_pairs, 1, out, ws,
                                            ws_bytes, stream);
}

}  // extern "C"
