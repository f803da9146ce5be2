// Principal coordinates of a condensed distance matrix (gfx950).
//
// PCoA (Gower): A = -d^2/2, B = A - r 1^T - 1 r^T + g 11^T with r the row means
// of A (zero diagonal included) and g their mean; the coordinates are the top
// eigenvectors of B scaled by sqrt(eigenvalue).  B is never formed: every
// product B X is computed as
//     B X = A X - r (1^T X) - 1 (r^T X) + g 1 (1^T X),
// where A X reads the condensed matrix once per row block (HBM-bound).  The
// eigenpairs come from randomized subspace iteration with a Rayleigh-Ritz
// projection (Halko, Martinsson, Tropp 2011): Y = B Omega, then orthonormal
// bases of B Q, and T = Q^T B Q, whose small eigenproblem gives the Ritz pairs.
// Orthonormalisation is SVQB (Stathopoulos and Wu 2002): from the Gram matrix
// G = Y^T Y = U S U^T, Q = Y U S^{-1/2} over the directions with S above a
// relative floor (so rank-deficient B is handled), applied twice.  The small
// symmetric eigenproblems (at most 48 x 48) are solved on the host by cyclic
// Jacobi rotations.  All reductions over samples run in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "uf.h"
#include "uf_internal.h"

namespace ufq {
namespace {

constexpr int kRB = 64;          // rows per block of the A X kernel
constexpr int kMaxCols = 48;     // columns of the test matrix (LDS: 33 KiB + up to 24 KiB)
constexpr int kSegs = 8;         // column-block segments of the A X kernel

__device__ __forceinline__ int64_t cidx(int64_t n, int64_t a, int64_t b) {   // a < b
    return a * n - a * (a + 1) / 2 + (b - a - 1);
}

// P[seg][i][c] = sum over j in the segment's column blocks, j != i, of
// (-d_ij^2 / 2) X[j][c].  Block (ib, seg); 256 threads; tile 64 x 64 of A in
// LDS transposed (At[j][r]) so the inner loop reads consecutive rows.  The next
// tile is loaded into registers while the current one is multiplied.
template <int CPT>
__global__ __launch_bounds__(256) void k_ax(const double* __restrict__ dm, int64_t n,
                                            const double* __restrict__ X, int cols,
                                            int64_t nblk, double* __restrict__ P) {
    constexpr int kPer = kRB * kRB / 256;                 // tile elements per thread
    constexpr int kW = 4 * CPT;                           // X columns, zero-padded
    constexpr int kXPer = (kRB * kW + 255) / 256;         // X elements per thread
    __shared__ double At[kRB][kRB + 1];
    __shared__ double Xs[kRB][kW];
    const int tid = threadIdx.x;
    const int64_t ib = blockIdx.x, seg = blockIdx.y;
    const int64_t i0 = ib * kRB;
    const int64_t jb0 = nblk * seg / kSegs, jb1 = nblk * (seg + 1) / kSegs;
    const int r = tid & 63, cg = tid >> 6;      // output row; columns cg*CPT ..
    double acc[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) acc[k] = 0.0;
    // One tile's distances and X rows, all loads in flight at once: element u of
    // this thread is e = tid + 256 u, taken along the contiguous side of the
    // condensed rows (row i fixed and j consecutive above the diagonal, row j
    // fixed and i consecutive below it).  Zero outside the matrix and on it.
    double va[kPer], vx[kXPer];
    auto load = [&](int64_t jb) {
        const int64_t j0 = jb * kRB;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = jb >= ib ? e / kRB : e % kRB;
            const int cc = jb >= ib ? e % kRB : e / kRB;
            const int64_t i = i0 + rr, j = j0 + cc;
            va[u] = 0.0;
            if (i < n && j < n && i != j) va[u] = i < j ? dm[cidx(n, i, j)] : dm[cidx(n, j, i)];
        }
#pragma unroll
        for (int u = 0; u < kXPer; ++u) {
            const int e = tid + 256 * u;
            const int c = e % kW;
            const int64_t j = j0 + e / kW;
            vx[u] = (e < kRB * kW && c < cols && j < n) ? X[j * cols + c] : 0.0;
        }
    };
    auto store = [&](int64_t jb) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = jb >= ib ? e / kRB : e % kRB;
            const int cc = jb >= ib ? e % kRB : e / kRB;
            At[cc][rr] = 0.0 - 0.5 * va[u] * va[u];   // +0 where the distance is absent
        }
#pragma unroll
        for (int u = 0; u < kXPer; ++u) {
            const int e = tid + 256 * u;
            if (e < kRB * kW) Xs[e / kW][e % kW] = vx[u];
        }
    };
    if (jb0 < jb1) load(jb0);
    for (int64_t jb = jb0; jb < jb1; ++jb) {
        __syncthreads();
        store(jb);
        if (jb + 1 < jb1) load(jb + 1);          // next tile in flight during the FMAs
        __syncthreads();
        for (int jj = 0; jj < kRB; ++jj) {
            const double a = At[jj][r];
#pragma unroll
            for (int k = 0; k < CPT; ++k) acc[k] = fma(a, Xs[jj][cg * CPT + k], acc[k]);
        }
    }
    const int64_t i = i0 + r;
    if (i < n) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = cg * CPT + k;
            if (c < cols) P[(seg * n + i) * cols + c] = acc[k];
        }
    }
}

// k_ax for `cols` test columns: CPT = ceil(cols / 4) columns per thread.
template <int CPT>
hipError_t launch_ax_cpt(dim3 g, hipStream_t s, const double* dm, int64_t n, const double* X,
                         int cols, int64_t nblk, double* P) {
    hipLaunchKernelGGL(k_ax<CPT>, g, dim3(256), 0, s, dm, n, X, cols, nblk, P);
    return hipGetLastError();
}

hipError_t launch_ax(dim3 g, hipStream_t s, const double* dm, int64_t n, const double* X, int cols,
                     int64_t nblk, double* P) {
    switch ((cols + 3) / 4) {
        case 1: return launch_ax_cpt<1>(g, s, dm, n, X, cols, nblk, P);
        case 2: return launch_ax_cpt<2>(g, s, dm, n, X, cols, nblk, P);
        case 3: return launch_ax_cpt<3>(g, s, dm, n, X, cols, nblk, P);
        case 4: return launch_ax_cpt<4>(g, s, dm, n, X, cols, nblk, P);
        case 5: return launch_ax_cpt<5>(g, s, dm, n, X, cols, nblk, P);
        case 6: return launch_ax_cpt<6>(g, s, dm, n, X, cols, nblk, P);
        case 7: return launch_ax_cpt<7>(g, s, dm, n, X, cols, nblk, P);
        case 8: return launch_ax_cpt<8>(g, s, dm, n, X, cols, nblk, P);
        case 9: return launch_ax_cpt<9>(g, s, dm, n, X, cols, nblk, P);
        case 10: return launch_ax_cpt<10>(g, s, dm, n, X, cols, nblk, P);
        case 11: return launch_ax_cpt<11>(g, s, dm, n, X, cols, nblk, P);
        case 12: return launch_ax_cpt<12>(g, s, dm, n, X, cols, nblk, P);
        default: return hipErrorInvalidValue;
    }
}

// Fixed-order block reduction of 256 doubles held one per thread.
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

// sums[c] = sum_i X[i][c], sums[cols + c] = sum_i r_i X[i][c] (one block per column)
__global__ __launch_bounds__(256) void k_colsums(const double* __restrict__ X, int cols, int64_t n,
                                                 const double* __restrict__ rmean,
                                                 double* __restrict__ sums) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0, t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double x = X[i * cols + c];
        s += x;
        t += rmean[i] * x;
    }
    s = block_sum(s, red);
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
        sums[c] = s;
        sums[cols + c] = t;
    }
}

// Y = sum_seg P[seg] - r (1^T X) - 1 (r^T X) + g 1 (1^T X)
__global__ __launch_bounds__(256) void k_centre(const double* __restrict__ P, int64_t n, int cols,
                                                const double* __restrict__ rmean,
                                                const double* __restrict__ gmean,
                                                const double* __restrict__ sums,
                                                double* __restrict__ Y) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= n * cols) return;
    const int64_t i = e / cols;
    const int c = int(e % cols);
    double v = 0.0;
    for (int s = 0; s < kSegs; ++s) v += P[s * n * cols + e];
    const double g = gmean[0];
    Y[e] = v - rmean[i] * sums[c] - sums[cols + c] + g * sums[c];
}

// G_part[b][x][y] = sum over rows of block b (kGramRows rows) of Y[i][x] Z[i][y]
constexpr int kGramRows = 128;

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ Y, int cy,
                                              const double* __restrict__ Z, int cz, int64_t n,
                                              double* __restrict__ Gp) {
    const int64_t b = blockIdx.x;
    const int64_t r0 = b * kGramRows, r1 = min(n, r0 + kGramRows);
    for (int e = threadIdx.x; e < cy * cz; e += 256) {
        const int x = e / cz, y = e % cz;
        double s = 0.0;
        for (int64_t i = r0; i < r1; ++i) s = fma(Y[i * cy + x], Z[i * cz + y], s);
        Gp[(b * cy + x) * cz + y] = s;
    }
}

// Q[i][:] = Y[i][:] M with M (cy x cq) row major, one thread per (i, column)
__global__ __launch_bounds__(256) void k_rightmul(const double* __restrict__ Y, int cy, int64_t n,
                                                  const double* __restrict__ M, int cq,
                                                  double* __restrict__ Q) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= n * cq) return;
    const int64_t i = e / cq;
    const int c = int(e % cq);
    double s = 0.0;
    for (int k = 0; k < cy; ++k) s = fma(Y[i * cy + k], M[k * cq + c], s);
    Q[e] = s;
}

// Column k of V (n x dims): make its largest-magnitude entry (first on ties)
// positive.  One block per column; fixed-order arg-max.
__global__ __launch_bounds__(256) void k_signs(double* __restrict__ V, int dims, int64_t n) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    const int k = blockIdx.x;
    double best = -1.0;
    int64_t arg = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double a = fabs(V[i * dims + k]);
        if (a > best) {
            best = a;
            arg = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = arg;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = bv[threadIdx.x + w];
            const int64_t oi = bi[threadIdx.x + w];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const bool flip = V[bi[0] * dims + k] < 0.0;
    if (!flip) return;
    for (int64_t i = threadIdx.x; i < n; i += 256) V[i * dims + k] = -V[i * dims + k];
}

// --------------------------------------------------------------------- host
// Eigen-decomposition of a symmetric m x m matrix by cyclic Jacobi rotations:
// on return a holds nothing useful, w the eigenvalues, v (row major, columns =
// eigenvectors).
void jacobi_eig(std::vector<double> a, int m, std::vector<double>& w, std::vector<double>& v) {
    v.assign(size_t(m) * m, 0.0);
    for (int i = 0; i < m; ++i) v[size_t(i) * m + i] = 1.0;
    auto A = [&](int i, int j) -> double& { return a[size_t(i) * m + j]; };
    double norm = 0.0;
    for (double x : a) norm += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) off += A(i, j) * A(i, j);
        if (off <= 1e-30 * norm || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {   // columns p, q
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {   // rows p, q
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = v[size_t(k) * m + p], vkq = v[size_t(k) * m + q];
                    v[size_t(k) * m + p] = c * vkp - s * vkq;
                    v[size_t(k) * m + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(m);
    for (int i = 0; i < m; ++i) w[i] = A(i, i);
}

struct Plan {
    int64_t n = 0, nblk = 0;
    int cols = 0;
    size_t off_p = 0, off_y = 0, off_q = 0, off_z = 0, off_sums = 0, off_gp = 0, off_m = 0,
           off_r = 0, off_g = 0, off_one = 0, total = 0;
};

size_t take(size_t& off, size_t bytes) {
    const size_t at = (off + 255) & ~size_t(255);
    off = at + bytes;
    return at;
}

Plan make_plan(int64_t n, int cols) {
    Plan p;
    p.n = n;
    p.cols = cols;
    p.nblk = (n + kRB - 1) / kRB;
    const size_t nc = size_t(n) * size_t(cols) * 8;
    size_t off = 0;
    p.off_p = take(off, nc * kSegs);
    p.off_y = take(off, nc);
    p.off_q = take(off, nc);
    p.off_z = take(off, nc);
    p.off_sums = take(off, size_t(2 * cols) * 8);
    p.off_gp = take(off, size_t((n + kGramRows - 1) / kGramRows) * cols * cols * 8);
    p.off_m = take(off, size_t(cols) * cols * 8);
    p.off_r = take(off, size_t(n) * 8);
    p.off_g = take(off, 8);
    p.off_one = take(off, size_t(n) * 8);
    p.total = off + 256;
    return p;
}

}  // namespace
}  // namespace ufq

using ufh::fail;
using ufh::hip_fail;

#define UFQ_HIP(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

extern "C" {

uf_status uf_pcoa_workspace_size(int64_t n, int64_t n_cols, size_t* bytes) {
    if (!bytes) return fail(UF_ERR_ARG, "bytes is NULL");
    if (n < 2 || n_cols < 1 || n_cols > ufq::kMaxCols)
        return fail(UF_ERR_ARG, "need n >= 2 and 1 <= n_cols <= 48");
    *bytes = ufq::make_plan(n, int(std::min<int64_t>(n_cols, n))).total;
    return UF_OK;
}

uf_status uf_pcoa(const double* dm, int64_t n, const double* row_means, const double* grand_mean,
                  int64_t dims, int64_t n_cols, int power_iters, const double* omega,
                  double* coords, double* eigvals, double* trace, void* ws, size_t ws_bytes,
                  void* stream) {
    using namespace ufq;
    if (!dm || !omega || !coords || !eigvals) return fail(UF_ERR_ARG, "NULL argument");
    if (n < 2) return fail(UF_ERR_ARG, "need at least 2 samples");
    if (dims < 1 || n_cols < dims || n_cols > kMaxCols)
        return fail(UF_ERR_ARG, "need 1 <= dims <= n_cols <= 48");
    if (power_iters < 0 || power_iters > 64) return fail(UF_ERR_ARG, "power_iters in [0, 64]");
    if ((row_means == nullptr) != (grand_mean == nullptr))
        return fail(UF_ERR_ARG, "pass both row_means and grand_mean, or neither");
    int dev = 0;
    uf_status st = ufh::check_device(&dev);
    if (st != UF_OK) return st;
    const int l0 = int(n_cols);
    const int cols = int(std::min<int64_t>(n_cols, n));   // at most n independent directions
    const Plan p = make_plan(n, cols);
    if (!ws || ws_bytes < p.total) return fail(UF_ERR_WORKSPACE, "workspace missing or too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    double* P = reinterpret_cast<double*>(base + p.off_p);
    double* Y = reinterpret_cast<double*>(base + p.off_y);
    double* Q = reinterpret_cast<double*>(base + p.off_q);
    double* Z = reinterpret_cast<double*>(base + p.off_z);
    double* sums = reinterpret_cast<double*>(base + p.off_sums);
    double* Gp = reinterpret_cast<double*>(base + p.off_gp);
    double* Md = reinterpret_cast<double*>(base + p.off_m);
    const int64_t nbg = (n + kGramRows - 1) / kGramRows;
    const dim3 gax{unsigned(p.nblk), unsigned(kSegs)};

    // row means of A and grand mean: given, or A 1 / n and its mean
    const double* rm = row_means;
    const double* gm = grand_mean;
    if (!rm) {
        double* r = reinterpret_cast<double*>(base + p.off_r);
        double* g = reinterpret_cast<double*>(base + p.off_g);
        double* one = reinterpret_cast<double*>(base + p.off_one);
        std::vector<double> h1(static_cast<size_t>(n), 1.0);
        UFQ_HIP(hipMemcpyAsync(one, h1.data(), size_t(n) * 8, hipMemcpyHostToDevice, s));
        UFQ_HIP(launch_ax(gax, s, dm, n, one, 1, p.nblk, P));
        // r = (sum_seg P) / n via k_centre with zero means: reuse Y as scratch
        UFQ_HIP(hipMemsetAsync(sums, 0, size_t(2 * cols) * 8, s));
        UFQ_HIP(hipMemsetAsync(g, 0, 8, s));
        UFQ_HIP(hipMemsetAsync(Y, 0, size_t(n) * 8, s));
        hipLaunchKernelGGL(k_centre, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, P, n, 1, Y, g,
                           sums, r);
        UFQ_HIP(hipGetLastError());
        std::vector<double> hr(static_cast<size_t>(n));
        UFQ_HIP(hipMemcpyAsync(hr.data(), r, size_t(n) * 8, hipMemcpyDeviceToHost, s));
        UFQ_HIP(hipStreamSynchronize(s));
        double tot = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            hr[size_t(i)] /= double(n);
            tot += hr[size_t(i)];
        }
        const double hg = tot / double(n);
        UFQ_HIP(hipMemcpyAsync(r, hr.data(), size_t(n) * 8, hipMemcpyHostToDevice, s));
        UFQ_HIP(hipMemcpyAsync(g, &hg, 8, hipMemcpyHostToDevice, s));
        UFQ_HIP(hipStreamSynchronize(s));   // host sources go out of scope
        rm = r;
        gm = g;
    }

    // X (n x c) -> B X into out
    auto bx = [&](const double* X, int c, double* out) -> uf_status {
        UFQ_HIP(launch_ax(gax, s, dm, n, X, c, p.nblk, P));
        hipLaunchKernelGGL(k_colsums, dim3(unsigned(c)), dim3(256), 0, s, X, c, n, rm, sums);
        UFQ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_centre, dim3(unsigned((n * c + 255) / 256)), dim3(256), 0, s, P, n, c, rm,
                           gm, sums, out);
        UFQ_HIP(hipGetLastError());
        return UF_OK;
    };
    // host copy of the fixed-order sum of Y^T Z (cy x cz)
    auto gram = [&](const double* A, int ca, const double* B, int cb, std::vector<double>& G) -> uf_status {
        hipLaunchKernelGGL(k_gram, dim3(unsigned(nbg)), dim3(256), 0, s, A, ca, B, cb, n, Gp);
        UFQ_HIP(hipGetLastError());
        std::vector<double> part(size_t(nbg) * ca * cb);
        UFQ_HIP(hipMemcpyAsync(part.data(), Gp, part.size() * 8, hipMemcpyDeviceToHost, s));
        UFQ_HIP(hipStreamSynchronize(s));
        G.assign(size_t(ca) * cb, 0.0);
        for (int64_t b = 0; b < nbg; ++b)
            for (size_t e = 0; e < G.size(); ++e) G[e] += part[size_t(b) * G.size() + e];
        return UF_OK;
    };
    // SVQB: out = Yin U S^{-1/2} over the directions of Yin above the floor; returns
    // the number of columns kept
    auto svqb = [&](const double* Yin, int c, double* out, int* kept) -> uf_status {
        std::vector<double> G, w, v;
        uf_status e = gram(Yin, c, Yin, c, G);
        if (e != UF_OK) return e;
        jacobi_eig(G, c, w, v);
        std::vector<int> order(static_cast<size_t>(c));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
        const double top = c > 0 ? w[size_t(order[0])] : 0.0;
        int k = 0;
        while (k < c && top > 0.0 && w[size_t(order[size_t(k)])] > 1e-14 * top) ++k;
        std::vector<double> M(size_t(c) * std::max(k, 1), 0.0);
        for (int j = 0; j < k; ++j) {
            const int o = order[size_t(j)];
            const double sc = 1.0 / std::sqrt(w[size_t(o)]);
            for (int r = 0; r < c; ++r) M[size_t(r) * k + j] = v[size_t(r) * c + o] * sc;
        }
        *kept = k;
        if (k == 0) return UF_OK;
        UFQ_HIP(hipMemcpyAsync(Md, M.data(), M.size() * 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_rightmul, dim3(unsigned((n * k + 255) / 256)), dim3(256), 0, s, Yin, c, n,
                           Md, k, out);
        UFQ_HIP(hipGetLastError());
        UFQ_HIP(hipStreamSynchronize(s));   // M is reused by the next call
        return UF_OK;
    };
    auto orth = [&](double* Yin, int c, double* out, int* kept) -> uf_status {
        int k1 = 0;
        uf_status e = svqb(Yin, c, Z, &k1);   // Z as scratch
        if (e != UF_OK || k1 == 0) {
            *kept = k1;
            return e;
        }
        return svqb(Z, k1, out, kept);
    };

    // Omega is n x l0; a narrower basis (l0 > n) keeps its first `cols` columns
    const double* Om = omega;
    if (cols < l0) {
        std::vector<double> h(size_t(n) * l0), hs(size_t(n) * cols);
        UFQ_HIP(hipMemcpyAsync(h.data(), omega, h.size() * 8, hipMemcpyDeviceToHost, s));
        UFQ_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < cols; ++c) hs[size_t(i) * cols + c] = h[size_t(i) * l0 + c];
        UFQ_HIP(hipMemcpyAsync(Q, hs.data(), hs.size() * 8, hipMemcpyHostToDevice, s));
        UFQ_HIP(hipStreamSynchronize(s));   // hs goes out of scope
        Om = Q;
    }
    st = bx(Om, cols, Y);
    if (st != UF_OK) return st;
    int k = 0;
    st = orth(Y, cols, Q, &k);
    if (st != UF_OK) return st;
    for (int it = 0; it < power_iters && k > 0; ++it) {
        st = bx(Q, k, Y);
        if (st != UF_OK) return st;
        st = orth(Y, k, Q, &k);
        if (st != UF_OK) return st;
    }
    std::vector<double> lam(size_t(dims), 0.0);
    std::vector<double> W(size_t(std::max(k, 1)) * dims, 0.0);   // k x dims, scaled
    if (k > 0) {
        st = bx(Q, k, Y);   // Y = B Q
        if (st != UF_OK) return st;
        std::vector<double> T, w, v;
        st = gram(Q, k, Y, k, T);
        if (st != UF_OK) return st;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                const double m = 0.5 * (T[size_t(a) * k + b] + T[size_t(b) * k + a]);
                T[size_t(a) * k + b] = T[size_t(b) * k + a] = m;
            }
        jacobi_eig(T, k, w, v);
        std::vector<int> order(static_cast<size_t>(k));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
        for (int j = 0; j < dims && j < k; ++j) {
            const int o = order[size_t(j)];
            lam[size_t(j)] = w[size_t(o)];
            const double sc = std::sqrt(std::max(w[size_t(o)], 0.0));
            for (int r = 0; r < k; ++r) W[size_t(r) * dims + j] = v[size_t(r) * k + o] * sc;
        }
        UFQ_HIP(hipMemcpyAsync(Md, W.data(), W.size() * 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_rightmul, dim3(unsigned((n * dims + 255) / 256)), dim3(256), 0, s, Q, k, n,
                           Md, int(dims), coords);
        UFQ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_signs, dim3(unsigned(dims)), dim3(256), 0, s, coords, int(dims), n);
        UFQ_HIP(hipGetLastError());
        UFQ_HIP(hipStreamSynchronize(s));   // W goes out of scope
    } else {
        UFQ_HIP(hipMemsetAsync(coords, 0, size_t(n) * dims * 8, s));
    }
    std::memcpy(eigvals, lam.data(), size_t(dims) * 8);
    if (trace) {
        double hg = 0.0;
        UFQ_HIP(hipMemcpyAsync(&hg, gm, 8, hipMemcpyDeviceToHost, s));
        UFQ_HIP(hipStreamSynchronize(s));
        *trace = -double(n) * hg;
    }
    UFQ_HIP(hipStreamSynchronize(s));
    return UF_OK;
}

}  // extern "C"
