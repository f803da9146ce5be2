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

// ------------------------------------------------------------------ PCA basis
// Principal directions of a BF16 data matrix X [n][d] (row stride ldx): the
// same randomized subspace iteration, on the covariance C = Xc^T Xc / n with
// Xc = X - column means.  C is never formed: C Q = Xc^T (Xc Q).
constexpr int kPcaMaxCols = 160;   // columns of the test matrix
constexpr int kPcaT = 64;          // rows and columns of an X tile
constexpr int kPcaSplits = 8;      // row ranges of the X^T Y kernel

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// mu[j] = (1/n) sum_i X[i][j] (FP64, fixed order)
__global__ __launch_bounds__(256) void k_pca_mean(const uint16_t* __restrict__ X, int64_t ldx,
                                                  int64_t n, int64_t d, double* __restrict__ mu) {
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= d) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += double(bf16_to_f32(X[i * ldx + j]));
    mu[j] = s / double(n);
}

// Y[i][c] = sum_j (X[i][j] - mu[j]) Q[j][c] for a block of 64 rows.  Thread t
// owns row t/4 and columns t%4 + 4m; tiles of 64 columns of X (centred, FP32)
// and the matching 64 rows of Q (FP64) pass through LDS.
__global__ __launch_bounds__(256) void k_pca_xq(const uint16_t* __restrict__ X, int64_t ldx,
                                                int64_t n, int64_t d, const double* __restrict__ mu,
                                                const double* __restrict__ Q, int c,
                                                double* __restrict__ Y) {
    __shared__ float xs[kPcaT][kPcaT + 1];
    __shared__ double qs[kPcaT][kPcaMaxCols];
    const int t = threadIdx.x, r = t >> 2, g = t & 3;
    const int64_t i0 = int64_t(blockIdx.x) * kPcaT;
    constexpr int kM = kPcaMaxCols / 4;
    double acc[kM];
#pragma unroll
    for (int m = 0; m < kM; ++m) acc[m] = 0.0;
    for (int64_t j0 = 0; j0 < d; j0 += kPcaT) {
        for (int e = t; e < kPcaT * kPcaT; e += 256) {
            const int rr = e / kPcaT, jj = e % kPcaT;
            const int64_t i = i0 + rr, j = j0 + jj;
            xs[rr][jj] = (i < n && j < d) ? float(double(bf16_to_f32(X[i * ldx + j])) - mu[j]) : 0.0f;
        }
        for (int e = t; e < kPcaT * c; e += 256) {
            const int jj = e / c, cc = e % c;
            const int64_t j = j0 + jj;
            qs[jj][cc] = j < d ? Q[j * c + cc] : 0.0;
        }
        __syncthreads();
        for (int jj = 0; jj < kPcaT; ++jj) {
            const double xv = xs[r][jj];
#pragma unroll
            for (int m = 0; m < kM; ++m)
                if (g + 4 * m < c) acc[m] = fma(xv, qs[jj][g + 4 * m], acc[m]);
        }
        __syncthreads();
    }
    const int64_t i = i0 + r;
    if (i >= n) return;
#pragma unroll
    for (int m = 0; m < kM; ++m)
        if (g + 4 * m < c) Y[i * c + g + 4 * m] = acc[m];
}

// Zp[s][j][c] = sum over rows i of range s of (X[i][j] - mu[j]) Y[i][c], for a
// block of 64 columns j; thread t owns column t/4 and outputs t%4 + 4m.
__global__ __launch_bounds__(256) void k_pca_xty(const uint16_t* __restrict__ X, int64_t ldx,
                                                 int64_t n, int64_t d, const double* __restrict__ mu,
                                                 const double* __restrict__ Y, int c,
                                                 double* __restrict__ Zp) {
    __shared__ float xs[kPcaT][kPcaT + 1];     // [row i][column j]
    __shared__ double ys[kPcaT][kPcaMaxCols];
    const int t = threadIdx.x, jl = t >> 2, g = t & 3;
    const int64_t j0 = int64_t(blockIdx.x) * kPcaT;
    const int64_t per = (n + kPcaSplits - 1) / kPcaSplits;
    const int64_t ib = int64_t(blockIdx.y) * per, ie = min(n, ib + per);
    constexpr int kM = kPcaMaxCols / 4;
    double acc[kM];
#pragma unroll
    for (int m = 0; m < kM; ++m) acc[m] = 0.0;
    for (int64_t r0 = ib; r0 < ie; r0 += kPcaT) {
        for (int e = t; e < kPcaT * kPcaT; e += 256) {
            const int rr = e / kPcaT, jj = e % kPcaT;
            const int64_t i = r0 + rr, j = j0 + jj;
            xs[rr][jj] = (i < ie && j < d) ? float(double(bf16_to_f32(X[i * ldx + j])) - mu[j]) : 0.0f;
        }
        for (int e = t; e < kPcaT * c; e += 256) {
            const int rr = e / c, cc = e % c;
            const int64_t i = r0 + rr;
            ys[rr][cc] = i < ie ? Y[i * c + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < kPcaT; ++rr) {
            const double xv = xs[rr][jl];
#pragma unroll
            for (int m = 0; m < kM; ++m)
                if (g + 4 * m < c) acc[m] = fma(xv, ys[rr][g + 4 * m], acc[m]);
        }
        __syncthreads();
    }
    const int64_t j = j0 + jl;
    if (j >= d) return;
    double* out = Zp + int64_t(blockIdx.y) * d * c;
#pragma unroll
    for (int m = 0; m < kM; ++m)
        if (g + 4 * m < c) out[j * c + g + 4 * m] = acc[m];
}

// Z = sum over the row ranges of Zp, in range order
__global__ __launch_bounds__(256) void k_pca_sum(const double* __restrict__ Zp, int64_t count,
                                                 double* __restrict__ Z) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= count) return;
    double v = 0.0;
    for (int s = 0; s < kPcaSplits; ++s) v += Zp[s * count + e];
    Z[e] = v;
}

// out[r][j] = B[j][r] as FP32 (B: d x k FP64)
__global__ __launch_bounds__(256) void k_pca_out(const double* __restrict__ B, int64_t d, int k,
                                                 float* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= d * k) return;
    const int64_t r = e / d, j = e % d;
    out[e] = float(B[j * k + r]);
}

struct PcaPlan {
    size_t off_mu = 0, off_y = 0, off_zp = 0, off_z = 0, off_q = 0, off_gp = 0, off_m = 0,
           off_b = 0, total = 0;
};

PcaPlan make_pca_plan(int64_t n, int64_t d, int c) {
    PcaPlan p;
    size_t off = 0;
    const int64_t rows = std::max(n, d);
    p.off_mu = take(off, size_t(d) * 8);
    p.off_y = take(off, size_t(n) * c * 8);
    p.off_zp = take(off, size_t(kPcaSplits) * d * c * 8);
    p.off_z = take(off, size_t(d) * c * 8);
    p.off_q = take(off, size_t(d) * c * 8);
    p.off_gp = take(off, size_t((rows + kGramRows - 1) / kGramRows) * c * c * 8);
    p.off_m = take(off, size_t(c) * c * 8);
    p.off_b = take(off, size_t(d) * c * 8);
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


uf_status uf_pca_workspace_size(int64_t n, int64_t d, int64_t n_cols, size_t* bytes) {
    if (!bytes) return fail(UF_ERR_ARG, "bytes is NULL");
    if (n < 2 || d < 1 || n_cols < 1 || n_cols > ufq::kPcaMaxCols || n_cols > d)
        return fail(UF_ERR_ARG, "need n >= 2, d >= 1 and 1 <= n_cols <= min(160, d)");
    *bytes = ufq::make_pca_plan(n, d, int(n_cols)).total;
    return UF_OK;
}

uf_status uf_pca_basis(const void* x_bf16, int64_t n, int64_t d, int64_t ldx, int64_t k,
                       int64_t n_cols, int power_iters, const double* omega, float* basis,
                       double* eigvals, void* ws, size_t ws_bytes, void* stream) {
    using namespace ufq;
    if (!x_bf16 || !omega || !basis) return fail(UF_ERR_ARG, "NULL argument");
    if (n < 2 || d < 1 || ldx < d) return fail(UF_ERR_ARG, "need n >= 2, d >= 1 and ldx >= d");
    if (k < 1 || n_cols < k || n_cols > kPcaMaxCols || n_cols > d)
        return fail(UF_ERR_ARG, "need 1 <= k <= n_cols <= min(160, d)");
    if (power_iters < 0 || power_iters > 64) return fail(UF_ERR_ARG, "power_iters in [0, 64]");
    if (n > (int64_t(1) << 31) || d > (int64_t(1) << 24)) return fail(UF_ERR_ARG, "matrix too large");
    int dev = 0;
    uf_status st = ufh::check_device(&dev);
    if (st != UF_OK) return st;
    const int c = int(n_cols);
    const PcaPlan p = make_pca_plan(n, d, c);
    if (!ws || ws_bytes < p.total) return fail(UF_ERR_WORKSPACE, "workspace missing or too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    const uint16_t* X = static_cast<const uint16_t*>(x_bf16);
    double* mu = reinterpret_cast<double*>(base + p.off_mu);
    double* Y = reinterpret_cast<double*>(base + p.off_y);
    double* Zp = reinterpret_cast<double*>(base + p.off_zp);
    double* Z = reinterpret_cast<double*>(base + p.off_z);
    double* Q = reinterpret_cast<double*>(base + p.off_q);
    double* Gp = reinterpret_cast<double*>(base + p.off_gp);
    double* Md = reinterpret_cast<double*>(base + p.off_m);
    double* B = reinterpret_cast<double*>(base + p.off_b);

    hipLaunchKernelGGL(k_pca_mean, dim3(unsigned((d + 255) / 256)), dim3(256), 0, s, X, ldx, n, d, mu);
    UFQ_HIP(hipGetLastError());
    // Y = Xc Qin (n x cq)
    auto xq = [&](const double* Qin, int cq) -> uf_status {
        hipLaunchKernelGGL(k_pca_xq, dim3(unsigned((n + kPcaT - 1) / kPcaT)), dim3(256), 0, s, X, ldx,
                           n, d, mu, Qin, cq, Y);
        UFQ_HIP(hipGetLastError());
        return UF_OK;
    };
    // Z = Xc^T Y (d x cq)
    auto xty = [&](int cq) -> uf_status {
        hipLaunchKernelGGL(k_pca_xty, dim3(unsigned((d + kPcaT - 1) / kPcaT), unsigned(kPcaSplits)),
                           dim3(256), 0, s, X, ldx, n, d, mu, Y, cq, Zp);
        UFQ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pca_sum, dim3(unsigned((d * cq + 255) / 256)), dim3(256), 0, s, Zp,
                           d * cq, Z);
        UFQ_HIP(hipGetLastError());
        return UF_OK;
    };
    // host copy of the fixed-order sum of A^T A over `rows` rows (ca x ca)
    auto gram = [&](const double* A, int ca, int64_t rows, std::vector<double>& G) -> uf_status {
        const int64_t nbg = (rows + kGramRows - 1) / kGramRows;
        hipLaunchKernelGGL(k_gram, dim3(unsigned(nbg)), dim3(256), 0, s, A, ca, A, ca, rows, Gp);
        UFQ_HIP(hipGetLastError());
        std::vector<double> part(size_t(nbg) * ca * ca);
        UFQ_HIP(hipMemcpyAsync(part.data(), Gp, part.size() * 8, hipMemcpyDeviceToHost, s));
        UFQ_HIP(hipStreamSynchronize(s));
        G.assign(size_t(ca) * ca, 0.0);
        for (int64_t b = 0; b < nbg; ++b)
            for (size_t e = 0; e < G.size(); ++e) G[e] += part[size_t(b) * G.size() + e];
        return UF_OK;
    };
    // SVQB of the d x cin matrix Ain into out (columns above the relative floor)
    auto svqb = [&](const double* Ain, int cin, double* out, int* kept) -> uf_status {
        std::vector<double> G, w, v;
        uf_status e = gram(Ain, cin, d, G);
        if (e != UF_OK) return e;
        jacobi_eig(G, cin, w, v);
        std::vector<int> order(static_cast<size_t>(cin));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
        const double top = cin > 0 ? w[size_t(order[0])] : 0.0;
        int kk = 0;
        while (kk < cin && top > 0.0 && w[size_t(order[size_t(kk)])] > 1e-14 * top) ++kk;
        *kept = kk;
        if (kk == 0) return UF_OK;
        std::vector<double> M(size_t(cin) * kk, 0.0);
        for (int j = 0; j < kk; ++j) {
            const int o = order[size_t(j)];
            const double sc = 1.0 / std::sqrt(w[size_t(o)]);
            for (int r = 0; r < cin; ++r) M[size_t(r) * kk + j] = v[size_t(r) * cin + o] * sc;
        }
        UFQ_HIP(hipMemcpyAsync(Md, M.data(), M.size() * 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_rightmul, dim3(unsigned((d * kk + 255) / 256)), dim3(256), 0, s, Ain, cin,
                           d, Md, kk, out);
        UFQ_HIP(hipGetLastError());
        UFQ_HIP(hipStreamSynchronize(s));   // M is reused by the next call
        return UF_OK;
    };
    // Q <- orthonormal basis of Z's columns (SVQB twice, through B as scratch)
    auto orth = [&](int cin, int* kept) -> uf_status {
        int k1 = 0;
        uf_status e = svqb(Z, cin, B, &k1);
        if (e != UF_OK || k1 == 0) {
            *kept = k1;
            return e;
        }
        return svqb(B, k1, Q, kept);
    };

    int kq = 0;
    st = xq(omega, c);
    if (st != UF_OK) return st;
    st = xty(c);
    if (st != UF_OK) return st;
    st = orth(c, &kq);
    if (st != UF_OK) return st;
    for (int it = 0; it < power_iters && kq > 0; ++it) {
        st = xq(Q, kq);
        if (st != UF_OK) return st;
        st = xty(kq);
        if (st != UF_OK) return st;
        st = orth(kq, &kq);
        if (st != UF_OK) return st;
    }
    // Rayleigh-Ritz: H = (Xc Q)^T (Xc Q) = Q^T C Q n; its top eigenvectors W give
    // the directions Q W and the eigenvalues of C
    const int kk = int(std::min<int64_t>(k, kq));
    std::vector<double> lam(size_t(k), 0.0);
    std::vector<double> W(size_t(std::max(kq, 1)) * k, 0.0);
    if (kq > 0) {
        st = xq(Q, kq);
        if (st != UF_OK) return st;
        std::vector<double> H, w, v;
        const int64_t nbg = (n + kGramRows - 1) / kGramRows;
        hipLaunchKernelGGL(k_gram, dim3(unsigned(nbg)), dim3(256), 0, s, Y, kq, Y, kq, n, Gp);
        UFQ_HIP(hipGetLastError());
        {
            std::vector<double> part(size_t(nbg) * kq * kq);
            UFQ_HIP(hipMemcpyAsync(part.data(), Gp, part.size() * 8, hipMemcpyDeviceToHost, s));
            UFQ_HIP(hipStreamSynchronize(s));
            H.assign(size_t(kq) * kq, 0.0);
            for (int64_t b = 0; b < nbg; ++b)
                for (size_t e = 0; e < H.size(); ++e) H[e] += part[size_t(b) * H.size() + e];
        }
        jacobi_eig(H, kq, w, v);
        std::vector<int> order(static_cast<size_t>(kq));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
        for (int j = 0; j < kk; ++j) {
            const int o = order[size_t(j)];
            lam[size_t(j)] = w[size_t(o)] / double(n);
            for (int r = 0; r < kq; ++r) W[size_t(r) * k + j] = v[size_t(r) * kq + o];
        }
    }
    UFQ_HIP(hipMemcpyAsync(Md, W.data(), size_t(std::max(kq, 1)) * k * 8, hipMemcpyHostToDevice, s));
    if (kq > 0) {
        hipLaunchKernelGGL(k_rightmul, dim3(unsigned((d * k + 255) / 256)), dim3(256), 0, s, Q, kq, d,
                           Md, int(k), B);
        UFQ_HIP(hipGetLastError());
    } else {
        UFQ_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(B), 2 * d * k, s));
    }
    hipLaunchKernelGGL(k_pca_out, dim3(unsigned((d * k + 255) / 256)), dim3(256), 0, s, B, d, int(k),
                       basis);
    UFQ_HIP(hipGetLastError());
    UFQ_HIP(hipStreamSynchronize(s));   // W goes out of scope
    if (eigvals) std::memcpy(eigvals, lam.data(), size_t(k) * 8);
    return UF_OK;
}

}  // extern "C"
