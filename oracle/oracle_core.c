/*
 * Plain FP64 UniFrac distances in C -- TEST INFRASTRUCTURE ONLY.
 *
 * Same definitions as oracle/unifrac.py (paper section II names the unweighted
 * and the weighted-normalized variants; the formulas are the standard ones):
 *   d_U(i,j) = sum_v l_v |a_iv - a_jv| / sum_v l_v max(a_iv, a_jv)
 *   d_W(i,j) = sum_v l_v |u_iv - u_jv| / sum_v l_v (u_iv + u_jv)
 * over non-root nodes v; u = embedded count / sample total, a = [count > 0];
 * a zero denominator gives 0.  Embedded counts come from an iterative
 * postorder pass in exact int64.  Pairs are summed node by node in postorder,
 * one pair at a time, parallel over rows with OpenMP.  No blocking, no
 * reordering beyond that; it exists to be obviously right and to time the CPU
 * baseline.  It shares no code with the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_TREE = 2, ORC_ERR_TABLE = 3, ORC_ERR_NOMEM = 4 };

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Postorder of a parent-array tree; returns number of nodes reached. */
static int64_t postorder(int64_t m, const int64_t* parent, int64_t root, int64_t* order) {
    int64_t* first = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
    int64_t* kids = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 1 ? m : 1));
    int64_t* fill = (int64_t*)calloc((size_t)m, sizeof(int64_t));
    int64_t* stack_v = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    int64_t* stack_k = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    int64_t n_out = 0, top = 0;
    if (!first || !kids || !fill || !stack_v || !stack_k) { n_out = -1; goto done; }
    for (int64_t v = 0; v < m; ++v)
        if (parent[v] >= 0) first[parent[v] + 1]++;
    for (int64_t v = 0; v < m; ++v) first[v + 1] += first[v];
    for (int64_t v = 0; v < m; ++v)
        if (parent[v] >= 0) { int64_t p = parent[v]; kids[first[p] + fill[p]++] = v; }
    stack_v[0] = root; stack_k[0] = 0; top = 1;
    while (top > 0) {
        int64_t v = stack_v[top - 1], k = stack_k[top - 1];
        if (first[v] + k < first[v + 1]) {
            stack_k[top - 1] = k + 1;
            if (top >= m) { n_out = -1; goto done; }
            stack_v[top] = kids[first[v] + k]; stack_k[top] = 0; ++top;
        } else {
            order[n_out++] = v;
            --top;
        }
    }
done:
    free(first); free(kids); free(fill); free(stack_v); free(stack_k);
    return n_out;
}

/*
 * Condensed distance matrix (row-major upper triangle, length n(n-1)/2).
 * variant: 0 = unweighted, 1 = weighted normalized.  n_threads <= 0: default.
 * *threads_used receives the OpenMP team size.
 */
int orc_dm(int64_t m, const int64_t* parent, const double* length,
           int64_t n, const int64_t* indptr, const int64_t* tips, const int64_t* counts,
           int variant, int n_threads, double* out, int* threads_used) {
    if (m < 1 || n < 0 || !parent || !length || !indptr || !out) return ORC_ERR_ARG;
    int64_t root = -1;
    for (int64_t v = 0; v < m; ++v) {
        if (parent[v] == -1) { if (root >= 0) return ORC_ERR_TREE; root = v; }
        else if (parent[v] < 0 || parent[v] >= m || parent[v] == v) return ORC_ERR_TREE;
        else if (!(length[v] >= 0.0) || !isfinite(length[v])) return ORC_ERR_TREE;
    }
    if (root < 0) return ORC_ERR_TREE;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    if (!order) return ORC_ERR_NOMEM;
    if (postorder(m, parent, root, order) != m) { free(order); return ORC_ERR_TREE; }
    char* is_tip = (char*)calloc((size_t)m, 1);
    if (!is_tip) { free(order); return ORC_ERR_NOMEM; }
    for (int64_t v = 0; v < m; ++v) is_tip[v] = 1;
    for (int64_t v = 0; v < m; ++v) if (parent[v] >= 0) is_tip[parent[v]] = 0;

    const int64_t b = m - 1;                 /* branches = non-root nodes, postorder */
    double* lb = (double*)malloc(sizeof(double) * (size_t)(b > 0 ? b : 1));
    for (int64_t k = 0; k < b; ++k) lb[k] = length[order[k]];
    double* u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(b > 0 ? b : 1));
    unsigned char* a = (unsigned char*)malloc((size_t)(n > 0 ? n : 1) * (size_t)(b > 0 ? b : 1));
    int rc = ORC_OK;
    if (!u || !a || !lb) { rc = ORC_ERR_NOMEM; goto out; }

    /* embedding: per sample, exact int64 counts pushed up the tree in postorder */
    {
        int64_t* c = (int64_t*)calloc((size_t)m, sizeof(int64_t));
        char* mark = (char*)calloc((size_t)m, 1);
        if (!c || !mark) { free(c); free(mark); rc = ORC_ERR_NOMEM; goto out; }
        for (int64_t s = 0; s < n && rc == ORC_OK; ++s) {
            memset(c, 0, sizeof(int64_t) * (size_t)m);
            for (int64_t e = indptr[s]; e < indptr[s + 1]; ++e) {
                int64_t t = tips[e];
                if (t < 0 || t >= m || !is_tip[t] || counts[e] < 0 || mark[t]) { rc = ORC_ERR_TABLE; break; }
                mark[t] = 1;
                c[t] = counts[e];
            }
            for (int64_t e = indptr[s]; e < indptr[s + 1]; ++e)
                if (tips[e] >= 0 && tips[e] < m) mark[tips[e]] = 0;
            if (rc != ORC_OK) break;
            for (int64_t k = 0; k < m; ++k) {
                int64_t v = order[k];
                if (parent[v] >= 0) c[parent[v]] += c[v];
            }
            if (c[root] <= 0) { rc = ORC_ERR_TABLE; break; }
            const double total = (double)c[root];
            for (int64_t k = 0; k < b; ++k) {
                int64_t v = order[k];
                u[s * b + k] = (double)c[v] / total;
                a[s * b + k] = c[v] > 0;
            }
        }
        free(c); free(mark);
        if (rc != ORC_OK) goto out;
    }

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    {
        int used = 1;
#pragma omp parallel
        {
#ifdef _OPENMP
#pragma omp single
            used = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < n; ++i) {
                const double* ui = u + i * b;
                const unsigned char* ai = a + i * b;
                int64_t row = n * i - i * (i + 1) / 2;
                for (int64_t j = i + 1; j < n; ++j) {
                    double num = 0.0, den = 0.0;
                    if (variant == 1) {
                        const double* uj = u + j * b;
                        for (int64_t k = 0; k < b; ++k) {
                            num += lb[k] * fabs(ui[k] - uj[k]);
                            den += lb[k] * (ui[k] + uj[k]);
                        }
                    } else {
                        const unsigned char* aj = a + j * b;
                        for (int64_t k = 0; k < b; ++k) {
                            double x = ai[k], y = aj[k];
                            num += lb[k] * fabs(x - y);
                            den += lb[k] * (x > y ? x : y);
                        }
                    }
                    out[row + (j - i - 1)] = den > 0.0 ? num / den : 0.0;
                }
            }
        }
        if (threads_used) *threads_used = used;
    }
out:
    free(order); free(is_tip); free(lb); free(u); free(a);
    return rc;
}
