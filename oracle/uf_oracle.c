/*
 * Plain FP64 CPU oracle for UniFrac distances.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (UniFrac, as introduced in the paper's Section 1 and ported in Sections
 * 2-3, where the per-branch update is an embedding difference weighted by the branch
 * length; the formulas themselves follow the published UniFrac definitions):
 *
 *   C[v][k]  number of reads of sample k on tips at or below node v          (embedding)
 *   t_k      total reads of sample k
 *   for every pair (i, j) and every non-root node v with branch length L_v:
 *     unweighted:          num += L_v * [ (C[v][i] > 0) != (C[v][j] > 0) ]
 *                          den += L_v * [ (C[v][i] > 0) || (C[v][j] > 0) ]
 *     weighted normalized: p = C[v][i] / t_i,  q = C[v][j] / t_j
 *                          num += L_v * |p - q|
 *                          den += L_v * (p + q)
 *   d_ij = num / den   (0 when den == 0)
 *   weighted unnormalized (the variant of the Striped UniFrac work the paper builds on,
 *   its reference [3]): d_ij = num of the weighted normalized form, no division
 *
 * Counts come from walking every tip's reads up its ancestor chain (deliberately unlike a
 * level-by-level gather).  Both sums are Neumaier-compensated, branches are visited in
 * ascending node id, and pairs are spread over OpenMP threads; nothing else is reordered.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC uf_oracle.c -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_E_ARG = 1, OR_E_TREE = 2, OR_E_TABLE = 3, OR_E_OOM = 6 };

/* Walk-up counts for the samples listed in `sel`:
 *   out[s * n_nodes + v] = sum of counts of sample sel[s] on tips at or below v.
 * feature_node may be NULL (feature f sits on node f).  Returns an OR_* code. */
int uf_oracle_counts(int32_t n_nodes, const int32_t *parent, int32_t n_samples,
                     int32_t n_features, const int64_t *indptr, const int32_t *indices,
                     const int32_t *counts, const int32_t *feature_node, int32_t n_sel,
                     const int32_t *sel, int64_t *out)
{
    if (n_nodes < 1 || !parent || !indptr || !out || n_sel < 0) return OR_E_ARG;
    for (int32_t s = 0; s < n_sel; ++s) {
        int32_t k = sel[s];
        if (k < 0 || k >= n_samples) return OR_E_ARG;
        int64_t *row = out + (int64_t)s * n_nodes;
        memset(row, 0, sizeof(int64_t) * (size_t)n_nodes);
        for (int64_t e = indptr[k]; e < indptr[k + 1]; ++e) {
            int32_t f = indices[e];
            if (f < 0 || f >= n_features) return OR_E_TABLE;
            int32_t v = feature_node ? feature_node[f] : f;
            if (v < 0 || v >= n_nodes) return OR_E_TABLE;
            int64_t c = counts[e];
            int32_t steps = 0;
            while (v >= 0) {                 /* the tip itself and every ancestor */
                row[v] += c;
                v = parent[v];
                if (++steps > n_nodes) return OR_E_TREE;   /* cycle */
            }
        }
    }
    return OR_OK;
}

static inline void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/* Distances for the pairs (a[p], b[p]) of rows of `rows` (the [n_rows][n_nodes] walk-up
 * counts) with totals tot[row].  method 0 = unweighted, 1 = weighted normalized,
 * 2 = weighted unnormalized.
 * n_threads <= 0 uses the OpenMP default.  Returns an OR_* code. */
int uf_oracle_pairs(int32_t n_nodes, const int32_t *parent, const double *length,
                    int32_t n_rows, const int64_t *rows, const int64_t *tot, int32_t method,
                    int64_t n_pairs, const int32_t *a, const int32_t *b, double *out,
                    int32_t n_threads)
{
    if (n_nodes < 1 || !parent || !length || !rows || !out || n_pairs < 0) return OR_E_ARG;
    if (method < 0 || method > 2) return OR_E_ARG;
    for (int64_t p = 0; p < n_pairs; ++p)
        if (a[p] < 0 || a[p] >= n_rows || b[p] < 0 || b[p] >= n_rows) return OR_E_ARG;
    /* the thread count applies to this call only (a num_threads clause, not the
     * process-wide default) */
#ifdef _OPENMP
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
#endif

#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int64_t *ci = rows + (int64_t)a[p] * n_nodes;
        const int64_t *cj = rows + (int64_t)b[p] * n_nodes;
        double num = 0.0, num_c = 0.0, den = 0.0, den_c = 0.0;
        if (method == 0) {
            for (int32_t v = 0; v < n_nodes; ++v) {
                if (parent[v] < 0) continue;            /* the root has no branch */
                int x = ci[v] > 0, y = cj[v] > 0;
                double L = length[v];
                neumaier_add(&num, &num_c, (x != y) ? L : 0.0);
                neumaier_add(&den, &den_c, (x || y) ? L : 0.0);
            }
        } else {
            double ti = (double)tot[a[p]], tj = (double)tot[b[p]];
            for (int32_t v = 0; v < n_nodes; ++v) {
                if (parent[v] < 0) continue;
                double pi = (double)ci[v] / ti;
                double pj = (double)cj[v] / tj;
                double L = length[v];
                neumaier_add(&num, &num_c, L * fabs(pi - pj));
                neumaier_add(&den, &den_c, L * (pi + pj));
            }
        }
        double N = num + num_c, D = den + den_c;
        if (method == 2)
            out[p] = N;
        else
            out[p] = (D == 0.0) ? 0.0 : N / D;
    }
    return OR_OK;
}

int uf_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
