/*
 * ls_cluster.c -- plain CPU reference for the consumers of the distance
 * matrix (Aslett & Christ, "kalis", arXiv 2212.11403): average pairwise
 * linkage, with which the paper clusters a distance matrix in section 6
 * (Sokal and Michener's unweighted pair-group method with arithmetic means),
 * and the standardisation of a recipient's column of distances with the
 * zero-deviation rule of section 2.2.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code with the GPU
 * path; built with -ffp-contract=off.
 *
 * Average linkage, as defined: every haplotype starts as its own cluster;
 * the two clusters at the smallest distance are merged, where the distance
 * between clusters A and B is the mean of d(a, b) over a in A and b in B;
 * this repeats until one cluster is left. The distance to a merged cluster is
 * kept with the update d(A u B, C) = (|A| d(A, C) + |B| d(B, C)) / (|A| + |B|),
 * which equals that mean (the tests check it against the mean), evaluated in
 * the precision of D, each operation rounded in that order:
 * t = |A| d(A,C); u = |B| d(B,C); s = t + u; d = s / (|A| + |B|).
 *
 * Slots and ties. Cluster k lives in slot k at the start; a merge of the
 * clusters in slots a < b puts the merged cluster in slot a and empties
 * slot b. Among the pairs of occupied slots at the smallest distance the
 * merge takes the pair (a, b), a < b, with the smallest a, then the smallest
 * b; a NaN distance (a column of a total underflow) comes after every
 * number. Ids follow the usual linkage-matrix convention: leaves 0..N-1, the
 * cluster made by merge m gets id N + m. Output row m of Z: the smaller id,
 * the larger id, the merge distance, the size of the merged cluster.
 *
 * Two evaluations of the same definition: linkage_naive scans every pair
 * for every merge (O(N^3)); linkage_nn keeps each occupied slot's nearest
 * occupied slot (ties: the smallest slot) and rescans only the rows whose
 * nearest slot was merged (O(N^2) typically). The tests check that both give
 * the same merges, bit for bit, on random and tie-heavy matrices.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The order in which candidate merges are taken: by distance, a NaN
 * distance after every number; equal distances (or two NaNs) by the slot
 * pair, smaller first. */
#define ORDER_DEF(T, SUF)                                                                        \
    static int before_##SUF(T d1, int32_t p1, int32_t q1, T d2, int32_t p2, int32_t q2)          \
    {                                                                                            \
        int n1 = isnan(d1), n2 = isnan(d2);                                                      \
        if (n1 != n2)                                                                            \
            return n2;                                                                           \
        if (!n1 && d1 != d2)                                                                     \
            return d1 < d2;                                                                      \
        return p1 < p2 || (p1 == p2 && q1 < q2);                                                 \
    }
ORDER_DEF(float, f32)
ORDER_DEF(double, f64)

#define LINKAGE_DEFS(T, SUF)                                                                     \
    static int linkage_naive_##SUF(T *D, int32_t N, double *Z)                                    \
    {                                                                                            \
        int32_t *size = malloc(sizeof(int32_t) * (size_t)N);                                     \
        int32_t *id = malloc(sizeof(int32_t) * (size_t)N);                                       \
        char *live = malloc((size_t)N);                                                          \
        if (!size || !id || !live) {                                                             \
            free(size);                                                                          \
            free(id);                                                                            \
            free(live);                                                                          \
            return 2;                                                                            \
        }                                                                                        \
        for (int32_t k = 0; k < N; ++k) {                                                        \
            size[k] = 1;                                                                         \
            id[k] = k;                                                                           \
            live[k] = 1;                                                                         \
        }                                                                                        \
        for (int32_t m = 0; m + 1 < N; ++m) {                                                    \
            int32_t a = -1, b = -1;                                                              \
            T best = 0;                                                                          \
            for (int32_t i = 0; i < N; ++i) {                                                    \
                if (!live[i])                                                                    \
                    continue;                                                                    \
                for (int32_t j = i + 1; j < N; ++j) {                                            \
                    if (!live[j])                                                                \
                        continue;                                                                \
                    T d = D[(int64_t)i * N + j];                                                 \
                    if (a < 0 || before_##SUF(d, i, j, best, a, b)) {                            \
                        best = d;                                                                \
                        a = i;                                                                   \
                        b = j;                                                                   \
                    }                                                                            \
                }                                                                                \
            }                                                                                    \
            merge_##SUF(D, N, live, a, b, size);                                                 \
            Z[4 * m + 0] = id[a] < id[b] ? id[a] : id[b];                                        \
            Z[4 * m + 1] = id[a] < id[b] ? id[b] : id[a];                                        \
            Z[4 * m + 2] = (double)best;                                                         \
            Z[4 * m + 3] = size[a];                                                              \
            id[a] = N + m;                                                                       \
        }                                                                                        \
        free(size);                                                                              \
        free(id);                                                                                \
        free(live);                                                                              \
        return 0;                                                                                \
    }                                                                                            \
                                                                                                 \
    /* nearest occupied slot of row i (ties: the smallest slot); -1 if none */                   \
    static int32_t nearest_##SUF(const T *D, int32_t N, const char *live, int32_t i, T *dist)   \
    {                                                                                            \
        int32_t best = -1;                                                                       \
        T bd = 0;                                                                                \
        for (int32_t k = 0; k < N; ++k) {                                                        \
            if (k == i || !live[k])                                                              \
                continue;                                                                        \
            T d = D[(int64_t)i * N + k];                                                         \
            if (best < 0 || before_##SUF(d, k, 0, bd, best, 0)) {                                \
                best = k;                                                                        \
                bd = d;                                                                          \
            }                                                                                    \
        }                                                                                        \
        *dist = bd;                                                                              \
        return best;                                                                             \
    }                                                                                            \
                                                                                                 \
    static int linkage_nn_##SUF(T *D, int32_t N, double *Z)                                       \
    {                                                                                            \
        int32_t *size = malloc(sizeof(int32_t) * (size_t)N);                                     \
        int32_t *id = malloc(sizeof(int32_t) * (size_t)N);                                       \
        int32_t *nn = malloc(sizeof(int32_t) * (size_t)N);                                       \
        T *nd = malloc(sizeof(T) * (size_t)N);                                                   \
        char *live = malloc((size_t)N);                                                          \
        if (!size || !id || !nn || !nd || !live) {                                               \
            free(size);                                                                          \
            free(id);                                                                            \
            free(nn);                                                                            \
            free(nd);                                                                            \
            free(live);                                                                          \
            return 2;                                                                            \
        }                                                                                        \
        for (int32_t k = 0; k < N; ++k) {                                                        \
            size[k] = 1;                                                                         \
            id[k] = k;                                                                           \
            live[k] = 1;                                                                         \
        }                                                                                        \
        for (int32_t k = 0; k < N; ++k)                                                          \
            nn[k] = nearest_##SUF(D, N, live, k, &nd[k]);                                        \
        for (int32_t m = 0; m + 1 < N; ++m) {                                                    \
            /* the row whose pair (smaller slot, larger slot) at the smallest                    \
               distance comes first */                                                           \
            int32_t a = -1, b = -1;                                                              \
            T best = 0;                                                                          \
            for (int32_t i = 0; i < N; ++i) {                                                    \
                if (!live[i])                                                                    \
                    continue;                                                                    \
                int32_t p = i < nn[i] ? i : nn[i], q = i < nn[i] ? nn[i] : i;                    \
                if (a < 0 || before_##SUF(nd[i], p, q, best, a, b)) {                           \
                    best = nd[i];                                                                \
                    a = p;                                                                       \
                    b = q;                                                                       \
                }                                                                                \
            }                                                                                    \
            merge_##SUF(D, N, live, a, b, size);                                                 \
            Z[4 * m + 0] = id[a] < id[b] ? id[a] : id[b];                                        \
            Z[4 * m + 1] = id[a] < id[b] ? id[b] : id[a];                                        \
            Z[4 * m + 2] = (double)best;                                                         \
            Z[4 * m + 3] = size[a];                                                              \
            id[a] = N + m;                                                                       \
            nn[a] = nearest_##SUF(D, N, live, a, &nd[a]);                                        \
            for (int32_t k = 0; k < N; ++k) {                                                    \
                if (!live[k] || k == a)                                                          \
                    continue;                                                                    \
                if (nn[k] == a || nn[k] == b) {                                                  \
                    nn[k] = nearest_##SUF(D, N, live, k, &nd[k]);                                \
                } else {                                                                         \
                    T d = D[(int64_t)k * N + a];                                                 \
                    if (before_##SUF(d, a, 0, nd[k], nn[k], 0)) {                                \
                        nn[k] = a;                                                               \
                        nd[k] = d;                                                               \
                    }                                                                            \
                }                                                                                \
            }                                                                                    \
        }                                                                                        \
        free(size);                                                                              \
        free(id);                                                                                \
        free(nn);                                                                                \
        free(nd);                                                                                \
        free(live);                                                                              \
        return 0;                                                                                \
    }

/* Merge slot b into slot a (a < b): distances of the merged cluster to every
 * other occupied slot, written to row a and column a; slot b emptied. */
#define MERGE_DEF(T, SUF)                                                                        \
    static void merge_##SUF(T *D, int32_t N, char *live, int32_t a, int32_t b, int32_t *size)   \
    {                                                                                            \
        T na = (T)size[a], nb = (T)size[b], n = (T)(size[a] + size[b]);                          \
        for (int32_t k = 0; k < N; ++k) {                                                        \
            if (!live[k] || k == a || k == b)                                                    \
                continue;                                                                        \
            T t = na * D[(int64_t)a * N + k];                                                    \
            T u = nb * D[(int64_t)b * N + k];                                                    \
            T s = t + u;                                                                         \
            T d = s / n;                                                                         \
            D[(int64_t)a * N + k] = d;                                                           \
            D[(int64_t)k * N + a] = d;                                                           \
        }                                                                                        \
        live[b] = 0;                                                                             \
        size[a] += size[b];                                                                      \
    }

MERGE_DEF(float, f32)
MERGE_DEF(double, f64)
LINKAGE_DEFS(float, f32)
LINKAGE_DEFS(double, f64)

/* Leaf order of the dendrogram: the leaves of the last merge's cluster from
 * left to right, each merge listing its smaller id first (the order in which
 * the usual dendrogram drawing lays out a linkage matrix). */
static void leaf_order(const double *Z, int32_t N, int32_t *order)
{
    if (N == 1) {
        order[0] = 0;
        return;
    }
    int32_t *stack = malloc(sizeof(int32_t) * (size_t)(2 * N));
    int32_t top = 0, out = 0;
    stack[top++] = 2 * N - 2;
    while (top > 0) {
        int32_t c = stack[--top];
        if (c < N) {
            order[out++] = c;
            continue;
        }
        const double *z = Z + 4 * (int64_t)(c - N);
        stack[top++] = (int32_t)z[1]; /* right, popped after the left subtree */
        stack[top++] = (int32_t)z[0];
    }
    free(stack);
}

/* Average linkage of the N x N symmetric matrix D (its diagonal is not
 * read). D is overwritten (its rows and columns of merged clusters hold the
 * merged distances). Z: [N-1][4] as described above; order: [N] leaf order
 * (may be NULL). is_f64: D holds doubles, else floats. naive: the O(N^3)
 * scan. Returns 0, 1 on a bad argument, 2 if memory ran out. */
int lso_average_linkage(void *D, int32_t N, int32_t is_f64, int32_t naive, double *Z,
                        int32_t *order)
{
    if (!D || N < 1 || !Z)
        return 1;
    int rc;
    if (is_f64)
        rc = naive ? linkage_naive_f64((double *)D, N, Z) : linkage_nn_f64((double *)D, N, Z);
    else
        rc = naive ? linkage_naive_f32((float *)D, N, Z) : linkage_nn_f32((float *)D, N, Z);
    if (rc == 0 && order)
        leaf_order(Z, N, order);
    return rc;
}

/* Standardised column of recipient i (section 2.2): over the donors j != i,
 * z_j = (e_j - mean) / sd with the mean and the population standard
 * deviation (divisor N - 1) of the e_j; z_i = 0. A column whose donor
 * entries are all equal has standard deviation 0 and standardises to 0
 * (tested as equality of the entries: their rounded mean need not equal
 * them exactly); a column with a NaN stays NaN. e, z: [N] FP64. */
void lso_standardise(const double *e, int32_t N, int32_t i, double *z)
{
    int all_equal = 1;
    double first = 0.0;
    int have = 0;
    for (int32_t j = 0; j < N; ++j) {
        if (j == i)
            continue;
        if (!have) {
            first = e[j];
            have = 1;
        } else if (!(e[j] == first)) {
            all_equal = 0;
        }
    }
    double s = 0.0;
    for (int32_t j = 0; j < N; ++j)
        if (j != i)
            s += e[j];
    double mean = s / (double)(N - 1);
    double v = 0.0;
    for (int32_t j = 0; j < N; ++j)
        if (j != i)
            v += (e[j] - mean) * (e[j] - mean);
    double sd = sqrt(v / (double)(N - 1));
    for (int32_t j = 0; j < N; ++j)
        z[j] = (j == i || all_equal) ? 0.0 : (e[j] - mean) / sd;
}
