/*
 * Oracle for exact density-peaks clustering: the plain O(n^2) method in C.
 *
 * TEST INFRASTRUCTURE.  Loaded only by tests, the smoke check and the CPU
 * baseline of the benchmark, through oracle/scan.py.  It shares no code, header
 * or constant with the HIP library.
 *
 * It follows the paper's straightforward algorithm (Section 2.2, steps 1-4)
 * for the quantities of Definitions 1-6 (Section 2.1), with the same readings
 * as oracle/dpc_oracle.py:
 *   - D2 is the exact int64 squared Euclidean distance of integer points;
 *   - rho_i = #{ j : D2(i,j) < R }, R = ceil(d_cut^2) supplied exactly by the
 *     caller, j = i included (Def. 1, Eq. 1);
 *   - "higher" is the strict order (rho descending, id ascending);
 *   - dep_i is the higher point with the smallest (D2, id), -1 for the densest
 *     point (Defs. 2-3); delta_i = sqrt((double)D2), +inf for the densest;
 *   - noise: rho < rho_min (Def. 4); center: non-noise with delta >= delta_min
 *     (Def. 5); labels by depth-first propagation from centers along reverse
 *     dependency lists (Def. 6 and step 4), -1 for noise.
 * The only parallelism is an OpenMP loop over independent query points.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t sqdist(const int32_t *a, const int32_t *b, int d) {
    int64_t s = 0;
    for (int t = 0; t < d; t++) {
        int64_t df = (int64_t)a[t] - (int64_t)b[t];
        s += df * df;
    }
    return s;
}

/* Step 1 / Def. 1: a linear scan of P for every point. */
void oracle_rho(const int32_t *pts, int64_t n, int32_t d, int64_t R, int32_t *rho) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        const int32_t *a = pts + i * d;
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++)
            c += sqdist(a, pts + j * d, d) < R;
        rho[i] = (int32_t)c;
    }
}

/* Def. 1 for the listed points only. */
void oracle_rho_of(const int32_t *pts, int64_t n, int32_t d, int64_t R,
                   const int64_t *which, int64_t m, int32_t *rho) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < m; k++) {
        const int32_t *a = pts + which[k] * d;
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++)
            c += sqdist(a, pts + j * d, d) < R;
        rho[k] = (int32_t)c;
    }
}

static const int32_t *g_rho; /* comparator context for qsort */

static int by_density(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    if (g_rho[a] != g_rho[b]) return g_rho[a] > g_rho[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

/* Step 2: order[r] = id at position r of the density-descending order. */
void oracle_order(const int32_t *rho, int64_t n, int64_t *order) {
    for (int64_t i = 0; i < n; i++) order[i] = i;
    g_rho = rho;
    qsort(order, (size_t)n, sizeof(int64_t), by_density);
}

/* Step 3 / Defs. 2-3: scan the sorted array up to the point itself.  As in
 * step 2, the points themselves are put in density order (sorted[k] is the
 * point order[k]), so the scan of every prefix reads memory in sequence. */
void oracle_dependent(const int32_t *pts, int64_t n, int32_t d, const int32_t *rho,
                      int32_t *dep, int64_t *d2) {
    int64_t *order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *rank = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *sorted = (int32_t *)malloc((size_t)n * (size_t)d * sizeof(int32_t));
    oracle_order(rho, n, order);
    for (int64_t r = 0; r < n; r++) {
        rank[order[r]] = r;
        memcpy(sorted + r * d, pts + order[r] * d, (size_t)d * sizeof(int32_t));
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        const int32_t *a = pts + i * d;
        int64_t best = INT64_MAX, bj = -1;
        for (int64_t k = 0; k < rank[i]; k++) {
            int64_t j = order[k];
            int64_t s = sqdist(a, sorted + k * d, d);
            if (s < best || (s == best && j < bj)) {
                best = s;
                bj = j;
            }
        }
        dep[i] = (int32_t)bj;
        d2[i] = best;
    }
    free(order);
    free(rank);
    free(sorted);
}

typedef struct {
    int64_t d2, id;
} cand_t;

static int by_distance(const void *x, const void *y) {
    const cand_t *a = (const cand_t *)x, *b = (const cand_t *)y;
    if (a->d2 != b->d2) return a->d2 < b->d2 ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/*
 * Defs. 1-3 for the listed points only, without the densities of all points:
 * visit the other points by increasing (D2, id) and return the first whose
 * own density (counted on demand, Def. 1) ranks higher.  Exact, and cheap when
 * the dependent point is near, which is the common case.  With max_walk > 0,
 * a point not decided after max_walk candidates gets dep = -2 (undecided).
 */
void oracle_dependent_of(const int32_t *pts, int64_t n, int32_t d, int64_t R,
                         const int64_t *which, int64_t m, int64_t max_walk,
                         int32_t *rho_out, int32_t *dep, int64_t *d2) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < m; k++) {
        int64_t i = which[k];
        const int32_t *a = pts + i * d;
        cand_t *c = (cand_t *)malloc((size_t)n * sizeof(cand_t));
        int64_t rho_i = 0;
        for (int64_t j = 0; j < n; j++) {
            c[j].d2 = sqdist(a, pts + j * d, d);
            c[j].id = j;
            rho_i += c[j].d2 < R;
        }
        qsort(c, (size_t)n, sizeof(cand_t), by_distance);
        int64_t bj = -1, best = INT64_MAX, walked = 0;
        for (int64_t t = 0; t < n; t++) {
            int64_t j = c[t].id;
            if (j == i) continue;
            if (max_walk > 0 && ++walked > max_walk) {
                bj = -2; /* undecided within the walk limit */
                break;
            }
            const int32_t *b = pts + j * d;
            int64_t rho_j = 0;
            for (int64_t u = 0; u < n; u++)
                rho_j += sqdist(b, pts + u * d, d) < R;
            if (rho_j > rho_i || (rho_j == rho_i && j < i)) {
                bj = j;
                best = c[t].d2;
                break;
            }
        }
        rho_out[k] = (int32_t)rho_i;
        dep[k] = (int32_t)bj;
        d2[k] = best;
        free(c);
    }
}

/* Def. 3. */
void oracle_delta(const int64_t *d2, int64_t n, double *delta) {
    for (int64_t i = 0; i < n; i++)
        delta[i] = d2[i] == INT64_MAX ? INFINITY : sqrt((double)d2[i]);
}

/* Step 4 / Defs. 4-6: noise, centers, then depth-first propagation from each
 * center along the reverse dependency lists.  Returns the number of centers. */
int64_t oracle_labels(const int32_t *rho, const int32_t *dep, const double *delta, int64_t n,
                      int32_t rho_min, double delta_min, int32_t *label) {
    int64_t *head = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *kids = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *stack = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++)
        if (dep[i] >= 0) head[dep[i] + 1]++;
    for (int64_t i = 0; i < n; i++) head[i + 1] += head[i];
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    memcpy(fill, head, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++)
        if (dep[i] >= 0) kids[fill[dep[i]]++] = i;
    free(fill);

    int64_t centers = 0;
    for (int64_t i = 0; i < n; i++) label[i] = -1;
    for (int64_t c = 0; c < n; c++) {
        if (rho[c] < rho_min || !(delta[c] >= delta_min)) continue;
        centers++;
        label[c] = (int32_t)c;
        int64_t top = 0;
        stack[top++] = c;
        while (top) {
            int64_t u = stack[--top];
            for (int64_t e = head[u]; e < head[u + 1]; e++) {
                int64_t v = kids[e];
                int noise = rho[v] < rho_min;
                int center = !noise && delta[v] >= delta_min;
                if (!noise && !center) {
                    label[v] = (int32_t)c;
                    stack[top++] = v;
                }
            }
        }
    }
    free(head);
    free(kids);
    free(stack);
    return centers;
}
