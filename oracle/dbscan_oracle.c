/*
 * CPU oracle for exact DBSCAN.  TEST INFRASTRUCTURE ONLY: nothing on the
 * product path may link, load or call this file; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg use it.
 *
 * It computes DBSCAN as the paper's Section 3.1 defines it, by plain
 * pointwise eps range queries, and shares no code with the GPU library:
 *
 *   N(p)      = { q in P : dist(p, q) <= eps }            (closed ball, p in N(p))
 *   core(p)   = |N(p)| >= MinPts                            (Definition 1)
 *   clusters  = connected components of the graph on core points with an
 *               edge wherever dist <= eps                   (Definitions 2-5)
 *   border p  = non-core point with a core point within eps; it joins the
 *               cluster of its lowest-index core neighbour  (Section 3.1 text;
 *               the tie-break among several clusters is this project's)
 *   noise     = every other point, label -1.
 *
 * Cluster ids are canonical: the smallest input index among the cluster's
 * core points.  Coordinates are integers with |x| <= 2^24, so the squared
 * distance D = sum_j (x_pj - x_qj)^2 < 8 * 2^50 is exact in int64 and the
 * test dist <= eps is the exact integer test D <= eps^2.
 *
 * Two entry points compute the same result:
 *   oracle_dbscan_brute : O(n^2) over all pairs, no index (tiny inputs);
 *   oracle_dbscan       : buckets points in cells of side eps (so any
 *                         eps-neighbour lies in one of the 3^d adjacent
 *                         cells) and runs the same range queries there; the
 *                         core-graph components use a concurrent union-find
 *                         that always links the larger root under the
 *                         smaller, so each root is its component's smallest
 *                         core index.
 * A helper counts |N(p)| by brute force for sampled points at full size.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-3)

static inline int64_t sqdist(const int32_t *a, const int32_t *b, int d) {
    int64_t s = 0;
    for (int j = 0; j < d; ++j) {
        int64_t t = (int64_t)a[j] - (int64_t)b[j];
        s += t * t;
    }
    return s;
}

static int check_args(const int32_t *X, int64_t n, int32_t d, int64_t eps, int64_t minpts) {
    if (n < 0 || d < 1 || d > 16 || eps < 1 || minpts < 1) return ORACLE_EINVAL;
    if (n > 0 && X == NULL) return ORACLE_EINVAL;
    if (eps > 3037000499LL) return ORACLE_EINVAL; /* eps^2 must fit int64 */
    for (int64_t i = 0; i < n * d; ++i)
        if (X[i] > (1 << 24) || X[i] < -(1 << 24)) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- brute -- */

static int64_t uf_find_seq(int64_t *par, int64_t x) {
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

int oracle_dbscan_brute(const int32_t *X, int64_t n, int32_t d, int64_t eps,
                        int64_t minpts, int32_t *labels, uint8_t *core) {
    int rc = check_args(X, n, d, eps, minpts);
    if (rc) return rc;
    const int64_t T = eps * eps;
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!par) return ORACLE_ENOMEM;
    /* Definition 1: count the closed eps-ball, the point itself included. */
    for (int64_t p = 0; p < n; ++p) {
        int64_t cnt = 0;
        for (int64_t q = 0; q < n; ++q)
            if (sqdist(X + p * d, X + q * d, d) <= T) ++cnt;
        core[p] = (uint8_t)(cnt >= minpts);
        par[p] = p;
    }
    /* Components of the core eps-graph. */
    for (int64_t p = 0; p < n; ++p) {
        if (!core[p]) continue;
        for (int64_t q = p + 1; q < n; ++q) {
            if (!core[q] || sqdist(X + p * d, X + q * d, d) > T) continue;
            int64_t a = uf_find_seq(par, p), b = uf_find_seq(par, q);
            if (a == b) continue;
            if (a < b) par[b] = a; else par[a] = b; /* root = smallest index */
        }
    }
    for (int64_t p = 0; p < n; ++p)
        labels[p] = core[p] ? (int32_t)uf_find_seq(par, p) : -1;
    /* Non-core points: the lowest-index core point within eps decides. */
    for (int64_t p = 0; p < n; ++p) {
        if (core[p]) continue;
        for (int64_t q = 0; q < n; ++q) {
            if (core[q] && sqdist(X + p * d, X + q * d, d) <= T) {
                labels[p] = (int32_t)uf_find_seq(par, q);
                break;
            }
        }
    }
    free(par);
    return ORACLE_OK;
}

/* ------------------------------------------------------------ eps cells -- */

typedef struct {
    int64_t n, ncell;
    int32_t d;
    int32_t *cc;      /* ncell x d: integer cell coordinates, sorted lexicographically */
    int64_t *start;   /* ncell + 1: first position of each cell in `order` */
    int64_t *order;   /* n: point indices grouped by cell, ascending index within a cell */
    int64_t *cell_of; /* n: cell of each point */
    int32_t *pc;      /* n x d: cell coordinates of each point */
    int32_t *xs;      /* n x d: coordinates in `order` (cell-grouped) order */
} ecells;

static const ecells *g_sort_ctx; /* qsort has no context argument */

static int cmp_point_cell(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, k = *(const int64_t *)b;
    const int32_t *ci = g_sort_ctx->pc + i * g_sort_ctx->d;
    const int32_t *ck = g_sort_ctx->pc + k * g_sort_ctx->d;
    for (int j = 0; j < g_sort_ctx->d; ++j) {
        if (ci[j] != ck[j]) return ci[j] < ck[j] ? -1 : 1;
    }
    return (i > k) - (i < k);
}

static void free_cells(ecells *c) {
    free(c->cc); free(c->start); free(c->order); free(c->cell_of); free(c->pc); free(c->xs);
    memset(c, 0, sizeof(*c));
}

/* Cells of side eps: cell coordinate floor((x_j - min_j) / eps). */
static int build_cells(const int32_t *X, int64_t n, int32_t d, int64_t eps, ecells *c) {
    memset(c, 0, sizeof(*c));
    c->n = n; c->d = d;
    size_t nn = (size_t)(n > 0 ? n : 1);
    c->pc = (int32_t *)malloc(sizeof(int32_t) * nn * d);
    c->order = (int64_t *)malloc(sizeof(int64_t) * nn);
    c->cell_of = (int64_t *)malloc(sizeof(int64_t) * nn);
    c->start = (int64_t *)malloc(sizeof(int64_t) * (nn + 1));
    c->cc = (int32_t *)malloc(sizeof(int32_t) * nn * d);
    c->xs = (int32_t *)malloc(sizeof(int32_t) * nn * d);
    if (!c->pc || !c->order || !c->cell_of || !c->start || !c->cc || !c->xs) { free_cells(c); return ORACLE_ENOMEM; }
    int32_t mn[16];
    for (int j = 0; j < d; ++j) mn[j] = n > 0 ? X[j] : 0;
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j)
            if (X[i * d + j] < mn[j]) mn[j] = X[i * d + j];
    for (int64_t i = 0; i < n; ++i) {
        c->order[i] = i;
        for (int j = 0; j < d; ++j)
            c->pc[i * d + j] = (int32_t)(((int64_t)X[i * d + j] - mn[j]) / eps);
    }
    g_sort_ctx = c;
    qsort(c->order, (size_t)n, sizeof(int64_t), cmp_point_cell);
    int64_t ncell = 0;
    for (int64_t r = 0; r < n; ++r) {
        int64_t i = c->order[r];
        int is_new = (r == 0) || memcmp(c->pc + i * d, c->pc + c->order[r - 1] * d, sizeof(int32_t) * d) != 0;
        if (is_new) {
            memcpy(c->cc + ncell * d, c->pc + i * d, sizeof(int32_t) * d);
            c->start[ncell++] = r;
        }
        c->cell_of[i] = ncell - 1;
        memcpy(c->xs + r * d, X + i * d, sizeof(int32_t) * d);
    }
    c->start[ncell] = n;
    c->ncell = ncell;
    return ORACLE_OK;
}

static int cmp_cc(const int32_t *a, const int32_t *b, int d) {
    for (int j = 0; j < d; ++j)
        if (a[j] != b[j]) return a[j] < b[j] ? -1 : 1;
    return 0;
}

/* Index of the cell with coordinates `key`, or -1 (binary search). */
static int64_t find_cell(const ecells *c, const int32_t *key) {
    int64_t lo = 0, hi = c->ncell - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int r = cmp_cc(c->cc + mid * c->d, key, c->d);
        if (r == 0) return mid;
        if (r < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* The (up to 3^d) non-empty cells adjacent to cell `ci`, itself included. */
static int64_t adjacent_cells(const ecells *c, int64_t ci, int64_t *out) {
    const int d = c->d;
    int64_t total = 1, cnt = 0;
    for (int j = 0; j < d; ++j) total *= 3;
    int32_t key[16];
    for (int64_t code = 0; code < total; ++code) {
        int64_t t = code;
        for (int j = 0; j < d; ++j) {
            key[j] = c->cc[ci * d + j] + (int32_t)(t % 3) - 1;
            t /= 3;
        }
        int64_t k = find_cell(c, key);
        if (k >= 0) out[cnt++] = k;
    }
    return cnt;
}

/* Concurrent union-find on point indices: a root's parent only ever moves
 * from itself to a smaller index, by compare-and-swap, so there are no
 * cycles and every root is the smallest index of its component. */
static int64_t uf_find(int64_t *par, int64_t x) {
    for (;;) {
        int64_t p = __atomic_load_n(&par[x], __ATOMIC_ACQUIRE);
        if (p == x) return x;
        x = p;
    }
}

static void uf_unite(int64_t *par, int64_t a, int64_t b) {
    for (;;) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a > b) { int64_t t = a; a = b; b = t; }
        int64_t expect = b;
        if (__atomic_compare_exchange_n(&par[b], &expect, a, 0, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE))
            return;
    }
}

int oracle_dbscan(const int32_t *X, int64_t n, int32_t d, int64_t eps, int64_t minpts,
                  int32_t *labels, uint8_t *core, int32_t nthreads) {
    int rc = check_args(X, n, d, eps, minpts);
    if (rc) return rc;
    if (n == 0) return ORACLE_OK;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t T = eps * eps;
    ecells c;
    rc = build_cells(X, n, d, eps, &c);
    if (rc) return rc;
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!par) { free_cells(&c); return ORACLE_ENOMEM; }
    int64_t max_adj = 1;
    for (int j = 0; j < d; ++j) max_adj *= 3;
    int failed = 0;

    /* Definition 1 for every point: |N(p)| >= MinPts. */
#pragma omp parallel
    {
        int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)max_adj);
        if (!adj) { __atomic_store_n(&failed, 1, __ATOMIC_RELAXED); }
#pragma omp for schedule(dynamic, 16)
        for (int64_t ci = 0; ci < c.ncell; ++ci) {
            if (!adj) continue;
            int64_t na = adjacent_cells(&c, ci, adj);
            for (int64_t r = c.start[ci]; r < c.start[ci + 1]; ++r) {
                int64_t p = c.order[r];
                int64_t cnt = 0;
                for (int64_t a = 0; a < na && cnt < minpts; ++a)
                    for (int64_t s = c.start[adj[a]]; s < c.start[adj[a] + 1]; ++s)
                        cnt += sqdist(c.xs + r * d, c.xs + s * d, d) <= T;
                core[p] = (uint8_t)(cnt >= minpts);
                par[p] = p;
            }
        }
        free(adj);
    }
    if (failed) { free(par); free_cells(&c); return ORACLE_ENOMEM; }

    /* Components of the core eps-graph: unite every core pair within eps. */
#pragma omp parallel
    {
        int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)max_adj);
        if (!adj) { __atomic_store_n(&failed, 1, __ATOMIC_RELAXED); }
#pragma omp for schedule(dynamic, 16)
        for (int64_t ci = 0; ci < c.ncell; ++ci) {
            if (!adj) continue;
            int64_t na = adjacent_cells(&c, ci, adj);
            for (int64_t r = c.start[ci]; r < c.start[ci + 1]; ++r) {
                int64_t p = c.order[r];
                if (!core[p]) continue;
                for (int64_t a = 0; a < na; ++a) {
                    if (adj[a] < ci) continue; /* each pair of cells once */
                    for (int64_t s = c.start[adj[a]]; s < c.start[adj[a] + 1]; ++s) {
                        if (s <= r) continue;  /* each pair of points once */
                        int64_t q = c.order[s];
                        if (core[q] && sqdist(c.xs + r * d, c.xs + s * d, d) <= T)
                            uf_unite(par, p, q);
                    }
                }
            }
        }
        free(adj);
    }
    if (failed) { free(par); free_cells(&c); return ORACLE_ENOMEM; }

    /* Labels: a core point takes its root (the component's smallest core
     * index); a non-core point takes the root of its lowest-index core
     * neighbour, or -1. */
#pragma omp parallel
    {
        int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)max_adj);
        if (!adj) { __atomic_store_n(&failed, 1, __ATOMIC_RELAXED); }
#pragma omp for schedule(dynamic, 16)
        for (int64_t ci = 0; ci < c.ncell; ++ci) {
            if (!adj) continue;
            int64_t na = adjacent_cells(&c, ci, adj);
            for (int64_t r = c.start[ci]; r < c.start[ci + 1]; ++r) {
                int64_t p = c.order[r];
                if (core[p]) { labels[p] = (int32_t)uf_find(par, p); continue; }
                int64_t best = -1;
                for (int64_t a = 0; a < na; ++a)
                    for (int64_t s = c.start[adj[a]]; s < c.start[adj[a] + 1]; ++s) {
                        int64_t q = c.order[s];
                        if (core[q] && (best < 0 || q < best) && sqdist(c.xs + r * d, c.xs + s * d, d) <= T)
                            best = q;
                    }
                labels[p] = best < 0 ? -1 : (int32_t)uf_find(par, best);
            }
        }
        free(adj);
    }
    free(par);
    free_cells(&c);
    return failed ? ORACLE_ENOMEM : ORACLE_OK;
}

/* |N(p)| by brute force over all n points, for each queried index. */
int oracle_neighbor_count_brute(const int32_t *X, int64_t n, int32_t d, int64_t eps,
                                const int64_t *qidx, int64_t nq, int64_t *counts, int32_t nthreads) {
    if (n < 0 || d < 1 || d > 16 || eps < 1 || nq < 0) return ORACLE_EINVAL;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t T = eps * eps;
    for (int64_t k = 0; k < nq; ++k)
        if (qidx[k] < 0 || qidx[k] >= n) return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nq; ++k) {
        const int32_t *p = X + qidx[k] * d;
        int64_t cnt = 0;
        for (int64_t q = 0; q < n; ++q)
            cnt += sqdist(p, X + q * d, d) <= T;
        counts[k] = cnt;
    }
    return ORACLE_OK;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
