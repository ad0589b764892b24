/*
 * oracle.c - plain CPU DBSCAN, written from the definition.
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the GPU library never links, loads or calls it, and
 * it shares no code, header or table with the GPU library.
 *
 * What it computes (the DBSCAN definition of Section 2.1 of the paper):
 *   N_eps(x) = { y in X : dist(x, y) <= eps }         (x itself included)
 *   core(x)  <=> |N_eps(x)| >= minPts
 *   clusters = connected components of the graph on core points whose
 *              edges join cores within eps of each other
 *   border   = non-core point within eps of some core point; it may reach
 *              several clusters, and the paper leaves the choice open
 *   noise    = every other point.
 *
 * Output encoding (the paper is silent here; this is the canonical reading):
 *   cluster ids 0..K-1 in increasing order of the smallest input index among
 *   each cluster's core points; a border point takes the smallest id among the
 *   clusters that hold a core point within eps of it; noise is -1.
 *
 * The distance test. The paper fixes neither precision nor evaluation order.
 * The test decides an integer outcome (neighbour or not), so both this oracle
 * and the GPU kernels take it in the kernels' precision, fp32, in one fixed
 * order: dx = p.x-q.x, dy = p.y-q.y, dz = p.z-q.z (each rounded);
 * s = (dx*dx + dy*dy) + dz*dz with every product and sum rounded separately
 * (no fused multiply-add); neighbour <=> s <= fl32(eps*eps). 2D drops dz.
 * Build with -ffp-contract=off and without fast-math, so gcc keeps that order.
 *
 * Neighbour enumeration. The brute mode tests every ordered pair. The grid
 * mode only skips pairs that cannot pass the test: points are bucketed into
 * cubic cells of side 1.001*eps (cell index computed in fp64); a pair that
 * passes the fp32 test has |p_k - q_k| <= eps*(1 + 2^-22) in every coordinate,
 * so it lies in the same or an adjacent cell. The brute mode is the grid mode
 * with one cell holding every point, and tests pin the two against each other.
 * Nothing else differs between the modes.
 *
 * Components are found with a sequential union-find over core pairs; union
 * is skipped when both ends already share a root (this changes nothing in the
 * result, only the work). Counting and the border scan run on OpenMP threads;
 * they only read shared data.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- the distance test ------------------------------------------------- */

int oracle_pred(const float *p, const float *q, int dim, float eps2)
{
    float dx = p[0] - q[0];
    float dy = p[1] - q[1];
    float s = dx * dx;
    float t = dy * dy;
    s = s + t;
    if (dim == 3) {
        float dz = p[2] - q[2];
        float u = dz * dz;
        s = s + u;
    }
    return s <= eps2;
}

float oracle_eps2(float eps)
{
    float e2 = eps * eps;
    return e2;
}

/* ---- cells -------------------------------------------------------------- */

typedef struct {
    int64_t n_cells;
    int64_t *cell_start;   /* [n_cells+1] offsets into order[] */
    int32_t *order;        /* [n] point indices grouped by cell */
    int64_t *cell_of;      /* [n] cell id of each point */
    int64_t *nbr;          /* [n_cells * 3^dim] neighbour cell ids, -1 = none */
    int n_nbr;             /* 3^dim, or 1 in brute mode */
} grid_t;

typedef struct {
    int64_t c[3];
    int32_t idx;
} keyed_t;

static int g_dim_for_cmp;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    for (int k = 0; k < g_dim_for_cmp; ++k) {
        if (x->c[k] < y->c[k]) return -1;
        if (x->c[k] > y->c[k]) return 1;
    }
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int cmp_coords(const int64_t *a, const int64_t *b, int dim)
{
    for (int k = 0; k < dim; ++k) {
        if (a[k] < b[k]) return -1;
        if (a[k] > b[k]) return 1;
    }
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->cell_start);
    free(g->order);
    free(g->cell_of);
    free(g->nbr);
    memset(g, 0, sizeof(*g));
}

/* One cell holding every point: each point's candidate set is all of X. */
static int grid_build_single(grid_t *g, int64_t n)
{
    memset(g, 0, sizeof(*g));
    g->n_cells = 1;
    g->n_nbr = 1;
    g->cell_start = (int64_t *)malloc(2 * sizeof(int64_t));
    g->order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    g->cell_of = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    g->nbr = (int64_t *)malloc(sizeof(int64_t));
    if (!g->cell_start || !g->order || !g->cell_of || !g->nbr) return -1;
    g->cell_start[0] = 0;
    g->cell_start[1] = n;
    for (int64_t i = 0; i < n; ++i) g->order[i] = (int32_t)i;
    g->nbr[0] = 0;
    return 0;
}

static int grid_build(grid_t *g, const float *pts, int64_t n, int dim, float eps)
{
    memset(g, 0, sizeof(*g));
    if (n == 0) return grid_build_single(g, n);
    double side = 1.001 * (double)eps;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { lo[k] = pts[k]; hi[k] = pts[k]; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            double v = pts[i * dim + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    for (int k = 0; k < dim; ++k)
        if (!((hi[k] - lo[k]) / side < 4.0e18)) return grid_build_single(g, n);

    keyed_t *kv = (keyed_t *)malloc((size_t)n * sizeof(keyed_t));
    if (!kv) return -1;
    for (int64_t i = 0; i < n; ++i) {
        kv[i].c[0] = kv[i].c[1] = kv[i].c[2] = 0;
        for (int k = 0; k < dim; ++k)
            kv[i].c[k] = (int64_t)floor(((double)pts[i * dim + k] - lo[k]) / side);
        kv[i].idx = (int32_t)i;
    }
    g_dim_for_cmp = dim;
    qsort(kv, (size_t)n, sizeof(keyed_t), cmp_keyed);

    int64_t n_cells = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || cmp_coords(kv[i].c, kv[i - 1].c, dim) != 0) ++n_cells;
    g->n_cells = n_cells;
    g->n_nbr = (dim == 3) ? 27 : 9;
    g->cell_start = (int64_t *)malloc((size_t)(n_cells + 1) * sizeof(int64_t));
    g->order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    g->cell_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    g->nbr = (int64_t *)malloc((size_t)n_cells * g->n_nbr * sizeof(int64_t));
    int64_t (*coords)[3] = malloc((size_t)n_cells * sizeof(*coords));
    if (!g->cell_start || !g->order || !g->cell_of || !g->nbr || !coords) {
        free(kv); free(coords); grid_free(g); return -1;
    }
    int64_t c = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || cmp_coords(kv[i].c, kv[i - 1].c, dim) != 0) {
            ++c;
            g->cell_start[c] = i;
            memcpy(coords[c], kv[i].c, sizeof(coords[c]));
        }
        g->order[i] = kv[i].idx;
        g->cell_of[kv[i].idx] = c;
    }
    g->cell_start[n_cells] = n;
    free(kv);

    #pragma omp parallel for schedule(static)
    for (int64_t cc = 0; cc < n_cells; ++cc) {
        int t = 0;
        for (int oz = (dim == 3 ? -1 : 0); oz <= (dim == 3 ? 1 : 0); ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int64_t want[3] = {coords[cc][0] + ox, coords[cc][1] + oy, coords[cc][2] + oz};
                    int64_t a = 0, b = n_cells - 1, hit = -1;
                    while (a <= b) {
                        int64_t mid = a + (b - a) / 2;
                        int r = cmp_coords(coords[mid], want, dim);
                        if (r == 0) { hit = mid; break; }
                        if (r < 0) a = mid + 1; else b = mid - 1;
                    }
                    g->nbr[cc * g->n_nbr + t++] = hit;
                }
    }
    free(coords);
    return 0;
}

/* ---- union-find (sequential) --------------------------------------------- */

static int32_t uf_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

static void uf_union(int32_t *parent, int32_t a, int32_t b)
{
    int32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra; else parent[ra] = rb;
}

/* ---- neighbour counts ---------------------------------------------------- */

static void count_all(const grid_t *g, const float *pts, int64_t n, int dim, float eps2,
                      int32_t *counts)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const float *p = pts + i * dim;
        int64_t ci = g->cell_of[i];
        int32_t cnt = 0;
        for (int t = 0; t < g->n_nbr; ++t) {
            int64_t cj = g->nbr[ci * g->n_nbr + t];
            if (cj < 0) continue;
            for (int64_t s = g->cell_start[cj]; s < g->cell_start[cj + 1]; ++s) {
                int32_t j = g->order[s];
                cnt += oracle_pred(p, pts + (int64_t)j * dim, dim, eps2);
            }
        }
        counts[i] = cnt;
    }
}

/* |N_eps(x)| for every point (x included). mode: 0 = brute, 1 = grid. */
int oracle_neighbor_counts(const float *pts, int64_t n, int dim, float eps, int mode,
                           int threads, int32_t *counts)
{
    if (n < 0 || (dim != 2 && dim != 3)) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    grid_t g;
    int rc = mode ? grid_build(&g, pts, n, dim, eps) : grid_build_single(&g, n);
    if (rc) return -2;
    count_all(&g, pts, n, dim, oracle_eps2(eps), counts);
    grid_free(&g);
    return 0;
}

/* ---- DBSCAN --------------------------------------------------------------- */

/*
 * labels[n] (int32, -1 = noise, else 0..K-1 canonical) and is_core[n] (0/1).
 * mode: 0 = brute, 1 = grid. threads: OpenMP threads (<=0: runtime default).
 * Returns K >= 0, or a negative error code.
 */
int64_t oracle_dbscan(const float *pts, int64_t n, int dim, float eps, int32_t min_pts,
                      int mode, int threads, int32_t *labels, uint8_t *is_core)
{
    if (n < 0 || n > INT32_MAX || (dim != 2 && dim != 3) || min_pts < 1) return -1;
    if (n == 0) return 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    const float eps2 = oracle_eps2(eps);
    grid_t g;
    int rc = mode ? grid_build(&g, pts, n, dim, eps) : grid_build_single(&g, n);
    if (rc) return -2;

    int32_t *counts = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *parent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *root = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *cid = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!counts || !parent || !root || !cid) {
        free(counts); free(parent); free(root); free(cid); grid_free(&g); return -2;
    }

    /* core points: |N_eps(x)| >= minPts */
    count_all(&g, pts, n, dim, eps2, counts);
    for (int64_t i = 0; i < n; ++i) is_core[i] = counts[i] >= min_pts;

    /* connected components of the core graph */
    for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i) {
        if (!is_core[i]) continue;
        const float *p = pts + i * dim;
        int64_t ci = g.cell_of[i];
        for (int t = 0; t < g.n_nbr; ++t) {
            int64_t cj = g.nbr[ci * g.n_nbr + t];
            if (cj < 0) continue;
            for (int64_t s = g.cell_start[cj]; s < g.cell_start[cj + 1]; ++s) {
                int32_t j = g.order[s];
                if (j <= i || !is_core[j]) continue;
                if (uf_find(parent, (int32_t)i) == uf_find(parent, j)) continue;
                if (oracle_pred(p, pts + (int64_t)j * dim, dim, eps2))
                    uf_union(parent, (int32_t)i, j);
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) root[i] = uf_find(parent, (int32_t)i);

    /* canonical cluster ids: order of the smallest input index among cores */
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) cid[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (!is_core[i]) continue;
        if (cid[root[i]] < 0) cid[root[i]] = (int32_t)k++;
        labels[i] = cid[root[i]];
    }

    /* border points take the smallest id among reachable clusters; else noise */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (is_core[i]) continue;
        const float *p = pts + i * dim;
        int64_t ci = g.cell_of[i];
        int32_t best = INT32_MAX;
        for (int t = 0; t < g.n_nbr; ++t) {
            int64_t cj = g.nbr[ci * g.n_nbr + t];
            if (cj < 0) continue;
            for (int64_t s = g.cell_start[cj]; s < g.cell_start[cj + 1]; ++s) {
                int32_t j = g.order[s];
                if (!is_core[j]) continue;
                int32_t c = cid[root[j]];
                if (c < best && oracle_pred(p, pts + (int64_t)j * dim, dim, eps2)) best = c;
            }
        }
        labels[i] = (best == INT32_MAX) ? -1 : best;
    }

    free(counts); free(parent); free(root); free(cid);
    grid_free(&g);
    return k;
}

/*
 * Checks a clustering's non-core points against the definition, for outputs
 * whose border choice is free (first-come assignment): every non-core point
 * with a label must have a core point of that same label within eps, and
 * every non-core point labelled noise (-1) must have no core point within eps.
 * Returns the number of violating points (>= 0), or a negative error code.
 */
int64_t oracle_check_border(const float *pts, int64_t n, int dim, float eps, const uint8_t *is_core,
                            const int32_t *labels, int mode, int threads)
{
    if (n < 0 || (dim != 2 && dim != 3)) return -1;
    if (n == 0) return 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    const float eps2 = oracle_eps2(eps);
    grid_t g;
    int rc = mode ? grid_build(&g, pts, n, dim, eps) : grid_build_single(&g, n);
    if (rc) return -2;
    int64_t bad = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
    for (int64_t i = 0; i < n; ++i) {
        if (is_core[i]) continue;
        const float *p = pts + i * dim;
        int64_t ci = g.cell_of[i];
        int any_core = 0, same = 0;
        for (int t = 0; t < g.n_nbr && !same; ++t) {
            int64_t cj = g.nbr[ci * g.n_nbr + t];
            if (cj < 0) continue;
            for (int64_t s = g.cell_start[cj]; s < g.cell_start[cj + 1]; ++s) {
                int32_t j = g.order[s];
                if (!is_core[j] || !oracle_pred(p, pts + (int64_t)j * dim, dim, eps2)) continue;
                any_core = 1;
                if (labels[j] == labels[i]) { same = 1; break; }
            }
        }
        if (labels[i] < 0 ? any_core : !same) ++bad;
    }
    grid_free(&g);
    return bad;
}

/*
 * Brute force over all n points for one query: the indices j with the query
 * within eps of point j (query itself included), in increasing order.
 * Writes at most cap indices; returns the full count.
 */
int64_t oracle_neighbors_of(const float *pts, int64_t n, int dim, float eps, int64_t i, int64_t *out,
                            int64_t cap)
{
    if (n < 0 || i < 0 || i >= n || (dim != 2 && dim != 3)) return -1;
    const float eps2 = oracle_eps2(eps);
    const float *p = pts + i * dim;
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (!oracle_pred(p, pts + j * dim, dim, eps2)) continue;
        if (k < cap) out[k] = j;
        ++k;
    }
    return k;
}
