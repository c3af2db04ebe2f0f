/*
 * CPU oracle for fixed-radius neighbour search (test infrastructure only).
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code, header or constant with the GPU path.
 *
 * What it computes (the plain definition the GPU path must reach exactly):
 *   N(i) = { j != i : r2(i,j) <= R*R }
 * with, in binary64 round-to-nearest and no fused multiply-add,
 *   dx_k = P[j][k] - P[i][k]
 *   r2   = ((dx_0*dx_0) + (dx_1*dx_1)) + (dx_2*dx_2)      (last term only in 3D)
 * Rows are emitted as CSR: row_ptr (int64, n+1 entries), col ascending (int32),
 * dist = (float) sqrt(r2).
 *
 * Sources in the paper:
 *   - neighbours are the particles inside the search radius 2h of particle i
 *     (SPH method section, Eq. 2 and the text after it);
 *   - all-list search: every particle is compared with every other one,
 *     N(N-1) comparisons (SPH method section, Fig. 3a text);
 *   - cell link-list search: a uniform background grid with cell size equal to
 *     the search radius; particles are assigned to cells and only the same and
 *     adjacent cells are checked (SPH method section, Fig. 3b text).
 * Readings where the paper is silent: the cutoff is inclusive; the particle
 * itself is excluded; coincident particles are neighbours; the row order is
 * ascending index.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -ffast-math, no -march=native).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDOMAIN (-2)
#define ORC_ENOMEM (-3)

typedef struct {
    int64_t n, nnz;
    int64_t *row_ptr; /* n+1 */
    int32_t *col;     /* nnz */
    float *dist;      /* nnz */
} orc_result;

typedef struct { int32_t j; float d; } orc_pair;

/* growable pair buffer */
typedef struct { orc_pair *v; int64_t len, cap; } orc_vec;

static int vec_push(orc_vec *b, int32_t j, float d)
{
    if (b->len == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 1024;
        orc_pair *nv = (orc_pair *)realloc(b->v, (size_t)nc * sizeof(orc_pair));
        if (!nv) return ORC_ENOMEM;
        b->v = nv;
        b->cap = nc;
    }
    b->v[b->len].j = j;
    b->v[b->len].d = d;
    b->len++;
    return ORC_OK;
}

static int cmp_pair(const void *a, const void *b)
{
    int32_t x = ((const orc_pair *)a)->j, y = ((const orc_pair *)b)->j;
    return (x > y) - (x < y);
}

/* The pair predicate, written out once: r2 in the fixed left-to-right order. */
static double pair_r2(int dim, const double *pi, const double *pj)
{
    double d0 = pj[0] - pi[0];
    double d1 = pj[1] - pi[1];
    double r2 = d0 * d0;
    double t = d1 * d1;
    r2 = r2 + t;
    if (dim == 3) {
        double d2 = pj[2] - pi[2];
        t = d2 * d2;
        r2 = r2 + t;
    }
    return r2;
}

/* Validation shared by both searches: dim in {2,3}; 0 <= n < 2^31; hi > lo;
 * 0 < radius <= cell_size; all finite; every position inside [lo, hi]. */
static int validate(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                    double cell_size, double radius)
{
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    if (n < 0 || n >= ((int64_t)1 << 31)) return ORC_EINVAL;
    if (!(radius > 0.0) || !(cell_size >= radius) || !isfinite(cell_size)) return ORC_EINVAL;
    for (int k = 0; k < dim; k++)
        if (!isfinite(lo[k]) || !isfinite(hi[k]) || !(hi[k] > lo[k])) return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < dim; k++) {
            double p = pos[i * dim + k];
            if (!(p >= lo[k] && p <= hi[k])) return ORC_EDOMAIN; /* also rejects NaN */
        }
    return ORC_OK;
}

/* Rows of the targets listed in `rows` (or all rows when rows == NULL). */
static int search_impl(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                       double cell_size, double radius, int brute, const int64_t *rows,
                       int64_t nrows, orc_result **out)
{
    *out = NULL;
    int st = validate(dim, n, pos, lo, hi, cell_size, radius);
    if (st) return st;
    if (!rows) nrows = n;
    for (int64_t r = 0; rows && r < nrows; r++)
        if (rows[r] < 0 || rows[r] >= n) return ORC_EINVAL;

    const double R2 = radius * radius;
    orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
    if (!res) return ORC_ENOMEM;
    res->n = nrows;
    res->row_ptr = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    if (!res->row_ptr) { free(res); return ORC_ENOMEM; }

    /* Background grid (cell link list). The cell width carries a relative slack of
     * 2^-20 so that rounding in the cell index can never push a pair within the
     * radius more than one cell apart. */
    double w = (cell_size > radius ? cell_size : radius) * (1.0 + ldexp(1.0, -20));
    int64_t nc[3] = {1, 1, 1};
    int64_t ncell = 1;
    for (int k = 0; k < dim; k++) {
        double c = ceil((hi[k] - lo[k]) / w);
        nc[k] = c < 1.0 ? 1 : (int64_t)c;
    }
    /* The grid is the oracle's own device: any width >= radius gives the same
     * answer, so widen it when the cell count would be unreasonable. */
    for (;;) {
        ncell = 1;
        for (int k = 0; k < dim; k++) ncell *= nc[k];
        if (ncell <= ((int64_t)1 << 26)) break;
        w *= 2.0;
        for (int k = 0; k < dim; k++) {
            double c = ceil((hi[k] - lo[k]) / w);
            nc[k] = c < 1.0 ? 1 : (int64_t)c;
        }
    }

    int64_t *head = NULL, *next = NULL, *cell = NULL;
    if (!brute) {
        head = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
        next = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
        cell = (int64_t *)malloc((size_t)(n ? n : 1) * 3 * sizeof(int64_t));
        if (!head || !next || !cell) { st = ORC_ENOMEM; goto fail; }
        for (int64_t c = 0; c < ncell; c++) head[c] = -1;
        for (int64_t i = 0; i < n; i++) {
            int64_t key = 0, mul = 1;
            for (int k = 0; k < dim; k++) {
                double t = floor((pos[i * dim + k] - lo[k]) / w);
                int64_t c = (int64_t)t;
                if (c < 0) c = 0;
                if (c > nc[k] - 1) c = nc[k] - 1;
                cell[i * 3 + k] = c;
                key += c * mul;
                mul *= nc[k];
            }
            next[i] = head[key]; /* prepend: the chain is the cell's link list */
            head[key] = i;
        }
    }

    orc_vec all = {0}, row = {0};
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows ? rows[r] : r;
        const double *pi = pos + i * dim;
        row.len = 0;
        if (brute) {
            for (int64_t j = 0; j < n; j++) {
                if (j == i) continue;
                double r2 = pair_r2(dim, pi, pos + j * dim);
                if (r2 <= R2 && (st = vec_push(&row, (int32_t)j, (float)sqrt(r2)))) goto fail2;
            }
        } else {
            int64_t lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
            for (int k = 0; k < dim; k++) {
                lo3[k] = cell[i * 3 + k] > 0 ? cell[i * 3 + k] - 1 : 0;
                hi3[k] = cell[i * 3 + k] < nc[k] - 1 ? cell[i * 3 + k] + 1 : nc[k] - 1;
            }
            for (int64_t cz = lo3[2]; cz <= hi3[2]; cz++)
                for (int64_t cy = lo3[1]; cy <= hi3[1]; cy++)
                    for (int64_t cx = lo3[0]; cx <= hi3[0]; cx++) {
                        int64_t key = cx + nc[0] * (cy + nc[1] * cz);
                        for (int64_t j = head[key]; j >= 0; j = next[j]) {
                            if (j == i) continue;
                            double r2 = pair_r2(dim, pi, pos + j * dim);
                            if (r2 <= R2 && (st = vec_push(&row, (int32_t)j, (float)sqrt(r2))))
                                goto fail2;
                        }
                    }
            qsort(row.v, (size_t)row.len, sizeof(orc_pair), cmp_pair);
        }
        for (int64_t e = 0; e < row.len; e++)
            if ((st = vec_push(&all, row.v[e].j, row.v[e].d))) goto fail2;
        res->row_ptr[r + 1] = all.len;
    }
    res->nnz = all.len;
    res->col = (int32_t *)malloc((size_t)(all.len ? all.len : 1) * sizeof(int32_t));
    res->dist = (float *)malloc((size_t)(all.len ? all.len : 1) * sizeof(float));
    if (!res->col || !res->dist) { st = ORC_ENOMEM; goto fail2; }
    for (int64_t e = 0; e < all.len; e++) {
        res->col[e] = all.v[e].j;
        res->dist[e] = all.v[e].d;
    }
    free(all.v);
    free(row.v);
    free(head);
    free(next);
    free(cell);
    *out = res;
    return ORC_OK;

fail2:
    free(all.v);
    free(row.v);
fail:
    free(head);
    free(next);
    free(cell);
    free(res->row_ptr);
    free(res->col);
    free(res->dist);
    free(res);
    return st;
}

/* Cell link-list search over every row (brute = 0) or the all-list search (brute = 1). */
int orc_search(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
               double cell_size, double radius, int brute, orc_result **out)
{
    return search_impl(dim, n, pos, lo, hi, cell_size, radius, brute, NULL, 0, out);
}

/* The same search restricted to the listed target rows (the CSR then has nrows rows). */
int orc_search_rows(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                    double cell_size, double radius, const int64_t *rows, int64_t nrows,
                    orc_result **out)
{
    if (!rows || nrows < 0) return ORC_EINVAL;
    return search_impl(dim, n, pos, lo, hi, cell_size, radius, 0, rows, nrows, out);
}

int64_t orc_nnz(const orc_result *r) { return r ? r->nnz : -1; }

void orc_copy(const orc_result *r, int64_t *row_ptr, int32_t *col, float *dist)
{
    if (!r) return;
    if (row_ptr) memcpy(row_ptr, r->row_ptr, (size_t)(r->n + 1) * sizeof(int64_t));
    if (col) memcpy(col, r->col, (size_t)r->nnz * sizeof(int32_t));
    if (dist) memcpy(dist, r->dist, (size_t)r->nnz * sizeof(float));
}

void orc_free(orc_result *r)
{
    if (!r) return;
    free(r->row_ptr);
    free(r->col);
    free(r->dist);
    free(r);
}

/* ---------------------------------------------------------------------------------
 * Row-parallel forms of the same search, for large inputs (the whole clustered batch)
 * and for the all-core CPU baseline. They build the same grid (cell link list with
 * head/next chains) and apply the same predicate; each row is computed exactly as in
 * search_impl, by one thread, and rows are independent, so the result does not depend
 * on the thread count. nthreads <= 0 takes OpenMP's default.
 */
typedef struct {
    int dim;
    int64_t n;
    const double *pos;
    double R2;
    int64_t nc[3];
    int64_t *head, *next, *cell;
} orc_grid;

static void grid_free(orc_grid *g)
{
    free(g->head);
    free(g->next);
    free(g->cell);
}

/* The grid of search_impl: cell width max(cell_size, radius)(1 + 2^-20), widened while the
 * cell count exceeds 2^26; chains built by prepending in index order. */
static int grid_build(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                      double cell_size, double radius, orc_grid *g)
{
    memset(g, 0, sizeof(*g));
    int st = validate(dim, n, pos, lo, hi, cell_size, radius);
    if (st) return st;
    g->dim = dim;
    g->n = n;
    g->pos = pos;
    g->R2 = radius * radius;
    double w = (cell_size > radius ? cell_size : radius) * (1.0 + ldexp(1.0, -20));
    int64_t ncell;
    g->nc[0] = g->nc[1] = g->nc[2] = 1;
    for (;;) {
        for (int k = 0; k < dim; k++) {
            double c = ceil((hi[k] - lo[k]) / w);
            g->nc[k] = c < 1.0 ? 1 : (int64_t)c;
        }
        ncell = g->nc[0] * g->nc[1] * g->nc[2];
        if (ncell <= ((int64_t)1 << 26)) break;
        w *= 2.0;
    }
    g->head = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    g->next = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    g->cell = (int64_t *)malloc((size_t)(n ? n : 1) * 3 * sizeof(int64_t));
    if (!g->head || !g->next || !g->cell) {
        grid_free(g);
        return ORC_ENOMEM;
    }
    for (int64_t c = 0; c < ncell; c++) g->head[c] = -1;
    for (int64_t i = 0; i < n; i++) {
        int64_t key = 0, mul = 1;
        for (int k = 0; k < 3; k++) g->cell[i * 3 + k] = 0;
        for (int k = 0; k < dim; k++) {
            double t = floor((pos[i * dim + k] - lo[k]) / w);
            int64_t c = (int64_t)t;
            if (c < 0) c = 0;
            if (c > g->nc[k] - 1) c = g->nc[k] - 1;
            g->cell[i * 3 + k] = c;
            key += c * mul;
            mul *= g->nc[k];
        }
        g->next[i] = g->head[key];
        g->head[key] = i;
    }
    return ORC_OK;
}

/* Neighbours of row i through the clipped 3^d block of cells: their number, and, when
 * out != NULL, the pairs (j, (float)sqrt(r2)) in chain order. */
static int64_t grid_row(const orc_grid *g, int64_t i, orc_pair *out)
{
    const int dim = g->dim;
    const double *pi = g->pos + i * dim;
    int64_t lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
    for (int k = 0; k < dim; k++) {
        lo3[k] = g->cell[i * 3 + k] > 0 ? g->cell[i * 3 + k] - 1 : 0;
        hi3[k] = g->cell[i * 3 + k] < g->nc[k] - 1 ? g->cell[i * 3 + k] + 1 : g->nc[k] - 1;
    }
    int64_t m = 0;
    for (int64_t cz = lo3[2]; cz <= hi3[2]; cz++)
        for (int64_t cy = lo3[1]; cy <= hi3[1]; cy++)
            for (int64_t cx = lo3[0]; cx <= hi3[0]; cx++) {
                int64_t key = cx + g->nc[0] * (cy + g->nc[1] * cz);
                for (int64_t j = g->head[key]; j >= 0; j = g->next[j]) {
                    if (j == i) continue;
                    double r2 = pair_r2(dim, pi, g->pos + j * dim);
                    if (r2 <= g->R2) {
                        if (out) {
                            out[m].j = (int32_t)j;
                            out[m].d = (float)sqrt(r2);
                        }
                        m++;
                    }
                }
            }
    return m;
}

/* counts[r] = |N(rows[r])| (or |N(r)| for every row when rows == NULL, nrows = n). */
int orc_count_rows(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                   double cell_size, double radius, const int64_t *rows, int64_t nrows, int nthreads,
                   int64_t *counts)
{
    if (!counts || (rows && nrows < 0)) return ORC_EINVAL;
    orc_grid g;
    int st = grid_build(dim, n, pos, lo, hi, cell_size, radius, &g);
    if (st) return st;
    if (!rows) nrows = n;
    for (int64_t r = 0; rows && r < nrows; r++)
        if (rows[r] < 0 || rows[r] >= n) {
            grid_free(&g);
            return ORC_EINVAL;
        }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (int64_t r = 0; r < nrows; r++) counts[r] = grid_row(&g, rows ? rows[r] : r, NULL);
    (void)nthreads;
    grid_free(&g);
    return ORC_OK;
}

/* The CSR of search_impl (cell-list form), rows computed in parallel: a counting pass,
 * the row offsets, then each row written at its offset and sorted by j. */
int orc_search_par(int dim, int64_t n, const double *pos, const double *lo, const double *hi,
                   double cell_size, double radius, const int64_t *rows, int64_t nrows, int nthreads,
                   orc_result **out)
{
    *out = NULL;
    if (rows && nrows < 0) return ORC_EINVAL;
    orc_grid g;
    int st = grid_build(dim, n, pos, lo, hi, cell_size, radius, &g);
    if (st) return st;
    if (!rows) nrows = n;
    for (int64_t r = 0; rows && r < nrows; r++)
        if (rows[r] < 0 || rows[r] >= n) {
            grid_free(&g);
            return ORC_EINVAL;
        }
    orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
    int64_t *cnt = (int64_t *)malloc((size_t)(nrows ? nrows : 1) * sizeof(int64_t));
    if (!res || !cnt) {
        free(res);
        free(cnt);
        grid_free(&g);
        return ORC_ENOMEM;
    }
    res->n = nrows;
    res->row_ptr = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    if (!res->row_ptr) {
        st = ORC_ENOMEM;
        goto done;
    }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (int64_t r = 0; r < nrows; r++) cnt[r] = grid_row(&g, rows ? rows[r] : r, NULL);
    for (int64_t r = 0; r < nrows; r++) res->row_ptr[r + 1] = res->row_ptr[r] + cnt[r];
    res->nnz = res->row_ptr[nrows];
    {
        size_t m = (size_t)(res->nnz ? res->nnz : 1);
        orc_pair *pairs = (orc_pair *)malloc(m * sizeof(orc_pair));
        res->col = (int32_t *)malloc(m * sizeof(int32_t));
        res->dist = (float *)malloc(m * sizeof(float));
        if (!pairs || !res->col || !res->dist) {
            free(pairs);
            st = ORC_ENOMEM;
            goto done;
        }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
        for (int64_t r = 0; r < nrows; r++) {
            orc_pair *row = pairs + res->row_ptr[r];
            int64_t len = grid_row(&g, rows ? rows[r] : r, row);
            qsort(row, (size_t)len, sizeof(orc_pair), cmp_pair);
            for (int64_t e = 0; e < len; e++) {
                res->col[res->row_ptr[r] + e] = row[e].j;
                res->dist[res->row_ptr[r] + e] = row[e].d;
            }
        }
        free(pairs);
    }
done:
    free(cnt);
    grid_free(&g);
    if (st) {
        free(res->row_ptr);
        free(res->col);
        free(res->dist);
        free(res);
        return st;
    }
    (void)nthreads;
    *out = res;
    return ORC_OK;
}
