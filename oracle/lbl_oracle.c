/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, obviously correct CPU implementation of what the labeling
 * path computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Semantics (Sec. 4.2, Eq. bool_dot and Eq. approx): with M the
 * trajectory-by-cell binary matrix and P the cell-by-proposition binary
 * matrix,
 *     L(i, j) = OR_k  M(i, k) AND P(k, j),
 * and pi_j belongs to the label of transition e_i iff L(i, j) is true.
 *
 * Encodings: input bytes follow C truthiness (nonzero = true); output bytes
 * are exactly 0 or 1.  P is stored dense, cell-major: O[c * n_props + p]
 * (Sec. 4.3 keeps P as a dense two-dimensional array).  M is stored in
 * compressed sparse row form (Sec. 4.3, Eq. csr_demo) with the arrays named
 * by their role in the worked example: row_ptr (the paper's r, running count
 * of true entries before each row) and col_idx (the paper's c, column index
 * of each true entry, left to right, top to bottom).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

/*
 * Sparse Boolean matrix product (Sec. 4.3, Alg. mat_mul), read with the
 * indices of Eq. approx: for each listed row t, for each stored entry k of
 * that row, OR the proposition values of cell col_idx[k] into L[t][*].  The
 * loop over propositions is innermost; OR is commutative and idempotent, so
 * the order of the loops does not change the result.  No early exit.
 *
 * rows lists which rows of M to label (n_rows of them); L receives
 * n_rows x n_props bytes, row i of L for row rows[i] of M.
 * Returns 0, or -1 if a column index is out of range (L is then unspecified).
 */
typedef struct {
    const uint64_t *row_ptr;
    const uint32_t *col_idx;
    uint64_t n_cells;
    const uint8_t *O;
    uint32_t n_props;
    const uint64_t *rows;
    uint64_t lo, hi;
    uint8_t *L;
    int bad;
} csr_job;

static void label_rows_csr(csr_job *j)
{
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        uint64_t t = j->rows[i];
        uint8_t *Lt = j->L + i * j->n_props;
        for (uint32_t p = 0; p < j->n_props; ++p) Lt[p] = 0;
        for (uint64_t k = j->row_ptr[t]; k < j->row_ptr[t + 1]; ++k) {
            uint64_t c = j->col_idx[k];
            if (c >= j->n_cells) {
                j->bad = 1;
                return;
            }
            const uint8_t *Oc = j->O + c * j->n_props;
            for (uint32_t p = 0; p < j->n_props; ++p) Lt[p] = (uint8_t)(Lt[p] | (Oc[p] != 0));
        }
    }
}

static void *csr_thread(void *v)
{
    label_rows_csr((csr_job *)v);
    return NULL;
}

int oracle_label_csr(const uint64_t *row_ptr, const uint32_t *col_idx, uint64_t n_cells,
                     const uint8_t *O, uint32_t n_props, const uint64_t *rows, uint64_t n_rows,
                     uint8_t *L, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n_rows) n_threads = n_rows ? (int)n_rows : 1;
    csr_job *jobs = (csr_job *)calloc((size_t)n_threads, sizeof(csr_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    /* static split of the row list; every thread writes disjoint rows of L */
    for (int i = 0; i < n_threads; ++i) {
        csr_job j = {row_ptr, col_idx, n_cells, O, n_props, rows,
                     n_rows * (uint64_t)i / (uint64_t)n_threads,
                     n_rows * (uint64_t)(i + 1) / (uint64_t)n_threads, L, 0};
        jobs[i] = j;
    }
    for (int i = 1; i < n_threads; ++i) pthread_create(&th[i], NULL, csr_thread, &jobs[i]);
    label_rows_csr(&jobs[0]);
    for (int i = 1; i < n_threads; ++i) pthread_join(th[i], NULL);
    int bad = 0;
    for (int i = 0; i < n_threads; ++i) bad |= jobs[i].bad;
    free(jobs);
    free(th);
    return bad ? -1 : 0;
}

/*
 * Eq. bool_dot written out for a dense M (n_traj x n_cells bytes, row-major):
 * L[t][p] = OR over every cell c of (M[t][c] AND P[c][p]).  A triple loop,
 * for small inputs.
 */
void oracle_label_dense(const uint8_t *M, uint64_t n_traj, uint64_t n_cells, const uint8_t *O,
                        uint32_t n_props, uint8_t *L)
{
    for (uint64_t t = 0; t < n_traj; ++t)
        for (uint32_t p = 0; p < n_props; ++p) {
            int acc = 0;
            for (uint64_t c = 0; c < n_cells; ++c)
                acc = acc || (M[t * n_cells + c] != 0 && O[c * n_props + p] != 0);
            L[t * n_props + p] = (uint8_t)acc;
        }
}

/*
 * z-order index of a point by descending a binary space partition
 * (Sec. 4.1, Alg. zcurve), as read here:
 *   - normalise each coordinate to [0, 1] over the workspace box;
 *   - visit axes cyclically, axis 0 first, for d levels;
 *   - at level i (1-based) the pivot of the current axis splits its current
 *     interval; a point at or above the pivot is on the high side and adds
 *     2^(d - i) to the index, and the pivot moves half the interval's half
 *     width towards the point: by 0.5^(floor((i - 1) / k) + 2).
 * Cells are half-open, so a point on a splitting plane goes to the high side.
 * With d = k * b this equals interleaving the b-bit cell coordinates with
 * axis 0 as the most significant bit of every k-bit group (the equivalence
 * the section states).
 */
uint64_t oracle_zorder(int k, int d, const double *x, const double *lo, const double *hi)
{
    double z[16], piv[16];
    for (int a = 0; a < k; ++a) {
        z[a] = (x[a] - lo[a]) / (hi[a] - lo[a]);
        piv[a] = 0.5;
    }
    uint64_t n = 0;
    int j = 0;
    for (int i = 1; i <= d; ++i) {
        double step = pow(0.5, (double)((i - 1) / k + 2));
        if (z[j] >= piv[j]) {
            n += (uint64_t)1 << (d - i);
            piv[j] += step;
        } else {
            piv[j] -= step;
        }
        j = (j + 1) % k;
    }
    return n;
}

/*
 * Binary-vector encoding of proposition regions (Sec. 4.1): entry i of a
 * proposition's vector is 1 iff its region intersects cell i of the
 * partition.  "Intersects" is read as an overlap of positive area with the
 * closed cell square, so a region that only touches a cell's boundary does
 * not mark it.  A region is a union of shapes; shape s belongs to
 * proposition prop[s] and is
 *   kind 0: the axis-aligned rectangle with centre (cx, cy) and half sizes
 *           (a, b), or
 *   kind 1: the disc with centre (cx, cy) and radius a.
 * Cells form an nx x ny grid of side cell, cell (ix, iy) the square
 * [x0, x0 + cell] x [y0, y0 + cell] with x0 = ix * cell, y0 = iy * cell,
 * stored row-major (c = iy * nx + ix).  O[c * n_props + p] is set to 1 iff
 * some shape of proposition p meets cell c, else 0.
 *
 * Every cell is tested against every shape (no bounding boxes):
 *   rectangle: the two intervals on each axis overlap with positive length,
 *              min of the upper ends minus max of the lower ends > 0;
 *   disc:      the square's point nearest the centre lies at a distance
 *              below the radius (squared distance < a * a).
 * Returns 0, or -1 for a kind other than 0 or 1 or a prop >= n_props.
 */
int oracle_raster_shapes(const uint32_t *kind, const uint32_t *prop, const double *cx, const double *cy,
                         const double *a, const double *b, uint64_t n_shapes, uint32_t nx, uint32_t ny,
                         double cell, uint32_t n_props, uint8_t *O)
{
    for (uint64_t s = 0; s < n_shapes; ++s)
        if (kind[s] > 1 || prop[s] >= n_props) return -1;
    for (uint32_t iy = 0; iy < ny; ++iy) {
        const double y0 = (double)iy * cell, y1 = y0 + cell;
        for (uint32_t ix = 0; ix < nx; ++ix) {
            const double x0 = (double)ix * cell, x1 = x0 + cell;
            uint8_t *o = O + ((uint64_t)iy * nx + ix) * n_props;
            for (uint32_t p = 0; p < n_props; ++p) o[p] = 0;
            for (uint64_t s = 0; s < n_shapes; ++s) {
                int hit;
                if (kind[s] == 0) {
                    const double ox = fmin(x1, cx[s] + a[s]) - fmax(x0, cx[s] - a[s]);
                    const double oy = fmin(y1, cy[s] + b[s]) - fmax(y0, cy[s] - b[s]);
                    hit = ox > 0.0 && oy > 0.0;
                } else {
                    const double qx = fmin(fmax(cx[s], x0), x1), qy = fmin(fmax(cy[s], y0), y1);
                    const double ex = cx[s] - qx, ey = cy[s] - qy;
                    hit = ex * ex + ey * ey < a[s] * a[s];
                }
                if (hit) o[prop[s]] = 1;
            }
        }
    }
    return 0;
}

/*
 * Early termination (Sec. 5.1, Eq. prob_term): the serial scan behind Eq.
 * bool_dot examines the cells of row t in ascending id order and may stop at
 * the first cell that both the trajectory and proposition prop occupy, since
 * the remaining cells cannot change L[t][prop].  out[i] is the number of cells
 * that scan compares for row rows[i]: the first shared cell's id plus one, or
 * n_cells when the row shares no cell with the proposition (L[t][prop] = 0).
 * Column ids must be ascending within each row.  Returns 0, -1 for a column
 * id out of range, -2 for ids not ascending.
 */
int oracle_scan_lengths(const uint64_t *row_ptr, const uint32_t *col_idx, uint64_t n_cells, const uint8_t *O,
                        uint32_t n_props, uint32_t prop, const uint64_t *rows, uint64_t n_rows, uint64_t *out)
{
    for (uint64_t i = 0; i < n_rows; ++i) {
        uint64_t t = rows[i];
        out[i] = n_cells;
        for (uint64_t k = row_ptr[t]; k < row_ptr[t + 1]; ++k) {
            if (col_idx[k] >= n_cells) return -1;
            if (k > row_ptr[t] && col_idx[k] <= col_idx[k - 1]) return -2;
        }
        for (uint64_t k = row_ptr[t]; k < row_ptr[t + 1]; ++k) {
            uint64_t c = col_idx[k];
            if (O[c * n_props + prop] != 0) {
                out[i] = c + 1;
                break;
            }
        }
    }
    return 0;
}

/*
 * Planning on the product graph (Sec. 3.2): vertices (v, q) of the
 * transition system and the monitor; transition e from u to v joins (u, q)
 * to (v, delta[q][sigma_e]) at cost cost[e], where sigma_e is e's label as a
 * bit set of its n_props propositions and a delta entry >= n_states means the
 * monitor has no move (a bad prefix: no product edge).  A minimum-cost path
 * from (v0, q0) is a shortest path in this graph.
 *
 * dist[v * Q + q]: the least path cost (Dijkstra with a binary heap; costs
 * at least 1; a path cost of 2^32 - 1 or more counts as unreachable, value
 * 0xFFFFFFFF).  pred[v * Q + q]: the smallest product edge id e * Q + q_u over
 * the product edges into (v, q) with dist[u, q_u] + cost[e] == dist[v, q],
 * 0xFFFFFFFF at the start and where unreachable.  Returns 0, -1 for a vertex
 * out of range or a zero cost, -2 if memory runs out.
 */
typedef struct { uint64_t d; uint64_t x; } heap_item;

static void heap_push(heap_item *h, uint64_t *n, heap_item it)
{
    uint64_t i = (*n)++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h[p].d < it.d || (h[p].d == it.d && h[p].x <= it.x)) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = it;
}

static heap_item heap_pop(heap_item *h, uint64_t *n)
{
    heap_item top = h[0], last = h[--(*n)];
    uint64_t i = 0;
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= *n) break;
        if (c + 1 < *n && (h[c + 1].d < h[c].d || (h[c + 1].d == h[c].d && h[c + 1].x < h[c].x))) ++c;
        if (last.d < h[c].d || (last.d == h[c].d && last.x <= h[c].x)) break;
        h[i] = h[c];
        i = c;
    }
    h[i] = last;
    return top;
}

int oracle_product_paths(uint64_t n_vertices, uint64_t n_edges, const uint32_t *src, const uint32_t *dst,
                         const uint32_t *cost, const uint8_t *L, uint32_t n_props, uint32_t n_states,
                         const uint8_t *delta, uint32_t v0, uint32_t q0, uint32_t *dist, uint32_t *pred)
{
    const uint64_t Q = n_states, n = n_vertices * Q, none = 0xFFFFFFFFull;
    for (uint64_t e = 0; e < n_edges; ++e)
        if (src[e] >= n_vertices || dst[e] >= n_vertices || cost[e] == 0) return -1;
    /* outgoing transitions of each vertex (counting sort by source) */
    uint64_t *first = (uint64_t *)calloc(n_vertices + 1, sizeof(uint64_t));
    uint64_t *order = (uint64_t *)malloc((n_edges ? n_edges : 1) * sizeof(uint64_t));
    uint32_t *sigma = (uint32_t *)malloc((n_edges ? n_edges : 1) * sizeof(uint32_t));
    uint64_t *d = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc(n, 1);
    heap_item *heap = (heap_item *)malloc((n_edges * Q + 1) * sizeof(heap_item));
    if (!first || !order || !sigma || !d || !done || !heap) {
        free(first); free(order); free(sigma); free(d); free(done); free(heap);
        return -2;
    }
    for (uint64_t e = 0; e < n_edges; ++e) {
        first[src[e] + 1]++;
        uint32_t s = 0;
        for (uint32_t p = 0; p < n_props; ++p) s |= (uint32_t)(L[e * n_props + p] != 0) << p;
        sigma[e] = s;
    }
    for (uint64_t v = 0; v < n_vertices; ++v) first[v + 1] += first[v];
    {
        uint64_t *fill = (uint64_t *)malloc((n_vertices + 1) * sizeof(uint64_t));
        if (!fill) { free(first); free(order); free(sigma); free(d); free(done); free(heap); return -2; }
        for (uint64_t v = 0; v <= n_vertices; ++v) fill[v] = first[v];
        for (uint64_t e = 0; e < n_edges; ++e) order[fill[src[e]]++] = e;
        free(fill);
    }
    for (uint64_t i = 0; i < n; ++i) d[i] = none;
    const uint64_t start = (uint64_t)v0 * Q + q0;
    d[start] = 0;
    uint64_t hn = 0;
    heap_item it0 = {0, start};
    heap_push(heap, &hn, it0);
    while (hn > 0) {
        heap_item it = heap_pop(heap, &hn);
        if (done[it.x] || it.d != d[it.x]) continue;
        done[it.x] = 1;
        const uint64_t u = it.x / Q, q = it.x % Q;
        for (uint64_t k = first[u]; k < first[u + 1]; ++k) {
            const uint64_t e = order[k];
            const uint32_t q2 = delta[(q << n_props) | sigma[e]];
            if (q2 >= n_states) continue;
            const uint64_t nd = it.d + cost[e];
            const uint64_t to = (uint64_t)dst[e] * Q + q2;
            if (nd >= none || nd >= d[to]) continue;
            d[to] = nd;
            heap_item nx = {nd, to};
            heap_push(heap, &hn, nx);
        }
    }
    /* canonical predecessors: the smallest tight product edge id */
    for (uint64_t i = 0; i < n; ++i) {
        dist[i] = (uint32_t)d[i];
        pred[i] = 0xFFFFFFFFu;
    }
    for (uint64_t e = 0; e < n_edges; ++e)
        for (uint64_t q = 0; q < Q; ++q) {
            const uint64_t from = (uint64_t)src[e] * Q + q;
            const uint32_t q2 = delta[(q << n_props) | sigma[e]];
            if (d[from] == none || q2 >= n_states) continue;
            const uint64_t to = (uint64_t)dst[e] * Q + q2;
            if (to == start || d[from] + cost[e] != d[to]) continue;
            const uint64_t id = e * Q + q;
            if (id < pred[to]) pred[to] = (uint32_t)id;
        }
    free(first); free(order); free(sigma); free(d); free(done); free(heap);
    return 0;
}
