/*
 * Synthetic input geometry: swept car footprints along arcs and clothoids,
 * rasterized conservatively onto a row-major occupancy grid.
 *
 * This file produces INPUTS only (the trajectory-by-cell matrix in CSR form).
 * It contains none of the labeling arithmetic: no product of a trajectory
 * matrix with a proposition map happens here.
 *
 * Geometry conventions (generator choices, documented with the workload
 * recipe):
 *   - grid of n x n square cells of side res, extent [0, n*res)^2,
 *     cell id = iy * n + ix (row-major);
 *   - a cell belongs to a swept set iff the footprint at some sampled pose
 *     overlaps the closed cell square with positive area (the conservative
 *     encoding of Sec. 4.1: a cell is set when the subset intersects it);
 *   - poses are sampled at arc length s = i*ds, plus the endpoint s = len;
 *   - footprint: rectangle of length fl (along the heading) and width fw,
 *     centred on the pose;
 *   - parts outside the grid are clipped away.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    /* per trajectory parameters, arrays of length n_traj */
    const double *x0, *y0, *th0, *k0, *k1, *len;
    const uint8_t *kind; /* 0 = arc (curvature k0), 1 = clothoid k0 -> k1 */
    uint64_t n_traj;
    uint32_t n;          /* grid side in cells */
    double res, ds, fl, fw;
} gen_params;

typedef struct {
    uint32_t *cells;     /* concatenated cell ids of this chunk's rows */
    uint64_t n_cells, cap;
    uint64_t row_lo, row_hi;
    uint64_t *counts;    /* points into the caller's counts array */
    int failed;
} chunk_out;

typedef struct {
    const void *p;       /* the generator's parameters */
    chunk_out *out;
} worker_arg;

typedef struct {
    chunk_out *chunks;
    int n_chunks;
    uint64_t total;
} gen_handle;

/* sin(u)/u, accurate near zero */
static double sinc(double u)
{
    if (fabs(u) < 1e-4) {
        double u2 = u * u;
        return 1.0 - u2 / 6.0 + u2 * u2 / 120.0;
    }
    return sin(u) / u;
}

/* Mark the cells of one footprint rectangle in a row-major bitmap. */
static void raster_rect(uint64_t *bm, uint32_t words_per_row, uint32_t n, double res,
                        const double cx[4], const double cy[4],
                        uint32_t *bb_lo, uint32_t *bb_hi)
{
    double ymin = cy[0], ymax = cy[0];
    for (int i = 1; i < 4; ++i) {
        if (cy[i] < ymin) ymin = cy[i];
        if (cy[i] > ymax) ymax = cy[i];
    }
    long iy_lo = (long)floor(ymin / res);
    long iy_hi = (long)ceil(ymax / res) - 1;
    if (iy_lo < 0) iy_lo = 0;
    if (iy_hi > (long)n - 1) iy_hi = (long)n - 1;
    for (long iy = iy_lo; iy <= iy_hi; ++iy) {
        double y0 = (double)iy * res, y1 = (double)(iy + 1) * res;
        double lo = y0 > ymin ? y0 : ymin, hi = y1 < ymax ? y1 : ymax;
        if (!(lo < hi)) continue; /* the strip meets the rectangle in measure zero */
        double xmin = INFINITY, xmax = -INFINITY;
        for (int i = 0; i < 4; ++i) {
            int j = (i + 1) & 3;
            double ax = cx[i], ay = cy[i], bx = cx[j], by = cy[j];
            if (ay >= y0 && ay <= y1) {
                if (ax < xmin) xmin = ax;
                if (ax > xmax) xmax = ax;
            }
            double ys[2] = {y0, y1};
            for (int q = 0; q < 2; ++q) {
                double yy = ys[q];
                if ((ay - yy) * (by - yy) < 0.0) {
                    double t = (yy - ay) / (by - ay);
                    double xx = ax + t * (bx - ax);
                    if (xx < xmin) xmin = xx;
                    if (xx > xmax) xmax = xx;
                }
            }
        }
        if (!(xmin < xmax)) continue;
        long ix_lo = (long)floor(xmin / res);
        long ix_hi = (long)ceil(xmax / res) - 1;
        if (ix_lo < 0) ix_lo = 0;
        if (ix_hi > (long)n - 1) ix_hi = (long)n - 1;
        if (ix_lo > ix_hi) continue;
        uint64_t *row = bm + (uint64_t)iy * words_per_row;
        for (long ix = ix_lo; ix <= ix_hi;) {
            long w = ix >> 6, b = ix & 63;
            long span = ix_hi - ix + 1;
            if (b == 0 && span >= 64) {
                row[w] = ~0ull;
                ix += 64;
            } else {
                long nb = 64 - b;
                if (nb > span) nb = span;
                uint64_t m = (nb == 64) ? ~0ull : (((1ull << nb) - 1ull) << b);
                row[w] |= m;
                ix += nb;
            }
        }
        if ((uint32_t)iy < bb_lo[1]) bb_lo[1] = (uint32_t)iy;
        if ((uint32_t)iy > bb_hi[1]) bb_hi[1] = (uint32_t)iy;
        if ((uint32_t)ix_lo < bb_lo[0]) bb_lo[0] = (uint32_t)ix_lo;
        if ((uint32_t)ix_hi > bb_hi[0]) bb_hi[0] = (uint32_t)ix_hi;
    }
}

static void footprint(double x, double y, double th, double fl, double fw, double cx[4], double cy[4])
{
    double c = cos(th), s = sin(th), a = 0.5 * fl, b = 0.5 * fw;
    /* corners in order around the rectangle */
    cx[0] = x + a * c - b * s; cy[0] = y + a * s + b * c;
    cx[1] = x - a * c - b * s; cy[1] = y - a * s + b * c;
    cx[2] = x - a * c + b * s; cy[2] = y - a * s - b * c;
    cx[3] = x + a * c + b * s; cy[3] = y + a * s - b * c;
}

/*
 * Poses of trajectory t: arcs in closed form, clothoids by midpoint
 * integration of the heading with step ds/4.  Calls emit(x, y, th) for
 * s = 0, ds, 2 ds, ..., and the endpoint s = len.
 */
typedef void (*pose_fn)(void *ctx, double x, double y, double th);

void gen_poses(const gen_params *p, uint64_t t, pose_fn emit, void *ctx)
{
    double L = p->len[t], ds = p->ds;
    uint64_t n_full = (uint64_t)floor(L / ds);
    int end_extra = (double)n_full * ds < L;
    if (p->kind[t] == 0) {
        double k = p->k0[t];
        for (uint64_t i = 0; i <= n_full + (uint64_t)end_extra; ++i) {
            double s = (i <= n_full) ? (double)i * ds : L;
            double half = 0.5 * k * s;
            double mid = p->th0[t] + half;
            double f = s * sinc(half);
            emit(ctx, p->x0[t] + f * cos(mid), p->y0[t] + f * sin(mid), p->th0[t] + k * s);
        }
    } else {
        double k0 = p->k0[t], dk = (p->k1[t] - p->k0[t]) / (L > 0 ? L : 1.0);
        double x = p->x0[t], y = p->y0[t], s = 0.0;
#define TH(ss) (p->th0[t] + k0 * (ss) + 0.5 * dk * (ss) * (ss))
        emit(ctx, x, y, TH(0.0));
        for (uint64_t i = 1; i <= n_full + (uint64_t)end_extra; ++i) {
            double target = (i <= n_full) ? (double)i * ds : L;
            double span = target - s;
            /* four midpoint steps per pose interval; the final partial
             * interval uses as many steps of at most ds/4 as it needs */
            uint64_t n_sub = (i <= n_full) ? 4 : (uint64_t)ceil(span / (0.25 * ds));
            if (n_sub < 1) n_sub = 1;
            double step = span / (double)n_sub;
            for (uint64_t q = 0; q < n_sub; ++q) {
                double th = TH(s + ((double)q + 0.5) * step);
                x += step * cos(th);
                y += step * sin(th);
            }
            s = target;
            emit(ctx, x, y, TH(target));
        }
#undef TH
    }
}

typedef struct {
    uint64_t *bm;
    uint32_t wpr, n;
    double res, fl, fw;
    uint32_t bb_lo[2], bb_hi[2];
} raster_ctx;

static void raster_emit(void *vctx, double x, double y, double th)
{
    raster_ctx *c = (raster_ctx *)vctx;
    double cx[4], cy[4];
    footprint(x, y, th, c->fl, c->fw, cx, cy);
    raster_rect(c->bm, c->wpr, c->n, c->res, cx, cy, c->bb_lo, c->bb_hi);
}

static int push_cell(chunk_out *o, uint32_t cell)
{
    if (o->n_cells == o->cap) {
        uint64_t nc = o->cap ? o->cap * 2 : (1u << 16);
        uint32_t *q = (uint32_t *)realloc(o->cells, nc * sizeof(uint32_t));
        if (!q) return -1;
        o->cells = q;
        o->cap = nc;
    }
    o->cells[o->n_cells++] = cell;
    return 0;
}

static void *worker(void *va)
{
    worker_arg *a = (worker_arg *)va;
    const gen_params *p = (const gen_params *)a->p;
    chunk_out *o = a->out;
    uint32_t wpr = (p->n + 63) / 64;
    uint64_t *bm = (uint64_t *)calloc((uint64_t)wpr * p->n, sizeof(uint64_t));
    if (!bm) { o->failed = 1; return NULL; }
    raster_ctx c;
    c.bm = bm; c.wpr = wpr; c.n = p->n; c.res = p->res; c.fl = p->fl; c.fw = p->fw;
    for (uint64_t t = o->row_lo; t < o->row_hi; ++t) {
        c.bb_lo[0] = c.bb_lo[1] = UINT32_MAX;
        c.bb_hi[0] = c.bb_hi[1] = 0;
        gen_poses(p, t, raster_emit, &c);
        uint64_t before = o->n_cells;
        if (c.bb_lo[1] != UINT32_MAX) {
            uint32_t w_lo = c.bb_lo[0] >> 6, w_hi = c.bb_hi[0] >> 6;
            for (uint32_t iy = c.bb_lo[1]; iy <= c.bb_hi[1]; ++iy) {
                uint64_t *row = bm + (uint64_t)iy * wpr;
                for (uint32_t w = w_lo; w <= w_hi; ++w) {
                    uint64_t v = row[w];
                    row[w] = 0;
                    while (v) {
                        uint32_t b = (uint32_t)__builtin_ctzll(v);
                        v &= v - 1;
                        if (push_cell(o, iy * p->n + w * 64 + b)) { o->failed = 1; free(bm); return NULL; }
                    }
                }
            }
        }
        o->counts[t - o->row_lo] = o->n_cells - before;
    }
    free(bm);
    return NULL;
}

/*
 * Rasterize every trajectory.  counts[t] receives the number of cells of row
 * t.  Returns an opaque handle holding the cell ids (fetch with
 * gen_raster_fill, release with gen_raster_free), or NULL on failure.
 */
/* Runs fn over n_chunks row ranges on n_threads threads; counts[t] receives
 * the number of cells of row t.  Returns the handle or NULL on failure. */
static gen_handle *run_chunks(void *(*fn)(void *), const void *params, uint64_t n_traj, int n_threads,
                              uint64_t *counts, uint64_t *total)
{
    if (n_threads < 1) n_threads = 1;
    int n_chunks = n_threads * 8;
    if ((uint64_t)n_chunks > n_traj) n_chunks = n_traj ? (int)n_traj : 1;
    gen_handle *h = (gen_handle *)calloc(1, sizeof(gen_handle));
    if (!h) return NULL;
    h->chunks = (chunk_out *)calloc((size_t)n_chunks, sizeof(chunk_out));
    h->n_chunks = n_chunks;
    for (int i = 0; i < n_chunks; ++i) {
        h->chunks[i].row_lo = n_traj * (uint64_t)i / (uint64_t)n_chunks;
        h->chunks[i].row_hi = n_traj * (uint64_t)(i + 1) / (uint64_t)n_chunks;
        h->chunks[i].counts = counts + h->chunks[i].row_lo;
    }
    /* a simple pool: thread k handles chunks k, k + n_threads, ... */
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    worker_arg *args = (worker_arg *)calloc((size_t)n_chunks, sizeof(worker_arg));
    for (int i = 0; i < n_chunks; ++i) { args[i].p = params; args[i].out = &h->chunks[i]; }
    int next = 0;
    while (next < n_chunks) {
        int launched = 0;
        for (int k = 0; k < n_threads && next < n_chunks; ++k, ++next, ++launched)
            pthread_create(&th[k], NULL, fn, &args[next]);
        for (int k = 0; k < launched; ++k) pthread_join(th[k], NULL);
    }
    free(th);
    free(args);
    uint64_t tot = 0;
    int failed = 0;
    for (int i = 0; i < n_chunks; ++i) {
        tot += h->chunks[i].n_cells;
        failed |= h->chunks[i].failed;
    }
    h->total = tot;
    *total = tot;
    if (failed) {
        for (int i = 0; i < n_chunks; ++i) free(h->chunks[i].cells);
        free(h->chunks);
        free(h);
        return NULL;
    }
    return h;
}

/*
 * Rasterize every trajectory.  counts[t] receives the number of cells of row
 * t.  Returns an opaque handle holding the cell ids (fetch with
 * gen_raster_fill, release with gen_raster_free), or NULL on failure.
 */
void *gen_raster(const double *x0, const double *y0, const double *th0, const double *k0,
                 const double *k1, const double *len, const uint8_t *kind, uint64_t n_traj,
                 uint32_t n, double res, double ds, double fl, double fw, int n_threads,
                 uint64_t *counts, uint64_t *total)
{
    gen_params p = {x0, y0, th0, k0, k1, len, kind, n_traj, n, res, ds, fl, fw};
    return run_chunks(worker, &p, n_traj, n_threads, counts, total);
}

/*
 * Space-time swept sets, for the time-augmented workspace (x, y, tau): the
 * grid has n x n cells of side res in the plane and n_tau time layers of dt
 * seconds; cell id = (layer * n + iy) * n + ix.  Transition t drives an arc
 * of curvature k[t] at speed v[t] from (x0, y0, th0); the footprint at the
 * pose of time j * dt occupies layer tau0[t] + j, j = 0 .. dur[t] - 1 (layers
 * at or beyond n_tau are dropped), rasterized as in gen_raster.  Cells come
 * out ascending within a row.
 */
typedef struct {
    const double *x0, *y0, *th0, *k, *v;
    const uint32_t *tau0, *dur;
    uint32_t n, n_tau;
    double res, dt, fl, fw;
} st_params;

static void *st_worker(void *va)
{
    worker_arg *a = (worker_arg *)va;
    const st_params *p = (const st_params *)a->p;
    chunk_out *o = a->out;
    uint32_t wpr = (p->n + 63) / 64;
    uint64_t *bm = (uint64_t *)calloc((uint64_t)wpr * p->n, sizeof(uint64_t));
    if (!bm) { o->failed = 1; return NULL; }
    for (uint64_t t = o->row_lo; t < o->row_hi; ++t) {
        uint64_t before = o->n_cells;
        for (uint32_t j = 0; j < p->dur[t]; ++j) {
            uint64_t layer = (uint64_t)p->tau0[t] + j;
            if (layer >= p->n_tau) break;
            double s = p->v[t] * (double)j * p->dt, half = 0.5 * p->k[t] * s;
            double f = s * sinc(half), mid = p->th0[t] + half;
            double cx[4], cy[4];
            footprint(p->x0[t] + f * cos(mid), p->y0[t] + f * sin(mid), p->th0[t] + p->k[t] * s, p->fl, p->fw,
                      cx, cy);
            uint32_t bb_lo[2] = {UINT32_MAX, UINT32_MAX}, bb_hi[2] = {0, 0};
            raster_rect(bm, wpr, p->n, p->res, cx, cy, bb_lo, bb_hi);
            if (bb_lo[1] == UINT32_MAX) continue;
            uint32_t w_lo = bb_lo[0] >> 6, w_hi = bb_hi[0] >> 6;
            for (uint32_t iy = bb_lo[1]; iy <= bb_hi[1]; ++iy) {
                uint64_t *row = bm + (uint64_t)iy * wpr;
                for (uint32_t w = w_lo; w <= w_hi; ++w) {
                    uint64_t val = row[w];
                    row[w] = 0;
                    while (val) {
                        uint32_t b = (uint32_t)__builtin_ctzll(val);
                        val &= val - 1;
                        uint64_t cell = (layer * p->n + iy) * p->n + w * 64 + b;
                        if (push_cell(o, (uint32_t)cell)) { o->failed = 1; free(bm); return NULL; }
                    }
                }
            }
        }
        o->counts[t - o->row_lo] = o->n_cells - before;
    }
    free(bm);
    return NULL;
}

void *gen_spacetime(const double *x0, const double *y0, const double *th0, const double *k, const double *v,
                    const uint32_t *tau0, const uint32_t *dur, uint64_t n_traj, uint32_t n, uint32_t n_tau,
                    double res, double dt, double fl, double fw, int n_threads, uint64_t *counts, uint64_t *total)
{
    st_params p = {x0, y0, th0, k, v, tau0, dur, n, n_tau, res, dt, fl, fw};
    return run_chunks(st_worker, &p, n_traj, n_threads, counts, total);
}

void gen_raster_fill(void *vh, uint32_t *col_idx)
{
    gen_handle *h = (gen_handle *)vh;
    uint64_t off = 0;
    for (int i = 0; i < h->n_chunks; ++i) {
        if (h->chunks[i].n_cells)
            memcpy(col_idx + off, h->chunks[i].cells, h->chunks[i].n_cells * sizeof(uint32_t));
        off += h->chunks[i].n_cells;
    }
}

void gen_raster_free(void *vh)
{
    gen_handle *h = (gen_handle *)vh;
    if (!h) return;
    for (int i = 0; i < h->n_chunks; ++i) free(h->chunks[i].cells);
    free(h->chunks);
    free(h);
}

/* Poses of one trajectory, for geometric checks in tests: writes up to cap
 * poses (x, y, th interleaved) and returns how many there are. */
typedef struct { double *out; uint64_t cap, n; } pose_buf;

static void pose_collect(void *vctx, double x, double y, double th)
{
    pose_buf *b = (pose_buf *)vctx;
    if (b->n < b->cap) {
        b->out[3 * b->n + 0] = x;
        b->out[3 * b->n + 1] = y;
        b->out[3 * b->n + 2] = th;
    }
    b->n++;
}

uint64_t gen_traj_poses(const double *x0, const double *y0, const double *th0, const double *k0,
                        const double *k1, const double *len, const uint8_t *kind, uint64_t t,
                        double ds, double *out, uint64_t cap)
{
    gen_params p = {x0, y0, th0, k0, k1, len, kind, t + 1, 0, 0.0, ds, 0.0, 0.0};
    pose_buf b = {out, cap, 0};
    gen_poses(&p, t, pose_collect, &b);
    return b.n;
}

/*
 * Proposition regions: each shape is an axis-aligned rectangle (kind 0,
 * centre cx, cy, half sizes a, b) or a disc (kind 1, centre cx, cy, radius a)
 * and belongs to proposition prop[i].  Sets O[c * n_props + prop] = 1 for
 * every cell c the shape overlaps with positive area.  O must be zeroed by the
 * caller; cells are row-major on the n x n grid of side res.
 */
void gen_raster_shapes(const uint8_t *kind, const double *cx, const double *cy, const double *a,
                       const double *b, const uint32_t *prop, uint64_t n_shapes, uint32_t n,
                       double res, uint32_t n_props, uint8_t *O)
{
    for (uint64_t i = 0; i < n_shapes; ++i) {
        double hx = a[i];
        double hy = kind[i] == 0 ? b[i] : a[i];
        long ix_lo = (long)floor((cx[i] - hx) / res), ix_hi = (long)ceil((cx[i] + hx) / res) - 1;
        long iy_lo = (long)floor((cy[i] - hy) / res), iy_hi = (long)ceil((cy[i] + hy) / res) - 1;
        if (ix_lo < 0) ix_lo = 0;
        if (iy_lo < 0) iy_lo = 0;
        if (ix_hi > (long)n - 1) ix_hi = (long)n - 1;
        if (iy_hi > (long)n - 1) iy_hi = (long)n - 1;
        double r2 = a[i] * a[i];
        for (long iy = iy_lo; iy <= iy_hi; ++iy) {
            double y0 = (double)iy * res, y1 = y0 + res;
            for (long ix = ix_lo; ix <= ix_hi; ++ix) {
                double x0 = (double)ix * res, x1 = x0 + res;
                int hit;
                if (kind[i] == 0) {
                    hit = x0 < cx[i] + hx && x1 > cx[i] - hx && y0 < cy[i] + hy && y1 > cy[i] - hy;
                } else {
                    double dx = cx[i] < x0 ? x0 - cx[i] : (cx[i] > x1 ? cx[i] - x1 : 0.0);
                    double dy = cy[i] < y0 ? y0 - cy[i] : (cy[i] > y1 ? cy[i] - y1 : 0.0);
                    hit = dx * dx + dy * dy < r2;
                }
                if (hit) O[((uint64_t)iy * n + (uint64_t)ix) * n_props + prop[i]] = 1;
            }
        }
    }
}
