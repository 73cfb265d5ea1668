/*
 * lbl.h -- C ABI of the MI355X labeling library.
 *
 * The library constructs the labeling function of a fixed discrete
 * abstraction from one perception frame (Sec. 4).  Following the reduction of
 * Sec. 4.2 (Eq. bool_dot, Eq. approx), the labels are the Boolean matrix
 * product
 *
 *     L[t][p] = OR_c  T[t][c] AND O[c][p]
 *
 * where T (the paper's M) is the trajectory-by-cell swept-set matrix: row t is
 * the binary vector of the grid cells swept by trajectory t (Sec. 4.1), and O
 * (the paper's P) is the cell-by-proposition matrix of one frame: column p is
 * the binary vector of the cells that proposition p's region intersects.
 * L[t][p] = 1 means proposition p belongs to the label of transition t
 * (Sec. 3, Eq. 3 and Sec. 4, Eq. labeling_op on the grid).
 *
 * T is precomputed once and stays resident in device memory (the abstraction
 * is fixed and reused across planning queries by equivariance, Sec. 1 and
 * Sec. 5); each query sends only O.
 *
 * Conventions shared by every call:
 *   - Every function returns an lbl_status; nothing throws across the ABI.
 *     On a non-OK status, lbl_last_error() returns a message for the calling
 *     thread, output buffers are unspecified, and no handle is leaked.
 *   - Cells are identified on the caller's side by ids in the grid's
 *     cell_order: row-major c = iy * nx + ix by default, or the z-order index
 *     (LBL_MORTON).  The library stores cells in its own device order
 *     internally; the result does not depend on it.
 *   - Input bytes follow C truthiness (nonzero = true).  Output bytes are
 *     exactly 0 or 1.
 *   - All sizes are element counts unless stated otherwise.
 *   - hip_stream arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Device work is stream-ordered: with device pointers a
 *     call returns once its work is enqueued, and the caller's buffers must
 *     stay valid until the stream reaches it.
 */
#ifndef LBL_H
#define LBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBL_OK = 0,
    LBL_EINVAL = 1,    /* invalid argument (null pointer, size, range, mismatch) */
    LBL_ENOMEM = 2,    /* device allocation or memory budget failure */
    LBL_EDEVICE = 3,   /* a HIP runtime error; the message names the call */
    LBL_EBUSY = 4,     /* the server's request queue is full */
    LBL_ETIMEDOUT = 5, /* lbl_serve_wait timed out; the request is still pending */
    LBL_ECLOSED = 6    /* the server is stopping or stopped */
} lbl_status;

typedef struct lbl_abs *lbl_abs_t;       /* owns the device-resident T */
typedef struct lbl_server *lbl_server_t; /* a serving loop */

/* Occupancy grid over the rectangular workspace (Sec. 4.1).  nx and ny are
 * cell counts per axis and must be positive multiples of 8; cell_m is the
 * cell side in metres (informational).
 *
 * cell_order says how the caller numbers the cells, in every array that is
 * indexed by cell (CSR column ids and dense columns of T at load, the rows
 * of O in lbl_label_frame / lbl_label_batch / lbl_serve_submit for an
 * abstraction loaded with this grid, the rows written by lbl_raster_frame,
 * the id given to lbl_cell_position):
 *   LBL_ROW_MAJOR  c = iy * nx + ix (the default);
 *   LBL_MORTON     c = the z-order index of cell (ix, iy) (Sec. 4.1,
 *                  Alg. zcurve, read as bit interleaving with x as the more
 *                  significant bit of each pair: c = sum over bits b of
 *                  bit b of ix * 2^(2b+1) + bit b of iy * 2^(2b)).  Needs a
 *                  square grid whose side is a power of two (nx == ny ==
 *                  2^k, k >= 3), so that the ids are exactly 0 .. nx*ny - 1.
 * Labels do not depend on the order: the same T and O numbered either way
 * give the same L. */
#define LBL_ROW_MAJOR 0u
#define LBL_MORTON 1u

typedef struct {
    uint32_t nx, ny;
    float cell_m;
    uint32_t cell_order; /* LBL_ROW_MAJOR or LBL_MORTON */
} lbl_grid;

/* ---- flags for lbl_load_abstraction* ---------------------------------- */
#define LBL_LOAD_KEEP_INT8 0x1u    /* also keep an int8 copy of T (N_t x N_c bytes) */
#define LBL_LOAD_INPUT_DEVICE 0x2u /* the input arrays are device pointers */
#define LBL_LOAD_NO_SPARSE 0x4u    /* do not build the sparse tiled layout */
#define LBL_LOAD_SPARSE_ONLY 0x8u  /* keep only the sparse tiled layout: the bitpacked T
                                     is built a run of row blocks at a time (about
                                     4 GiB) and dropped, so abstractions larger than
                                     device memory in bitpacked form fit; only
                                     LBL_KERNEL_SPARSE (or AUTO) can label them.
                                     lbl_load_abstraction only; not with
                                     LBL_LOAD_KEEP_INT8 or LBL_LOAD_NO_SPARSE */

/* ---- flags for lbl_label_frame / lbl_label_batch ---------------------- */
#define LBL_HOST_PTRS 0x1u      /* O and L are host pointers; the call is synchronous */
#define LBL_KERNEL_AUTO 0x00u   /* kernel and tile chosen by the autotuner cache */
#define LBL_KERNEL_BITS 0x10u   /* bitpacked AND/OR wavefront kernel (dense bitpacked T) */
#define LBL_KERNEL_SPARSE 0x80u /* sparse tiled T (non-zero words only), nibble
                                   tables per word, or for frames of at most
                                   4 propositions per-word proposition masks
                                   (needs the sparse layout, built by
                                   default) */
#define LBL_KERNEL_MFMA 0x20u   /* int8 MFMA kernel, T expanded from its bitpacked copy */
#define LBL_KERNEL_MFMA_I8 0x40u /* int8 MFMA kernel reading the int8 copy of T
                                   (needs LBL_LOAD_KEEP_INT8) */
#define LBL_KERNEL_MASK 0xF0u

/*
 * Load T given in compressed sparse row form (Sec. 4.3, Eq. csr_demo):
 * row_ptr[t] is the number of true entries in rows 0..t-1 (n_traj + 1
 * values, row_ptr[0] == 0, non-decreasing) and col_idx[row_ptr[t] ..
 * row_ptr[t+1]) are the cell ids (in the grid's cell_order) of row t's true
 * entries.  Column ids may be unsorted or repeated within a row (OR is
 * idempotent).
 *
 * The arrays are host pointers unless LBL_LOAD_INPUT_DEVICE is set.  They are
 * copied; the caller may free them when the call returns.  The returned
 * handle owns the device copy until lbl_free_abstraction.  The call is
 * synchronous and uses the current HIP device.
 *
 * With LBL_LOAD_SPARSE_ONLY the device holds only the sparse tiled layout
 * (non-zero 64-cell words of T, 10 bytes each, and its tilings): a workspace
 * of 2^21 cells and a million rows, 288 GB as bitpacked rows, takes about a
 * gigabyte.  Labels are identical to those of a full load.
 *
 * Errors: LBL_EINVAL for a null pointer, n_traj == 0, nx or ny not a positive
 * multiple of 8, an unknown cell_order or LBL_MORTON on a grid that is not a
 * square of power-of-two side, row_ptr[0] != 0 or decreasing, a column id
 * >= nx * ny, an unknown or contradictory flag, or LBL_LOAD_SPARSE_ONLY with
 * 2^32 rows or more; LBL_ENOMEM if device memory runs out; LBL_EDEVICE on a
 * HIP error.
 */
lbl_status lbl_load_abstraction(const lbl_grid *grid, uint64_t n_traj, const uint64_t *row_ptr,
                                const uint32_t *col_idx, uint32_t flags, lbl_abs_t *out);

/*
 * Load T given dense: n_traj x (nx * ny) bytes, row-major (row t holds its
 * cells in the grid's cell_order; nonzero = cell swept).  Otherwise as
 * lbl_load_abstraction.
 */
lbl_status lbl_load_abstraction_dense(const lbl_grid *grid, uint64_t n_traj, const uint8_t *T,
                                      uint32_t flags, lbl_abs_t *out);

/* Release an abstraction.  The caller must ensure no enqueued work still
 * uses it.  A NULL handle is accepted and ignored. */
lbl_status lbl_free_abstraction(lbl_abs_t a);

/* Sizes of a loaded abstraction. */
typedef struct {
    uint64_t n_traj;
    uint32_t nx, ny;
    uint32_t n_words;        /* 64-cell words per row (nx * ny / 64) */
    uint32_t row_stride;     /* words between consecutive rows of the bitpacked T */
    uint64_t bits_bytes;     /* device bytes of the bitpacked T */
    uint64_t int8_bytes;     /* device bytes of the int8 T (0 if not kept) */
    uint64_t nonzero_words;  /* words of the bitpacked T holding at least one set cell */
    uint64_t set_cells;      /* distinct (trajectory, cell) pairs set in T */
    uint64_t sparse_entries; /* (row, word) entries of the sparse layout (0 if not built) */
    uint64_t sparse_bytes;   /* device bytes of the sparse layout (entries and tilings) */
    uint64_t sparse_frame_bytes; /* bytes one frame's label kernel reads from it:
                                    every entry (16-bit row, 64-bit word), the
                                    one-frame tiling's task and round tables and
                                    the rows of its compact partial slots */
    uint32_t sparse_tiles;   /* workgroups of a one-frame launch */
    uint32_t sparse_row_block; /* rows per row block of the sparse layout */
    uint64_t sparse_frame_bytes_narrow; /* sparse_frame_bytes for frames of at
                                           most 32 propositions (their own
                                           tiling, 32-bit label masks) */
    uint32_t sparse_tiles_narrow;       /* workgroups of such a launch */
    uint32_t sparse_tiles_direct;       /* workgroups of the direct-mask launch
                                           (frames of at most 4 propositions;
                                           0 when that kernel is not built) */
    uint64_t sparse_frame_bytes_direct; /* bytes that launch reads from the
                                           layout: every entry, its chunk, part
                                           and tile records */
} lbl_abs_info;

lbl_status lbl_abstraction_info(lbl_abs_t a, lbl_abs_info *out);

/*
 * Label one frame (Eq. approx).
 *   O : n_cells x n_props bytes, cell-major (O[c * n_props + p]), c numbered
 *       in the cell_order of the grid the abstraction was loaded with;
 *   L : n_traj x n_props bytes, row-major (L[t * n_props + p]), written 0/1.
 *   n_props in [1, 64].
 * With LBL_HOST_PTRS, O and L are host memory and the call returns after L
 * is written (the transfers are part of the call).  Otherwise both are
 * device pointers and the call is asynchronous on hip_stream.  Distinct
 * streams may label the same abstraction concurrently.  Calls on one stream
 * from several host threads at once are not supported: they share that
 * stream's workspace.
 *
 * The first call on a stream (or one needing a larger workspace) allocates
 * and synchronizes that stream; later calls do not.
 *
 * Errors: LBL_EINVAL for a null handle or pointer, n_props outside [1, 64],
 * an unknown kernel flag, LBL_KERNEL_MFMA_I8 without an int8 copy of T, or
 * LBL_KERNEL_BITS / LBL_KERNEL_MFMA on an abstraction loaded with
 * LBL_LOAD_SPARSE_ONLY (no bitpacked T).
 */
lbl_status lbl_label_frame(lbl_abs_t a, const uint8_t *O, uint32_t n_props, uint8_t *L,
                           uint32_t flags, void *hip_stream);

/*
 * lbl_label_frame for callers that cannot allocate device memory: code
 * under HIP graph capture, serving loops or harnesses that forbid
 * hipMalloc.  Same operation and result as lbl_label_frame with device
 * pointers and LBL_KERNEL_AUTO resolved to the sparse kernel (or the
 * bitpacked kernel for an abstraction loaded with LBL_LOAD_NO_SPARSE):
 * O (n_cells x n_props bytes, the abstraction's cell order) and L (n_traj x
 * n_props bytes, written 0/1) are device memory owned by the caller, and the
 * call is asynchronous on hip_stream.
 *
 * The frame's intermediates (nibble tables and tile partials, per-word
 * proposition masks, or packed masks) go to one static device array of
 * 96 MiB that each GPU the library runs on holds until the process ends;
 * the call allocates nothing.  Every call on one GPU uses that GPU's array,
 * so calls that overlap on one GPU (two streams, or two host threads) race:
 * serialize them.  A call whose intermediates do not fit fails with
 * LBL_EINVAL and names the size it needs; lbl_label_frame serves such
 * frames.  The need depends on the frame: 2 KiB per 64-cell word of nibble
 * tables for more than 32 propositions (grids above about 2^20 cells do not
 * fit), 1 KiB for 5 to 32, and 8, 16 or 32 bytes for at most 4.
 *
 * Errors: LBL_EINVAL for a null handle or pointer, n_props outside [1, 64],
 * the current device not being the abstraction's, or intermediates larger
 * than the array; LBL_EDEVICE for a HIP error.
 */
lbl_status lbl_label_frame_noalloc(lbl_abs_t a, const uint8_t *O, uint32_t n_props, uint8_t *L,
                                   void *hip_stream);

/*
 * Label many frames, possibly against different abstractions, in one
 * persistent-kernel launch.  Each job is one frame as in lbl_label_frame
 * (device pointers; flags must be 0).  Jobs on the same abstraction share
 * each pass over T: their propositions are concatenated, up to
 * LBL_BATCH_MAX_PROPS per pass (more propositions on one abstraction take
 * further passes in the same launch).  Workgroups pull (abstraction, row
 * range) items from a queue, largest first.
 *
 * The whole pipeline of a batch (O packing, labeling, label bytes) is
 * recorded once as a HIP graph keyed by (hip_stream, jobs, launch choice)
 * and replayed when the same batch is submitted again on that stream; the
 * graph owns its tables and packed masks (up to 8 graphs are cached; the
 * oldest is released after a device synchronization).  Results are
 * identical to labeling each job alone.
 *
 * Jobs on one abstraction are placed into 64-column lane groups first-fit by
 * decreasing proposition count (a job never spans two lane groups).  With
 * the sparse layout on every abstraction, one wavefront per (word, lane
 * group) builds the nibble tables, one workgroup per CU pulls (tile, lane
 * group) items from per-XCD queues (items reading the same tables share an
 * XCD), and one wavefront per 64 rows of a lane group writes each job's
 * label bytes as one contiguous block.
 *
 * Errors: as lbl_label_frame for every job, plus LBL_EINVAL for n_jobs == 0,
 * nonzero flags, or a batch mixing an abstraction without the sparse layout
 * (LBL_LOAD_NO_SPARSE) and one without the bitpacked T
 * (LBL_LOAD_SPARSE_ONLY): such a batch has no common kernel.
 */
typedef struct {
    lbl_abs_t a;
    const uint8_t *O;
    uint32_t n_props;
    uint8_t *L;
} lbl_job;

#define LBL_BATCH_MAX_PROPS 1024u

lbl_status lbl_label_batch(const lbl_job *jobs, size_t n_jobs, uint32_t flags, void *hip_stream);

/*
 * Proposition regions of one frame, rasterized on the device into O
 * (Sec. 4.1: the binary vector of a region has a 1 at every cell the region
 * intersects; "intersects" read as an overlap of positive area with the
 * closed cell square, so touching a cell's boundary does not mark it).
 *
 * A region is a union of shapes in workspace coordinates (metres, the grid's
 * origin at (0, 0)); shape i belongs to proposition prop:
 *   LBL_SHAPE_RECT  axis-aligned rectangle, centre (cx, cy), half sizes (a, b);
 *   LBL_SHAPE_DISC  disc, centre (cx, cy), radius a (b unused).
 * Cell (ix, iy) is the square [ix * cell_m, ix * cell_m + cell_m] x
 * [iy * cell_m, iy * cell_m + cell_m], computed in double precision, and O is
 * written as lbl_label_frame reads it: n_cells x n_props bytes, cells
 * numbered in the grid's cell_order, exactly 0 or 1.  cell_m is given here in double
 * precision (the grid's float cell_m is informational).
 *
 * shapes: host array of n_shapes entries, read during the call (the caller
 * may reuse it on return); O: device buffer, written stream-ordered on
 * hip_stream (every byte, including those of propositions without shapes).
 *
 * Errors: LBL_EINVAL for a null grid, O, or shapes with n_shapes > 0;
 * n_props outside [1, 64]; cell_m not finite and positive; a kind other than
 * the two above; prop >= n_props; a coordinate or size not finite, or a
 * negative size.  LBL_EDEVICE for a HIP error.
 */
#define LBL_SHAPE_RECT 0u
#define LBL_SHAPE_DISC 1u

typedef struct {
    uint32_t kind; /* LBL_SHAPE_RECT or LBL_SHAPE_DISC */
    uint32_t prop; /* proposition index, < n_props */
    double cx, cy; /* centre, metres */
    double a, b;   /* half sizes (rectangle) or radius a (disc) */
} lbl_shape;

lbl_status lbl_raster_frame(const lbl_grid *grid, double cell_m, const lbl_shape *shapes, uint64_t n_shapes,
                            uint32_t n_props, uint8_t *O, void *hip_stream);

/*
 * Autotuner.  lbl_tune times the candidate kernels and tile shapes for the
 * abstraction's shape class (row count, word count, proposition count, T word
 * density) on one frame and records the fastest; LBL_KERNEL_AUTO then uses
 * it.  O_sample is a device frame (n_cells x n_props, as in lbl_label_frame)
 * or NULL, in which case every cell of every proposition is set independently
 * with probability density_pct / 100 (the Bernoulli subset model of Sec. 5.1,
 * which favours early termination; pass a real frame when one is available).
 * The call synchronizes hip_stream.  lbl_tune_save / lbl_tune_load persist the
 * cache as JSON text.
 */
lbl_status lbl_tune(lbl_abs_t a, const uint8_t *O_sample, uint32_t n_props, uint32_t density_pct,
                    void *hip_stream);
/* Time the batch's launch choices on this batch and record the fastest for
 * its shape class (whether every abstraction has the sparse layout, and the
 * multiset of (words per row, lane groups) of its passes); later
 * lbl_label_batch calls of that class use it, and the graph cached for
 * these jobs is rebuilt if it was made for another choice.  Sparse batches:
 * the tiling of the layout (the one-frame tiling, or 1, 2, 4, 8 tiles per row
 * block) and the launch (persistent workgroups pulling tiles from per-XCD
 * queues, or one workgroup per tile).  Bitpacked batches: rows per work
 * item, wavefronts per workgroup, loads in flight.  Runs the batch several
 * times (the jobs' L buffers are overwritten); synchronizes hip_stream. */
lbl_status lbl_tune_batch(const lbl_job *jobs, size_t n_jobs, void *hip_stream);
/* Describe into buf (NUL-terminated) the shape class of a batch and the
 * launch choice lbl_label_batch would use for it on hip_stream, followed by
 * "cached" if a graph for these jobs with that choice exists, else "not
 * built".  Host only; launches nothing. */
lbl_status lbl_tune_batch_describe(const lbl_job *jobs, size_t n_jobs, void *hip_stream, char *buf, size_t buf_len);
lbl_status lbl_tune_save(const char *path);
lbl_status lbl_tune_load(const char *path);
/* Describe the choice AUTO makes for (a, n_props) into buf (NUL-terminated). */
lbl_status lbl_tune_describe(lbl_abs_t a, uint32_t n_props, char *buf, size_t buf_len);

/*
 * Serving loop (continuous batching).  lbl_serve_start creates a server with
 * its own streams and a worker thread.  lbl_serve_submit enqueues one frame
 * (device pointers, as in lbl_label_frame) and returns a ticket; requests are
 * admitted onto the GPU as memory within hbm_budget_bytes (for the server's
 * internal per-request buffers) frees up, grouped per abstraction into
 * batches of at most max_batch_frames, and a batch is launched while earlier
 * ones are still running (a batch of one frame on an abstraction with the
 * sparse layout runs the kernels lbl_label_frame's sparse path runs; the
 * labels are the same either way).  The library does not copy O or L: both must stay
 * valid until lbl_serve_wait returns LBL_OK for the ticket.  The server's
 * streams are not ordered after the caller's: O (and any earlier write to L)
 * must be complete on the device when lbl_serve_submit is called, e.g. by
 * synchronizing the stream that produced them.
 *
 * lbl_serve_wait blocks until the ticket completes (LBL_OK), timeout_us
 * elapses (LBL_ETIMEDOUT; negative = wait forever), or the request failed
 * (its error status).  Each ticket can be waited for successfully once.
 * Latency is measured from submit to completion on the host's monotonic
 * clock.  submit, wait and stats may be called from any thread.
 */
typedef struct {
    uint64_t hbm_budget_bytes; /* bytes for in-flight requests' internal buffers */
    uint32_t max_batch_frames; /* frames per launched batch, >= 1 */
    uint32_t max_wait_us;      /* how long a non-full batch may wait for company */
    uint32_t max_queue;        /* pending requests before submit returns LBL_EBUSY */
    uint32_t n_streams;        /* batches that may be in flight at once, 1..8 */
} lbl_serve_cfg;

typedef struct {
    uint64_t submitted, completed, rejected, failed;
    uint64_t batches;
    uint64_t pairs;          /* labeled (trajectory, proposition) pairs */
    double p50_ms, p99_ms, mean_ms, max_ms;
    double wall_s;           /* time since start */
    double pairs_per_s;
    uint64_t max_in_flight;  /* most requests on the GPU at once */
    uint64_t budget_high_water;
} lbl_serve_stats;

lbl_status lbl_serve_start(const lbl_serve_cfg *cfg, lbl_server_t *out);
lbl_status lbl_serve_submit(lbl_server_t s, lbl_abs_t a, const uint8_t *O, uint32_t n_props,
                            uint8_t *L, uint64_t *ticket);
lbl_status lbl_serve_wait(lbl_server_t s, uint64_t ticket, int64_t timeout_us);
lbl_status lbl_serve_stats_get(lbl_server_t s, lbl_serve_stats *out);
lbl_status lbl_serve_stop(lbl_server_t s);

/*
 * Kernel timing for measurement.  While enabled, lbl_label_frame and
 * lbl_label_batch record HIP events on their stream around each kernel they
 * launch.  lbl_profile_read waits for the recorded events and returns totals
 * since the last lbl_profile_enable.  Disabled by default; enabling or
 * disabling resets the totals.  Not for use under graph capture.
 */
typedef struct {
    uint64_t pack_launches;   /* O packing kernels timed (lbl_label_frame) */
    uint64_t label_launches;  /* labeling kernels timed (lbl_label_frame) */
    uint64_t batch_launches;  /* whole batches timed (lbl_label_batch) */
    uint64_t emit_launches;   /* label-bit to byte kernels timed (sparse kernel only) */
    double pack_ms;           /* summed durations */
    double label_ms;
    double batch_ms;
    double emit_ms;
} lbl_profile;

lbl_status lbl_profile_enable(int on);
lbl_status lbl_profile_read(lbl_profile *out);

/*
 * Device cell order.  Cells are grouped into 8 x 8 tiles, one 64-bit word per
 * tile; words follow the z-order of the tiles (Sec. 4.1, Alg. zcurve; ranked
 * among the grid's tiles when the tile grid is not a power-of-two square) and
 * bits follow the z-order of the cells inside the tile, x as the more
 * significant bit of each pair.  For a 2^k x 2^k grid, word * 64 + bit is the
 * cell's z-order index (so with LBL_MORTON ids, word = cell / 64 and bit =
 * cell % 64).  cell is numbered in the grid's cell_order.  Host-only; needs
 * no device.
 */
lbl_status lbl_cell_position(const lbl_grid *grid, uint32_t cell, uint32_t *word, uint32_t *bit);

/*
 * Minimum-cost paths on the product graph of the transition system and a
 * runtime monitor (Sec. 3.2): product vertices are pairs (v, q) of a vertex
 * and a monitor state; a transition e from u to v of cost C(e) joins (u, q)
 * to (v, q') when the monitor moves from q to q' on the label L(e), and its
 * product edge costs C(e).  A monitor with no move for a label has met a bad
 * prefix of the specification (the finite automaton of Sec. 3.2 whose
 * rejected words are the bad prefixes), so that product edge is absent and
 * every path found satisfies the specification so far.
 *
 *   n_vertices, n_edges  sizes of the transition system; n_vertices > 0,
 *                        n_vertices * n_states and n_edges * n_states below
 *                        2^32 - 1.
 *   src, dst, cost       device arrays of n_edges uint32: the transition's
 *                        end vertices (< n_vertices) and its cost (>= 1;
 *                        integer costs make sums exact).
 *   L, l_stride, n_props device array of n_edges rows of l_stride bytes,
 *                        row e the label of transition e (as written by
 *                        lbl_label_frame for the rows of T, l_stride = that
 *                        frame's proposition count); the monitor reads the
 *                        first n_props bytes of a row as the bit set sigma =
 *                        OR over p of (L[e][p] != 0) << p, 1 <= n_props <= 8
 *                        and n_props <= l_stride.
 *   n_states, delta      the monitor: 1 <= n_states <= 8 states, and a host
 *                        table of n_states << n_props bytes, delta[(q <<
 *                        n_props) | sigma] = the next state, or
 *                        LBL_MONITOR_REJECT where there is no move.
 *   v0, q0               the start (distance 0).
 *   dist, pred           device outputs of n_vertices * n_states uint32,
 *                        index v * n_states + q: the least cost of a path
 *                        from (v0, q0), and the product edge id e * n_states +
 *                        q_u of the last step of such a path (the smallest
 *                        id among the edges that end a least-cost path);
 *                        0xFFFFFFFF for both when (v, q) is unreachable or
 *                        only reachable at a cost of 2^32 - 1 or more, and
 *                        pred = 0xFFFFFFFF at the start.  Following pred
 *                        from any reached vertex leads back to the start.
 *   n_sweeps             optional: relaxation sweeps up to and including
 *                        the first that changed nothing (at most n_vertices *
 *                        n_states + 1; up to three more run, changing
 *                        nothing, since sweeps go in groups of four between
 *                        reads of their flags).
 *
 * Synchronous: enqueued on hip_stream (0 = the null stream), returns when the
 * outputs are written.  Uses the stream's workspace (8 bytes per product
 * vertex).  Errors: LBL_EINVAL for a null pointer, a size or state out of
 * range, l_stride < n_props, a delta entry that is neither a state nor LBL_MONITOR_REJECT, or an
 * edge whose vertex is out of range or whose cost is 0 (found on the device;
 * dist and pred are then unspecified); LBL_ENOMEM; LBL_EDEVICE.
 */
#define LBL_MONITOR_REJECT 0xFFu
lbl_status lbl_product_shortest_paths(uint64_t n_vertices, uint64_t n_edges, const uint32_t *src, const uint32_t *dst,
                                      const uint32_t *cost, const uint8_t *L, uint32_t l_stride, uint32_t n_props,
                                      uint32_t n_states,
                                      const uint8_t *delta, uint32_t v0, uint32_t q0, uint32_t *dist, uint32_t *pred,
                                      uint32_t *n_sweeps, void *hip_stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *lbl_last_error(void);

/* Library version string. */
const char *lbl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBL_H */
