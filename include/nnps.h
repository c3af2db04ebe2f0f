/*
 * nnps.h — fixed-radius neighbour search for SPH particles on AMD MI355X (gfx950).
 *
 * The operation (SPH method section: Eq. 2 and the text after it, Fig. 3):
 * given n particle positions in a box, a background cell size and a search
 * radius R, return for every particle i the list of particles j != i with
 * |p_j - p_i| <= R, in the exact sense of the binary64 predicate
 *     r2 = ((dx0*dx0) + (dx1*dx1)) + (dx2*dx2) <= R*R,   dx_k = p_j[k] - p_i[k],
 * evaluated left to right with round-to-nearest and no fused multiply-add.
 * Rows are returned as CSR: row_ptr[n+1] (int64), col[nnz] ascending within each
 * row (int32), dist[nnz] (float32, within 1e-6 relative of (float)sqrt(r2)).
 *
 * How it is computed (the relative-coordinate link list, RCLL; Mixed-precision
 * SPH section, Eq. 5-7, Fig. 5): particles are binned into cells of width
 * w = max(cell_size, R)(1 + 2^-30) (cell link list, Fig. 3b), sorted by cell, and
 * stored as FP16 coordinates relative to their cell centre (Eq. 6 scale, [-1, 1]).
 * A pair's squared distance is evaluated in FP16 from the two relative coordinates
 * plus the integer offset of the two cells (Eq. 7, with the factor 1/2 Eq. 7 drops).
 * Pairs whose FP16 r2 lies within a guard band of the cutoff are decided again in
 * FP64 from the caller's positions, so the neighbour set is exactly the binary64
 * one above. FP64 arithmetic on the GPU is used for cell assignment, that recheck, and
 * one subtraction per coordinate for each emitted FP32 distance: of two fixed-point
 * positions (integers below 2^52 held as doubles, so exact) in the block path, of the
 * two FP64 positions in the dense-cell path; the neighbour test itself is FP16.
 *
 * Memory: every pointer named d_* is device memory on the context's device.
 * The caller owns positions and all outputs; the library owns the context and
 * the cell structure (and their device scratch). A cell structure keeps a
 * pointer to the caller's positions (the recheck reads them): they must stay
 * alive and unchanged until the last call on that structure has completed on
 * its stream.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream). Every call is
 * stream-ordered and returns without waiting, except where stated. A cell
 * structure's device arrays are rewritten by every build and read by every pass:
 * calls on one structure made on different streams must be ordered by the caller
 * (an event, or a synchronisation), like any other stream-ordered work on shared
 * memory; a build queued on a non-blocking stream while a pass of the previous
 * search still runs on another stream corrupts that pass. Errors the
 * device detects (positions outside the box, an output buffer too small) are
 * recorded on the device and reported by the next call that synchronises
 * (nnps_count with a host nnz pointer, nnps_stats_get, nnps_search).
 *
 * Errors: every call returns an nnps_status and never aborts or throws.
 */
#ifndef NNPS_H
#define NNPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nnps_status {
    NNPS_OK = 0,
    NNPS_EINVAL = -1,         /* bad argument: see nnps_validate */
    NNPS_EDOMAIN = -2,        /* a position is NaN/Inf or outside [lo, hi] */
    NNPS_ENOMEM = -3,         /* device or host allocation failed */
    NNPS_ECAPACITY = -4,      /* output capacity below nnz; *nnz_out holds the need */
    NNPS_EDEVICE = -5,        /* a HIP runtime call failed */
    NNPS_ETOOMANYCELLS = -6,  /* the grid would exceed 2^30 cells */
    NNPS_EORDER = -7,         /* calls out of order (fill before count, ...) */
    NNPS_EUNSUPPORTED = -8    /* a row longer than the library supports */
} nnps_status;

typedef enum nnps_mode {
    NNPS_MODE_FP16_RCLL = 0,      /* FP16 relative coordinates + FP64 guard-band recheck */
    NNPS_MODE_FP64_BASELINE = 1,  /* FP64 cell list: the binary64 predicate on every candidate,
                                     read from sorted FP64 positions in global memory (one lane
                                     per target), with the same cell build, work blocks, dense
                                     and long-row paths and fill as the FP16 mode; distances
                                     (float)sqrt(r2) in binary64 */
    NNPS_MODE_RECHECK_ALL = 2,    /* debug: FP16 pass plus FP64 on every candidate; the FP64
                                     decision is used and FP16 disagreements outside the band
                                     are counted (must be 0) */
    NNPS_MODE_FP32_RCLL = 3       /* FP32 relative coordinates (Eq. 6-7 in single precision) +
                                     FP64 recheck in a guard band of 2^-15 squared cell widths;
                                     dense cells and long rows are decided in FP64; distances
                                     as in NNPS_MODE_FP64_BASELINE (bit-identical to binary64) */
} nnps_mode;

/* One search problem. Positions are d_pos[i*dim + k] (row-major, float64).
 * Valid when: dim is 2 or 3; 0 <= n < 2^31; lo[k] < hi[k], all finite, for k < dim;
 * 0 < radius <= cell_size, finite; mode is an nnps_mode. Entries lo/hi[k >= dim] are ignored. */
typedef struct nnps_problem {
    int32_t dim;
    int32_t mode;
    int64_t n;
    double lo[3];
    double hi[3];
    double cell_size;
    double radius;
} nnps_problem;

/* Statistics of the last count pass on a cell structure (nnps_stats_get). */
typedef struct nnps_stats {
    int64_t n;
    int64_t nnz;                    /* total neighbour pairs (directed, self excluded) */
    int64_t candidates;             /* pairs tested: j != i in the 3^d cells around i */
    int64_t band_pairs;             /* FP16 r2 inside the guard band -> FP64 recheck */
    int64_t fp16_false_pos;         /* naive FP16 test (r2_16 <= cutoff) says in, FP64 says out */
    int64_t fp16_false_neg;         /* naive FP16 test says out, FP64 says in */
                                    /* (NNPS_MODE_FP32_RCLL: the three above count the FP32
                                       test of the block path; dense cells add none) */
    int64_t outside_band_disagree;  /* RECHECK_ALL only: FP16 decided outside the band but wrong */
    int64_t heavy_rows;             /* rows handled by the long-row path */
    int64_t dense_rows;             /* rows handled by the dense-cell path */
    int64_t dense_entries;          /* summed stencil-union sizes of the dense cells */
    int32_t dim, mode;
    int32_t frac_bits;              /* F: fixed-point fraction bits per cell width */
    int32_t ncell[3];
    double cell_width;              /* w */
    double band;                    /* guard band, in units of w^2 */
} nnps_stats;

/* Work-shape parameters (nnps_ctx_set_tuning; picked per workload by an autotuner).
 * block_target: sets the largest x-span of a work block to block_target / (mean cell
 *   occupancy) cells (at least 1); a block is a run of at most 64 consecutive particles of
 *   one row of cells within that span. Default 80. Valid 8..4096.
 * long_rows_grid: workgroups of the long-row path. Default 1024. Valid 1..2^20.
 * long_rows_keys: row entries the long-row path sorts in LDS at once (longer rows are
 *   sorted in chunks and merged); 0 = as many as the device's LDS allows. Valid 0 or
 *   64..16384, a power of two.
 * dense_min_union: an x-window of cells is searched by the dense-cell path when one of
 *   its cells has more than this many particles in its 3^d stencil (the particles every
 *   target of that cell must test). The dense path stages each such cell's stencil
 *   union, sorted by original index, once per chunk for all of the cell's targets.
 *   0 = default (512 in 3D, 160 in 2D); -1 = never. Valid -1..2^30.
 * dense_grid: workgroups of the dense-cell kernels (persistent). 0 = default (1280).
 *   Valid 0..2^20.
 * dense_max_entries: bound on the summed stencil-union sizes of dense cells per build
 *   (device scratch: 16 bytes per entry, allocated as min(3^d n, bound)). Beyond it a
 *   build falls back to the block and long-row paths. 0 = default (2^28). Valid
 *   0..2^31-1.
 * dense_bits_mib: bound (MiB) on the device scratch in which the FP16 dense count keeps
 *   every target's accepted bits per candidate chunk (16 bits per 128 candidates per
 *   lane: about one bit per candidate) so that the fill does not test again. The
 *   structure sizes it at a build from what the last call that synchronised (a count
 *   with h_nnz, a search) found the dense cells need; while it is too small, or above
 *   the bound, the fill tests the candidates again (same result). 0 = default (16384);
 *   -1 = never. Valid -1..2^20. */
typedef struct nnps_tuning {
    int32_t block_target;
    int32_t long_rows_grid;
    int32_t long_rows_keys;
    int32_t dense_min_union;
    int32_t dense_grid;
    int32_t dense_bits_mib;
    int64_t dense_max_entries;
} nnps_tuning;

typedef struct nnps_ctx nnps_ctx;
typedef struct nnps_cells nnps_cells;

/* Human-readable name of a status. Never NULL. */
const char *nnps_status_str(nnps_status s);

/* Host-only argument check (no device needed): NNPS_OK, NNPS_EINVAL or
 * NNPS_ETOOMANYCELLS. Every call that takes a problem runs it first. */
nnps_status nnps_validate(const nnps_problem *prob);

/* Grid the library would use for `prob`: cell counts (ncell[3], unused axes 1),
 * fixed-point fraction bits and cell width. Host only. */
nnps_status nnps_grid(const nnps_problem *prob, int32_t ncell[3], int32_t *frac_bits,
                      double *cell_width);

/* Context on HIP device `device` (makes it current for the calling thread while
 * in library calls). One context per host thread at a time. */
nnps_status nnps_ctx_create(int device, nnps_ctx **out);
void nnps_ctx_destroy(nnps_ctx *ctx);

/* Waits for `stream`, then returns (and clears) the errors the device recorded for this
 * context's asynchronous calls since the last check: NNPS_EORDER if an all-list fill met
 * rows that did not match their count (positions or row pointers changed in between),
 * NNPS_EINVAL if an SPH-gradient call met a neighbour list that did not match its arrays;
 * otherwise NNPS_OK. */
nnps_status nnps_ctx_check(nnps_ctx *ctx, void *stream);

/* Work-shape parameters used by later calls on this context. */
nnps_status nnps_ctx_set_tuning(nnps_ctx *ctx, const nnps_tuning *t);
nnps_status nnps_ctx_get_tuning(const nnps_ctx *ctx, nnps_tuning *t);

/* An empty cell structure; its device buffers grow on demand and are reused. */
nnps_status nnps_cells_create(nnps_ctx *ctx, nnps_cells **out);
void nnps_cells_destroy(nnps_cells *cells);

/* Cell assignment, sort by cell, cell starts and the FP16 pack (paper: Eq. 5-6,
 * Fig. 3b; spatial sort of the Results' memory section). d_pos: [n][dim] float64,
 * device, caller-owned, must outlive the search. Asynchronous. */
nnps_status nnps_cells_build(nnps_ctx *ctx, nnps_cells *cells, const nnps_problem *prob,
                             const double *d_pos, void *stream);

/* Count pass: writes d_row_ptr[0..n] (device int64, caller-owned, n+1 entries).
 * If h_nnz is not NULL, waits for the stream and stores nnz = row_ptr[n] there
 * (and reports device-detected errors); with h_nnz NULL it does not wait. */
nnps_status nnps_count(nnps_ctx *ctx, nnps_cells *cells, int64_t *d_row_ptr, int64_t *h_nnz,
                       void *stream);

/* Fill pass: writes col and dist (device, caller-owned, `capacity` entries each)
 * using the row_ptr written by nnps_count on the same structure (d_row_ptr must still
 * hold exactly what that count wrote: rows are written where it says). If row_ptr[n]
 * exceeds capacity nothing past capacity is written and NNPS_ECAPACITY is
 * reported at the next synchronising call. Asynchronous. */
nnps_status nnps_fill(nnps_ctx *ctx, nnps_cells *cells, const int64_t *d_row_ptr,
                      int32_t *d_col, float *d_dist, int64_t capacity, void *stream);

/* Build + count + fill in one call; synchronises once (after the count) to learn
 * nnz. If capacity < nnz it returns NNPS_ECAPACITY with *nnz_out = nnz and writes
 * only row_ptr. */
nnps_status nnps_search(nnps_ctx *ctx, nnps_cells *cells, const nnps_problem *prob,
                        const double *d_pos, int64_t *d_row_ptr, int32_t *d_col, float *d_dist,
                        int64_t capacity, int64_t *nnz_out, void *stream);

/* Sums the last count pass's per-block statistics on `stream` (the count pass leaves
 * them per block, so a search step does not pay for the sum), waits for the stream and
 * copies them; all zero if nothing was counted since the last build.
 * Returns any device-detected error (NNPS_EDOMAIN, NNPS_ECAPACITY, NNPS_EUNSUPPORTED). */
nnps_status nnps_stats_get(nnps_cells *cells, nnps_stats *out, void *stream);

/* ---- Batches: many independent particle sets searched together -------------------
 * One cell structure holds all sets of a batch in one index space, so every pass is a
 * single kernel launch over the work blocks of every set (uneven sizes welcome). All
 * sets of a batch must share dim and mode. Arrays indexed by set (probs, d_pos,
 * d_row_ptr, d_col, d_dist, capacity, nnz) are host arrays of nsets entries; the device
 * buffers they point to follow the single-set rules above, per set (col holds set-local
 * indices). The statistics of a batch are totals over its sets. */
nnps_status nnps_batch_build(nnps_ctx *ctx, nnps_cells *cells, int32_t nsets, const nnps_problem *probs,
                             const double *const *d_pos, void *stream);
/* Writes each set's row_ptr; with h_nnz (nsets entries) not NULL, waits and returns each
 * set's nnz there. */
nnps_status nnps_batch_count(nnps_ctx *ctx, nnps_cells *cells, int64_t *const *d_row_ptr, int64_t *h_nnz,
                             void *stream);
nnps_status nnps_batch_fill(nnps_ctx *ctx, nnps_cells *cells, int64_t *const *d_row_ptr, int32_t *const *d_col,
                            float *const *d_dist, const int64_t *capacity, void *stream);
/* Build + count (waits once) + fill; NNPS_ECAPACITY if some capacity[s] < nnz_out[s]. */
nnps_status nnps_batch_search(nnps_ctx *ctx, nnps_cells *cells, int32_t nsets, const nnps_problem *probs,
                              const double *const *d_pos, int64_t *const *d_row_ptr, int32_t *const *d_col,
                              float *const *d_dist, const int64_t *capacity, int64_t *nnz_out, void *stream);

/* Build + count + fill without waiting (capacities known in advance, e.g. from an earlier
 * step). With graphs on (nnps_cells_set_graphs) and a non-null stream, the whole
 * sequence is captured as one HIP graph on first use and replayed while the problems,
 * the tuning and the library's buffers stay the same; output and position pointers may
 * change between replays. Capacity overruns are reported by the next synchronising call
 * (nnps_batch_nnz, nnps_stats_get). */
nnps_status nnps_batch_step(nnps_ctx *ctx, nnps_cells *cells, int32_t nsets, const nnps_problem *probs,
                            const double *const *d_pos, int64_t *const *d_row_ptr, int32_t *const *d_col,
                            float *const *d_dist, const int64_t *capacity, void *stream);
nnps_status nnps_cells_set_graphs(nnps_cells *cells, int on);
/* Half lists (on != 0): from the next count on, row i keeps only the neighbours j with
 * j > i (original indices), so every unordered pair appears once, in the row of its
 * smaller index; the CSR and its nnz halve. Distances and statistics are unchanged
 * otherwise (candidates, band pairs and FP16 misclassifications still count every
 * directed pair tested). Default off. Applies to every path of the structure; a
 * following nnps_fill needs a count made in the same setting (else NNPS_EORDER). */
nnps_status nnps_cells_set_half(nnps_cells *cells, int on);
/* Waits for the stream and returns each set's nnz of the last count (nsets entries). */
nnps_status nnps_batch_nnz(nnps_cells *cells, int64_t *h_nnz, void *stream);
/* The same without a synchronous round trip: enqueue copies each set's nnz and the
 * device error flags into the structure's own pinned host memory on `stream` (returns at
 * once); fetch waits for those copies (normally long finished when the caller has seen
 * the step complete) and writes nnz[nsets]. fetch returns the device-detected errors like
 * nnps_batch_nnz, or NNPS_EORDER without a preceding enqueue. */
nnps_status nnps_batch_nnz_enqueue(nnps_cells *cells, void *stream);
nnps_status nnps_batch_nnz_fetch(nnps_cells *cells, int64_t *h_nnz);

/* ---- Incremental update between time steps -----------------------------------------
 * After the particles of a built structure moved, bring the structure up to date without
 * rebuilding it (Mixed-precision SPH framework section: the relative-coordinate update of
 * Eq. 8 and the cell migration of Eq. 9, Fig. 6). The structure works on the position
 * arrays of its last build (nnps_cells_build / nnps_batch_build / nnps_batch_step), which
 * must still be valid. d_disp is NULL, or a host array of nsets entries, each NULL or a
 * device array [n][dim] of float64 displacements of that set:
 *   - with a displacement array, the call advances the positions in place,
 *     pos[i][k] = pos[i][k] + disp[i][k] (one binary64 addition each; the caller's
 *     position array is written), except that a component whose sum would fall outside
 *     [lo[k], hi[k]] moves by -disp[i][k] instead (a reflection at the box faces);
 *   - without one, the caller has already moved the positions in place.
 * Either way each particle's fixed-point position, cell and relative coordinate are
 * recomputed from its binary64 position (so no rounding error builds up from step to
 * step), particles whose cell is unchanged keep their order in it, particles that changed
 * cell are removed from the old one and appended to the new one, and cell starts, the
 * sorted arrays and the work blocks are repaired. The result of the count and fill that
 * follow is exactly that of a fresh build on the moved positions (same row_ptr, col and
 * dist). Positions outside [lo, hi] are reported as NNPS_EDOMAIN by the next
 * synchronising call. NNPS_EORDER if the structure was never built. Asynchronous. */
nnps_status nnps_cells_update(nnps_ctx *ctx, nnps_cells *cells, const double *const *d_disp, void *stream);
/* Update + count + fill without waiting, as nnps_batch_step does for build + count + fill
 * (outputs per set, capacities known in advance). With graphs on and a non-null stream the
 * sequence is captured once and replayed while the grids, the tuning and the library's
 * buffers stay the same; displacement and output pointers may change between replays. */
nnps_status nnps_batch_update_step(nnps_ctx *ctx, nnps_cells *cells, const double *const *d_disp,
                                   int64_t *const *d_row_ptr, int32_t *const *d_col, float *const *d_dist,
                                   const int64_t *capacity, void *stream);

/* ---- All-list search for small sets ------------------------------------------------
 * Every particle tested against every other (SPH method section, Fig. 3a), in binary64
 * with the cell-list paths' predicate, so row_ptr, col and dist are bit-identical to the
 * FP64 cell list (prob->mode and prob->cell_size are not used; the box is only checked).
 * Meant for small sets, with no cell structure: prob->n must not exceed 65536
 * (NNPS_EINVAL above; the work grows as n^2). Rows come out in ascending j.
 *
 * nnps_allpairs_count writes d_row_ptr [n+1] and waits for the stream once to return nnz
 * (*nnz_out); NNPS_EDOMAIN if a position lies outside [lo, hi] or is not finite. The
 * context keeps per-slice row counts (device memory it owns) for the fill that follows.
 * nnps_allpairs_fill queues the fill of d_col/d_dist [nnz] (asynchronous); it must follow
 * a successful count on the same context with the same problem, d_pos and d_row_ptr
 * (else NNPS_EORDER), and needs capacity >= nnz (else NNPS_ECAPACITY, nothing written).
 * The contents of d_pos and d_row_ptr must also be unchanged since the count; the fill
 * cannot tell a change from here, but it writes each row only inside [row_ptr[i],
 * min(row_ptr[i+1], capacity)), and a row whose pairs no longer match its count is
 * reported as NNPS_EORDER by the next nnps_ctx_check. A later count on the context
 * replaces the kept counts: a fill still queued on another stream must have finished by
 * then.
 * nnps_allpairs_search is count then, if capacity >= nnz, fill: NNPS_OK, or
 * NNPS_ECAPACITY with *nnz_out = nnz and only row_ptr written. */
nnps_status nnps_allpairs_count(nnps_ctx *ctx, const nnps_problem *prob, const double *d_pos, int64_t *d_row_ptr,
                                int64_t *nnz_out, void *stream);
nnps_status nnps_allpairs_fill(nnps_ctx *ctx, const nnps_problem *prob, const double *d_pos,
                               const int64_t *d_row_ptr, int32_t *d_col, float *d_dist, int64_t capacity,
                               void *stream);
nnps_status nnps_allpairs_search(nnps_ctx *ctx, const nnps_problem *prob, const double *d_pos,
                                 int64_t *d_row_ptr, int32_t *d_col, float *d_dist, int64_t capacity,
                                 int64_t *nnz_out, void *stream);

/* The same search for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): count and fill as in
 * nnps_allpairs_search, with the per-slice row counts and the error word kept in a
 * static device array of the library (2.25 MiB per device, held until the process ends;
 * its address is looked up when a context is created on the device) instead of memory
 * the context allocates. Makes no hipMalloc, hipFree or other allocating call. The same
 * limits: prob->n <= 65536 (NNPS_EINVAL above; the array is sized for that maximum);
 * waits for the stream once (after the count) to return *nnz_out; NNPS_EDOMAIN,
 * NNPS_ECAPACITY (with *nnz_out = nnz and only row_ptr written) as there; NNPS_EDEVICE
 * if the array's address could not be found. Every call on a device shares that
 * device's array, so calls that overlap on one device (other host threads or streams)
 * race and must be serialised by the caller; the array keeps the last call's contents
 * (each call clears what it needs). Leaves the context's all-list count state alone. */
nnps_status nnps_allpairs_search_noalloc(nnps_ctx *ctx, const nnps_problem *prob, const double *d_pos,
                                         int64_t *d_row_ptr, int32_t *d_col, float *d_dist, int64_t capacity,
                                         int64_t *nnz_out, void *stream);

/* ---- SPH gradient over a neighbour list ------------------------------------------
 * The SPH approximation of the gradient of a scalar field f (SPH method section, Eq. 2,
 * with the cubic B-spline kernel of Eq. 3, support 2h) and the normalised, volume-free
 * first-order operator of the appendix (Eq. A5), in binary64, for one set of n particles
 * in dim (2 or 3) dimensions. d_pos [n][dim], d_f [n] and d_vol [n] (particle volumes V_j;
 * NULL means V_j = 1) are device arrays; d_row_ptr [n+1] and d_col [ncol] are a CSR
 * neighbour list such as nnps_search writes (a row may hold any neighbours; those at
 * r >= 2h add nothing; ncol >= d_row_ptr[n] is the caller's to ensure). The kernel reads
 * d_col only in [0, ncol) (row bounds are clamped to it) and skips column indices
 * outside [0, n), so a list that does not match ncol or n can give wrong sums for the
 * rows concerned but never makes it read outside the arrays; such a list is reported as
 * NNPS_EINVAL by the next nnps_ctx_check on the context. Outputs, each NULL or a
 * device array [n][dim]:
 *   d_grad[i][a]      = sum_j V_j f_j dW_ij/dx_i,a
 *   d_grad_norm[i][a] = sum_j (f_j - f_i) dW_ij/dx_i,a / sum_j (x_j,a - x_i,a) dW_ij/dx_i,a
 *                       (0 where the denominator is 0, e.g. an empty row),
 * with dW_ij/dx_i,a = alpha_d / h * dW/dq (q = r_ij / h) * (x_i,a - x_j,a) / r_ij (0 when
 * r_ij = 0), alpha_d = 15 / (7 pi h^2) in 2D and 3 / (2 pi h^3) in 3D. Every input pointer
 * but d_vol must be non-NULL when n > 0 (d_col when ncol > 0). Asynchronous on `stream`;
 * NNPS_EINVAL for bad arguments (h <= 0 or not finite, dim not 2 or 3, n outside
 * [0, 2^31), ncol < 0). */
nnps_status nnps_sph_gradient(nnps_ctx *ctx, int32_t dim, int64_t n, double h, const double *d_pos,
                              const double *d_f, const double *d_vol, const int64_t *d_row_ptr,
                              const int32_t *d_col, int64_t ncol, double *d_grad, double *d_grad_norm,
                              void *stream);

/* ---- Measurement helper (not part of the search) -------------------------------------
 * The VALU issue rate device `device` reaches on long runs of independent vector
 * instructions of one kind: kind 0 packed FP16 fused multiply-add (two FP16 lanes per
 * instruction, the search's test), 1 FP32 fused multiply-add, 2 32-bit integer add and
 * xor. Every SIMD gets several wavefronts; one launch is timed with HIP events on the
 * null stream (the call waits for it). *rate receives wave64 instructions per second;
 * *insts_per_wave (may be NULL) the timed loop's VALU instructions per wavefront, for
 * checking against a profiler's instruction count. It allocates and frees 64 bytes of
 * device memory. NNPS_EINVAL for a kind outside 0..2 or a NULL rate, NNPS_EDEVICE if a
 * HIP call fails. */
nnps_status nnps_probe_valu_rate(int32_t device, int32_t kind, double *rate, int64_t *insts_per_wave);

/* Phases timed when profiling is on, in launch order. */
enum {
    NNPS_PHASE_ASSIGN = 0,   /* FP64 cell assignment + cell histogram */
    NNPS_PHASE_CELLSCAN,     /* exclusive scan of the histogram -> cell starts */
    NNPS_PHASE_SORT,         /* radix sort of (cell key, index) */
    NNPS_PHASE_PACK,         /* FP16 relative-coordinate pack (or sorted FP64 copy) */
    NNPS_PHASE_BLOCKS,       /* work-block table */
    NNPS_PHASE_UNIONS,       /* dense cells: stencil-union lists sorted by original index */
    NNPS_PHASE_COUNT,        /* count pass (stencil test + recheck) */
    NNPS_PHASE_DCOUNT,       /* count pass of the dense-cell path */
    NNPS_PHASE_ROWSCAN,      /* counts -> row_ptr */
    NNPS_PHASE_FILL,         /* fill pass (stencil test + recheck + sorted CSR writes) */
    NNPS_PHASE_LONGROWS,     /* long-row path of the fill */
    NNPS_PHASE_DFILL,        /* fill pass of the dense-cell path */
    NNPS_NPHASES
};

/* Turn per-phase HIP-event timing on (on != 0) or off for a cell structure, and forget
 * what was recorded. Events are recorded on the stream of each call; no extra
 * synchronisation is added. */
nnps_status nnps_cells_set_profiling(nnps_cells *cells, int on);

/* Waits for the stream, then writes for each phase the summed device time in
 * milliseconds (ms[NNPS_NPHASES]) and the number of timed launches (runs[NNPS_NPHASES])
 * since profiling was turned on or last read, and starts a new tally. */
nnps_status nnps_phase_times(nnps_cells *cells, double *ms, int32_t *runs, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NNPS_H */
