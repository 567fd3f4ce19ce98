/*
 * sigk.h -- C ABI of libsigk: the signature kernel of pairs of time series on
 * AMD Instinct MI355X (gfx950), by tile-wise local power-series (Neumann)
 * propagation over the Goursat grid (arXiv 2502.20392, "PowerSig").
 *
 * Problem statement (Sec. 2.1, Definition 2.1).  A time series z is a
 * row-major array [len][d] of FP64 points; its affine interpolant has
 * increments dz_k = z_{k+1} - z_k.  The signature kernel k(x, y) = K(1, 1),
 * where K solves the Goursat problem d2K/dsdt = rho K on [0,1]^2 with
 * K(0, .) = K(., 0) = 1 and rho tilewise constant.  Cell (k, l) of the grid
 * (k indexes the len_x - 1 segments of x, l those of y) carries the
 * coefficient <dx_k, dy_l>.  Lengths may differ (no padding is applied; the
 * paper's padding by repeated end points gives the same value).  A path with
 * fewer than two points gives k = 1.  The Gram matrix of a family is
 * G_ij = k(x_i, x_j) (Proposition A.3).
 *
 * Method (Prop. 2.5, Prop. 2.8).  Each cell's solution is a local power
 * series; the boundary series (top and right edges) of each cell feed the
 * next cells along the tile DAG in topological (anti-diagonal) order.  The
 * Neumann series of a cell is cut adaptively: its terms are dropped once
 * their bound falls under `tol` relative to the edge data (the per-tile
 * stopping rule of App. B, with a tolerance scaled to the pair's size).  The
 * edge series keep `order` coefficients; the error this drops is estimated
 * cell by cell and summed over each pair (the local truncation error of
 * App. C, "Error Analysis and Limitations"), and a pair whose estimate
 * exceeds its budget raises SIGK_WARN_TRUNC.
 *
 * Conventions for every entry point below:
 *   - All array pointers are DEVICE pointers unless marked "host".
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *     = the null stream).  No call allocates device memory or synchronises
 *     the device, except those marked "synchronous".
 *   - `ws` is a caller-owned device workspace of at least the size returned
 *     by the matching *_workspace_size call.  The library keeps no pointer
 *     after a call returns.  Two calls may not share a workspace concurrently.
 *   - Return value: SIGK_OK or a negative SIGK_E* code from host-side
 *     validation or the kernel launch.  Numerical warnings raised on the
 *     device are written to a status word inside `ws`; read them with
 *     sigk_read_status after the stream has reached the call.
 *   - Outputs not written because of an error are left undefined.
 */
#ifndef SIGK_H
#define SIGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SIGK_OK 0
#define SIGK_EINVAL (-1)      /* null pointer, bad size, d < 1, id out of range  */
#define SIGK_EWORKSPACE (-2)  /* workspace too small                             */
#define SIGK_EDEVICE (-3)     /* HIP runtime error (see sigk_strerror)          */
#define SIGK_EUNSUPPORTED (-4) /* order or dimension outside the compiled range  */

/* device status bits (sigk_read_status) */
#define SIGK_WARN_TRUNC 1u     /* a pair's estimated truncation error exceeded
                                  its budget (tail_tol): raise the order        */
#define SIGK_WARN_NONFINITE 2u /* NaN or Inf produced                              */
#define SIGK_ERR_WATCHDOG 4u   /* a dependency wait exceeded its time limit; the
                                  results of that call are invalid                */
#define SIGK_ERR_TABLE 8u      /* a device pair table named a path id out of range,
                                  an offset outside the pool or a path longer than
                                  max_len: those pairs are skipped (value NaN, no
                                  gradient)                                       */

/* flags */
#define SIGK_FLAG_FIXED_DEPTH 1u /* no adaptive Neumann depth: all order-1 terms  */
#define SIGK_FLAG_SQUARE 2u      /* square truncation of every tile's coefficient
                                    matrix, 0 <= i, j <= N = order-1: the fixed-
                                    order approximant of App. C and Prop. A.3.
                                    With SIGK_FLAG_FIXED_DEPTH and order 8 it is
                                    the paper's default fixed order N = 7 (Sec. 3).
                                    Compiled for order 8, forward calls only;
                                    other orders and the adjoint return
                                    SIGK_EUNSUPPORTED.                          */

typedef struct sigk_opts {
    double tol;        /* Neumann-depth tolerance per cell: term n is skipped for
                          the whole wave once |c|^n/(n!)^2 <= tol in every lane of
                          a chunk.  These per-cell bounds add up over the cells
                          of a pair, so <= 0 selects min(2^-53, 2^-36/cells) with
                          cells = (lx-1)(ly-1) of the largest pair of the call.   */
    double tail_tol;   /* budget of a pair's estimated relative truncation error:
                          the sum over its cells of |c| (|A'_{P-1}| + |B'_{P-1}|)/P!
                          (the leading dropped coefficient of both output edges,
                          in the derivative basis) relative to the local size of
                          K; above it SIGK_WARN_TRUNC is raised.  <= 0: 2^-36.   */
    int32_t order;     /* P = coefficients kept per edge series (degree P-1);
                          0 selects 12.  Rounded up to a compiled value
                          (4,5,6,8,10,12,16,20,24).                               */
    int32_t grid;      /* persistent workgroups; 0 = fill the device              */
    uint32_t flags;    /* SIGK_FLAG_*                                              */
    int32_t tile_cols; /* work tile of the forward sweeps with d <= 32: 64 grid
                          rows x tile_cols columns per frontier chunk.  0 = the
                          compiled default for (order, d); the other compiled
                          width (32 or 64) may be chosen, e.g. by an autotuner;
                          any other value gives SIGK_EUNSUPPORTED.  The
                          checkpointing and adjoint sweeps ignore it.           */
} sigk_opts;

typedef struct sigk_counters {
    uint64_t cells; /* Goursat cells evaluated                                 */
    uint64_t flops; /* algorithmic FP64 flops of the truncated cell maps applied
                       (FMA = 2), including the increment inner products     */
    uint32_t status;
    uint32_t order; /* compiled edge order P used by the last call          */
    double trunc_est; /* largest per-pair truncation estimate (see tail_tol) of
                         the last forward sweep                              */
    uint64_t bwd_cells; /* cells of the last adjoint sweep                     */
    uint64_t bwd_flops; /* its algorithmic FP64 flops: adjoint cell maps, the
                           forward maps they recompute, dL/dc and its chain to
                           both increments (FMA = 2)                         */
} sigk_counters;

/* Default options (tol by size, tail_tol 2^-36, order 12). host */
void sigk_default_opts(sigk_opts* o);

#define SIGK_FLAG_FIELD 4u /* compute the cell coefficients of a pair or Gram
                              call with the matrix-core field stage even for
                              d <= 32 (it is always used for d > 32)          */

/* ---------------------------------------------------------------- one pair */
/*
 * Workspace bytes for sigk_pair with these sizes (host, no device access).
 * lx, ly: points of x and y; d: channels.
 */
int sigk_pair_workspace_size(int64_t lx, int64_t ly, int64_t d, const sigk_opts* o,
                             size_t* bytes);
/*
 * k(x, y) for one pair (Definition 2.1).  x: [lx][d], y: [ly][d] row-major
 * FP64; k_out: one double.  Any lx, ly >= 0 (fewer than 2 points: k = 1).
 * Any d >= 1: up to d = 32 the cell coefficients <dx_k, dy_l> are formed in
 * the sweep; for d > 32 (or with SIGK_FLAG_FIELD) they are computed first on
 * the FP64 matrix cores as the product of the two increment sequences and
 * stored in the workspace, (lx + 63) x 64 doubles per 64 rows of y (the
 * ragged plans, the one-call ragged forms and the adjoint take d <= 32).
 */
int sigk_pair(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
              const sigk_opts* o, double* k_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- Gram */
int sigk_gram_workspace_size(int64_t nx, int64_t ny, int64_t lx, int64_t ly, int64_t d,
                             int symmetric, const sigk_opts* o, size_t* bytes);
/*
 * Gram matrix G[i*ny + j] = k(X_i, Y_j) (Proposition A.3).  X: [nx][lx][d],
 * Y: [ny][ly][d], G: [nx][ny] row-major.  symmetric != 0 requires X == Y
 * (same pointer, nx == ny, lx == ly): only i <= j is computed and mirrored.
 */
int sigk_gram(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t lx, int64_t ly,
              int64_t d, int symmetric, const sigk_opts* o, double* G, void* ws,
              size_t ws_bytes, void* stream);

/*
 * sigk_gram without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP-graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, values and kernels as sigk_gram
 * (sigk_pair is its 1 x 1 case); the workspace is a file-scope device array of
 * SIGK_STATIC_WS_BYTES held by every device the library runs on until the
 * process ends.  Calls that would need more return SIGK_EWORKSPACE before
 * any device work.  The call allocates nothing (no hipMalloc, no hipFree, no
 * allocating library routine) and is asynchronous on `stream`.
 *   status (device, optional): receives the call's SIGK_WARN_* / SIGK_ERR_*
 *          bits, written on `stream` after the launch (NULL: not reported).
 * All calls on one device share the array: calls that overlap on a device
 * (other streams, unordered host threads) race and give undefined results.
 */
#define SIGK_STATIC_WS_BYTES (64u << 20)
int sigk_gram_static(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t lx,
                     int64_t ly, int64_t d, int symmetric, const sigk_opts* o, double* G,
                     uint32_t* status, void* stream);

/* ---------------------------------------------------------------- ragged batch */
/*
 * A plan describes a ragged batch of pairs of paths of different lengths
 * stored back to back in one pool.  It is built on the host from host
 * arrays:
 *   offsets (host) [npaths+1]: first point of each path in the pool; path p has
 *           offsets[p+1]-offsets[p] points;
 *   pairs   (host) [npairs][2]: path ids (x, y) of each pair.
 * The plan fixes the work order (strips of all pairs, largest pairs first)
 * and the workspace layout.  It is owned by the caller (sigk_plan_destroy).
 */
typedef struct sigk_plan sigk_plan;
int sigk_plan_ragged(const int64_t* offsets, int64_t npaths, int64_t d, const int32_t* pairs,
                     int64_t npairs, const sigk_opts* o, sigk_plan** plan);
void sigk_plan_destroy(sigk_plan* plan);
/* Workspace bytes for sigk_plan_run / sigk_plan_backward (host). */
size_t sigk_plan_workspace_size(const sigk_plan* plan);
size_t sigk_plan_backward_workspace_size(const sigk_plan* plan);
/* Number of Goursat cells of the batch (host). */
uint64_t sigk_plan_cells(const sigk_plan* plan);
/*
 * Copy the plan's device tables into ws (asynchronous on stream from host
 * memory held by the plan; keep the plan alive until the stream has passed
 * this call).  Needed once per workspace before sigk_plan_run.
 */
int sigk_plan_upload(const sigk_plan* plan, void* ws, size_t ws_bytes, void* stream);
/*
 * Output slots (host, before sigk_plan_upload): pair p writes
 * out[out_index[p]] instead of out[p], and the plan's calls touch no other
 * element of out, so several plans (for example one per edge order) can fill
 * one output array.  out_index [npairs]: distinct values in
 * [0, 2^30); SIGK_EINVAL otherwise.  out must then hold max(out_index) + 1
 * doubles.  The adjoint's grad_out stays indexed by the plan's pair order.
 */
int sigk_plan_set_outputs(sigk_plan* plan, const int64_t* out_index);
/*
 * Byte offset in the plan's workspace of its per-pair truncation estimates
 * (npairs doubles, the sum over each pair's cells described under tail_tol),
 * valid once the stream has passed a forward call of the plan (host).
 */
size_t sigk_plan_estimates_offset(const sigk_plan* plan);
/*
 * The plan's work order (host, diagnostics): the forward (adjoint != 0: the
 * adjoint) ticket table as [n][2] (pair, strip) into out (host, cap pairs of
 * int32; out NULL: only the count).  Every strip of every pair with cells
 * appears once; a strip's producer (the strip below it in the forward, the
 * strip above it in the adjoint) comes earlier, so a persistent workgroup
 * never waits on a ticket nobody has claimed.  SIGK_EINVAL for plans of the
 * one-call forms (their tables are built on the device; see
 * sigk_ragged_tables) or cap < n.
 */
int sigk_plan_tickets(const sigk_plan* plan, int adjoint, int32_t* out, int64_t cap,
                      int64_t* n_out);
/*
 * Evaluate the batch: out[p] = k(path pairs[p][0], path pairs[p][1]).
 * pool: [sum len][d] FP64 device.  One persistent launch preceded by a small
 * reset kernel, no host-device copies: capturable in a HIP graph.
 */
int sigk_plan_run(const sigk_plan* plan, const double* pool, double* out, void* ws,
                  size_t ws_bytes, void* stream);
/*
 * One-call ragged batch on DEVICE tables (Proposition A.3's Gram entries for
 * an arbitrary list of pairs of paths of different lengths, Definition 2.1
 * for each): out[p] = k(path pairs[p][0], path pairs[p][1]).
 *   pool (device) [pool_points][d]: the paths back to back;
 *   offsets (device) [npaths+1]: first point of each path in the pool;
 *   pairs (device) [npairs][2]: path ids of each pair;
 *   max_len: an upper bound on the points of every path a pair names (host
 *            scalar; it sizes the workspace: every pair is laid out for paths
 *            of max_len points);
 *   out (device) [npairs].
 * The descriptor and ticket tables are built on the device by small kernels
 * before the persistent launch, so the call allocates nothing, copies nothing
 * from the host, never synchronises and can be captured in a HIP graph.
 * Pairs whose table entries are invalid (path id out of range, offsets
 * decreasing or outside [0, pool_points], a path longer than max_len) get
 * out = NaN and raise SIGK_ERR_TABLE; the others are computed normally.
 * ws: at least sigk_gram_ragged_workspace_size bytes (host, from the same
 * scalars).
 */
int sigk_gram_ragged_workspace_size(int64_t npaths, int64_t npairs, int64_t max_len,
                                    int64_t pool_points, int64_t d, const sigk_opts* o,
                                    size_t* bytes);
int sigk_gram_ragged(const double* pool, int64_t pool_points, const int64_t* offsets,
                     int64_t npaths, int64_t d, const int32_t* pairs, int64_t npairs,
                     int64_t max_len, const sigk_opts* o, double* out, void* ws, size_t ws_bytes,
                     void* stream);

/* ---------------------------------------------------------------- adjoint */
/*
 * Gradient of L = sum_p grad_out[p] * k(pair p) with respect to the pool:
 * grad_pool[i][c] += dL/dpool[i][c] (ACCUMULATED).  grad_out: [npairs]
 * device; grad_pool: [sum len][d] device.  The plan must have been uploaded
 * into ws (workspace of sigk_plan_backward_workspace_size bytes).  Runs a
 * checkpointing forward pass and a reverse (adjoint) sweep of the discrete
 * cell maps in reverse wavefront order, then chains through
 * c_kl = <dx_k, dy_l> and dx_k = x_{k+1} - x_k.
 */
int sigk_plan_backward(const sigk_plan* plan, const double* pool, const double* grad_out,
                       double* grad_pool, void* ws, size_t ws_bytes, void* stream);
/*
 * The two halves of sigk_plan_backward, for callers that need the kernel
 * values before the gradient (an autograd forward pass):
 * sigk_plan_run_checkpointed computes out[p] = k(pair p) like sigk_plan_run
 * by the checkpointing forward sweep, leaving its checkpoints in ws (backward
 * workspace size; the plan must have been uploaded into ws);
 * sigk_plan_backward_checkpointed then accumulates the gradient of
 * sum_p grad_out[p] k_p into grad_pool from those checkpoints, without
 * recomputing the forward.  The pool must be unchanged in between and ws not
 * used for any other call; the adjoint may be run several times (different
 * grad_out) on one set of checkpoints.
 */
int sigk_plan_run_checkpointed(const sigk_plan* plan, const double* pool, double* out, void* ws,
                               size_t ws_bytes, void* stream);
int sigk_plan_backward_checkpointed(const sigk_plan* plan, const double* pool,
                                    const double* grad_out, double* grad_pool, void* ws,
                                    size_t ws_bytes, void* stream);

/*
 * Gradient of L = sum_p grad_out[p] * k(pair p) with respect to the pool, on
 * DEVICE tables as for sigk_gram_ragged (same arguments and validation), in
 * one asynchronous call: grad_pool[i][c] += dL/dpool[i][c] (ACCUMULATED).
 * dk/dpool follows from the Volterra form of the Goursat problem (Sec. 2.1):
 * the derivative of K(1, 1) with respect to the coefficient of a cell is the
 * integral over the cell of K times the solution of the adjoint (reversed)
 * problem; it is evaluated here as the exact adjoint of the truncated cell
 * maps, swept in reverse wavefront order over checkpoints of a forward sweep,
 * then chained through c_kl = <dx_k, dy_l> and dx_k = x_{k+1} - x_k.
 *   grad_out (device) [npairs]; grad_pool (device) [pool_points][d].
 * Allocates nothing, never synchronises, capturable; invalid pairs raise
 * SIGK_ERR_TABLE and contribute no gradient.  ws: at least
 * sigk_backward_workspace_size bytes.
 */
/*
 * Where the one-call forms build their ticket table in ws (host,
 * diagnostics): byte offset of the [ntickets][2] int32 (pair, strip) table of
 * sigk_gram_ragged (adjoint == 0) or of sigk_backward's adjoint order
 * (adjoint != 0; its forward order sits at the offset returned for 0 with the
 * same sizes), valid once the stream has passed the call.  Unused slots at
 * the end hold pair -1.
 */
int sigk_ragged_tables(int64_t npaths, int64_t npairs, int64_t max_len, int64_t pool_points,
                       int64_t d, const sigk_opts* o, int adjoint, size_t* tickets_offset,
                       int64_t* ntickets);
int sigk_backward_workspace_size(int64_t npaths, int64_t npairs, int64_t max_len,
                                 int64_t pool_points, int64_t d, const sigk_opts* o,
                                 size_t* bytes);
int sigk_backward(const double* pool, int64_t pool_points, const int64_t* offsets,
                  int64_t npaths, int64_t d, const int32_t* pairs, int64_t npairs,
                  int64_t max_len, const double* grad_out, const sigk_opts* o, double* grad_pool,
                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- long pair gradient */
/*
 * k(x, y) and its gradient for ONE pair with block (two-level) checkpointing,
 * for pairs too long for per-strip checkpoints (memory of order
 * (lx + ly) P sqrt(lx ly) instead of lx ly P):
 *   grad_x[i][c] += grad_out[0] dk/dx[i][c],  grad_y[j][c] += grad_out[0] dk/dy[j][c].
 * The derivative is the one sigk_backward computes (the exact adjoint of the
 * truncated cell maps, chained through c_kl = <dx_k, dy_l>; Sec. 2.1, Prop.
 * 2.5), evaluated in three stages on `stream`:
 *   1. one forward sweep of the whole pair, which writes k(x, y) and keeps
 *      the edge series on the boundaries of blocks of block_rows x block_cols
 *      cells (the top edges of every block row's last row, the right edges of
 *      every block column's last column);
 *   2. block anti-diagonal by anti-diagonal, from the top-right corner down:
 *      the forward sweep of each block recomputed from its boundary series
 *      with per-strip checkpoints, then its adjoint sweep, which takes the
 *      cotangents of the block's top and right edges from the blocks above
 *      and to the right and leaves those of its bottom and left edges;
 *   3. the chain to the points.
 * x: [lx][d], y: [ly][d] (device, FP64); d <= 32.  grad_out (device) [1].
 * k_out (device) [1] or NULL.  grad_x [lx][d], grad_y [ly][d] (device),
 * ACCUMULATED.  block_rows: a multiple of 64, block_cols >= 1; 0 chooses a
 * square block near sqrt(14.2 max(lx, ly)) (least workspace).  Truncation
 * warnings of the forward sweep go to the status word as for sigk_pair.
 * Allocates nothing, never synchronises.  ws: at least
 * sigk_pair_backward_workspace_size bytes (host, same sizes);
 * sigk_pair_backward_blocks (host) returns the block sizes used.
 */
int sigk_pair_backward_workspace_size(int64_t lx, int64_t ly, int64_t d, int64_t block_rows,
                                      int64_t block_cols, const sigk_opts* o, size_t* bytes);
int sigk_pair_backward_blocks(int64_t lx, int64_t ly, int64_t d, int64_t block_rows,
                              int64_t block_cols, const sigk_opts* o, int64_t* rows_out,
                              int64_t* cols_out);
int sigk_pair_backward(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                       const double* grad_out, int64_t block_rows, int64_t block_cols,
                       const sigk_opts* o, double* k_out, double* grad_x, double* grad_y,
                       void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- order estimate */
/*
 * A-priori truncation order (App. C, "Error Analysis and Limitations": the
 * tile matrix at the largest cell coefficient, its last row and column summed
 * and scaled to the cell size, searched over N).  Reading taken here: with
 * cmax the largest |<dx_k, dy_l>| of the grid and h the derivative scale of
 * the edges in unit cells (max(max|dx| max|y - y_0|, max|dy| max|x - x_0|)),
 * the edge coefficients are bounded by h^r/r!, the last row and column of the
 * (N+1) x (N+1) tile matrix sum to E(N) = 2/N! sum_{j<=N} cmax^j h^(N-j)/j!,
 * and the local errors add up over the cells.
 *
 * sigk_order_bound (host only): the least N in [1, 64] with
 * cells * E(N) <= tol -> *N_out (and the bound); SIGK_EUNSUPPORTED with
 * N_out = 64 if none.  SIGK_EINVAL on negative or non-finite arguments.
 */
int sigk_order_bound(double cmax, double h, double cells, double tol, int* N_out,
                     double* bound_out);
/*
 * The same for a pair on the device: x [lx][d], y [ly][d]; the statistics
 * (cmax over all cells, path increments and excursions) come from small
 * kernels on `stream`, then the call WAITS for them (synchronous) and returns
 * *order_out = the smallest compiled edge order P >= N + 1 (0 and
 * SIGK_EUNSUPPORTED if none) and the bound at N.  ws: at least 256 bytes of
 * device scratch.  Paths of more than 4,194,240 points are not supported.
 */
int sigk_estimate_order(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                        double tol, int* order_out, double* bound_out, void* ws,
                        size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- status */
/* Synchronous: waits for stream, reads counters and the status word of ws. */
int sigk_read_counters(const void* ws, sigk_counters* out, void* stream);
int sigk_read_status(const void* ws, uint32_t* status_bits, void* stream);
/* Message for a return code (static string). */
const char* sigk_strerror(int code);
/* Compiled edge orders and dimension buckets (host). */
int sigk_supported_order(int order); /* smallest compiled P >= order, or 0 */
/* Forward work-tile widths (sigk_opts.tile_cols) compiled for this order and
   d (host): the default (alternative == 0) or the other one; 0 if none (d > 32
   has only the default of the coefficient-field sweep). */
int sigk_tile_cols(int order, int64_t d, int alternative);
/* Persistent workgroups that fill the current device for this variant (host;
   queries the HIP runtime, no device work).  0 if the variant does not exist. */
int sigk_device_grid(int order, int64_t d, int backward);

#ifdef __cplusplus
}
#endif
#endif /* SIGK_H */
