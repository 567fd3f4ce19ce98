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
 * next cells along the tile DAG in topological (anti-diagonal) order.  Per
 * cell, the Neumann series is cut adaptively once the next term is below
 * `tol` relative to the edge data (Sec. C.3: "stops once the next term is
 * below machine precision"); the edge series keep `order` coefficients.
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
#define SIGK_WARN_TRUNC 1u     /* an edge series' last kept coefficient exceeded
                                  tail_tol relative to the edge norm: raise order */
#define SIGK_WARN_NONFINITE 2u /* NaN or Inf produced                              */
#define SIGK_ERR_WATCHDOG 4u   /* a dependency wait exceeded its time limit; the
                                  results of that call are invalid                */

/* flags */
#define SIGK_FLAG_FIXED_DEPTH 1u /* no adaptive Neumann depth: all order-1 terms  */

typedef struct sigk_opts {
    double tol;        /* Neumann-depth tolerance per cell: term n is skipped for
                          the whole wave once |c|^n/(n!)^2 <= tol in every lane of
                          a chunk.  These per-cell bounds add up over the cells
                          of a pair, so <= 0 selects min(2^-53, 2^-36/cells) with
                          cells = (lx-1)(ly-1) of the largest pair of the call.   */
    double tail_tol;   /* truncation warning threshold for the last edge
                          coefficient relative to the edge norm; <= 0: 2^-50.     */
    int32_t order;     /* P = coefficients kept per edge series (degree P-1);
                          0 selects 12.  Rounded up to a compiled value
                          (4,5,6,8,10,12,16,20,24).                               */
    int32_t grid;      /* persistent workgroups; 0 = fill the device              */
    uint32_t flags;    /* SIGK_FLAG_*                                              */
    int32_t reserved;
} sigk_opts;

typedef struct sigk_counters {
    uint64_t cells; /* Goursat cells evaluated                                 */
    uint64_t flops; /* algorithmic FP64 flops of the truncated cell maps applied
                       (FMA = 2), including the increment inner products     */
    uint32_t status;
    uint32_t order; /* compiled edge order P used by the last call          */
} sigk_counters;

/* Default options (tol by size, tail_tol 2^-50, order 12). host */
void sigk_default_opts(sigk_opts* o);

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
 * Evaluate the batch: out[p] = k(path pairs[p][0], path pairs[p][1]).
 * pool: [sum len][d] FP64 device.  One persistent launch preceded by a small
 * reset kernel, no host-device copies: capturable in a HIP graph.
 */
int sigk_plan_run(const sigk_plan* plan, const double* pool, double* out, void* ws,
                  size_t ws_bytes, void* stream);
/*
 * Convenience: plan + upload + run in one call (synchronous with respect to
 * the host for the table copy; not capturable).  offsets and pairs are host
 * arrays as for sigk_plan_ragged.
 */
int sigk_gram_ragged(const double* pool, const int64_t* offsets, int64_t npaths, int64_t d,
                     const int32_t* pairs, int64_t npairs, const sigk_opts* o, double* out,
                     void* ws, size_t ws_bytes, void* stream);
/* Workspace bytes for sigk_gram_ragged (host; host offsets and pairs). */
int sigk_gram_ragged_workspace_size(const int64_t* offsets, int64_t npaths, int64_t d,
                                    const int32_t* pairs, int64_t npairs, const sigk_opts* o,
                                    size_t* bytes);

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
 * Convenience: plan + upload + sigk_plan_backward in one call for a ragged
 * batch (the gradient of L = sum_p grad_out[p] k(pair p) with respect to the
 * pool, ACCUMULATED into grad_pool).  offsets and pairs are host arrays as for
 * sigk_plan_ragged; synchronous with respect to the host (the plan's tables
 * are copied from host memory); not capturable.  ws: at least
 * sigk_backward_workspace_size bytes.
 */
int sigk_backward_workspace_size(const int64_t* offsets, int64_t npaths, int64_t d,
                                 const int32_t* pairs, int64_t npairs, const sigk_opts* o,
                                 size_t* bytes);
int sigk_backward(const double* pool, const int64_t* offsets, int64_t npaths, int64_t d,
                  const int32_t* pairs, int64_t npairs, const double* grad_out, const sigk_opts* o,
                  double* grad_pool, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- status */
/* Synchronous: waits for stream, reads counters and the status word of ws. */
int sigk_read_counters(const void* ws, sigk_counters* out, void* stream);
int sigk_read_status(const void* ws, uint32_t* status_bits, void* stream);
/* Message for a return code (static string). */
const char* sigk_strerror(int code);
/* Compiled edge orders and dimension buckets (host). */
int sigk_supported_order(int order); /* smallest compiled P >= order, or 0 */
/* Persistent workgroups that fill the current device for this variant (host;
   queries the HIP runtime, no device work).  0 if the variant does not exist. */
int sigk_device_grid(int order, int64_t d, int backward);

#ifdef __cplusplus
}
#endif
#endif /* SIGK_H */
