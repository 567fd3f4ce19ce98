// sigk_internal.h -- device/host structures shared by the kernels and the
// C-ABI layer of libsigk.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sigk {

constexpr int kWave = 64;   // one wavefront = one strip of 64 grid rows
constexpr int kMaxP = 24;   // largest compiled edge order

// Compiled (P, D) variants of the forward kernel: edge order P (coefficients
// per edge series), channel bucket D (d <= D, padded with zeros).
#define SIGK_FWD_VARIANTS(X) \
    X(4, 8) X(5, 8) X(6, 8) X(8, 8) X(10, 8) X(12, 8) X(16, 8) X(20, 8) X(24, 8) \
    X(4, 16) X(5, 16) X(6, 16) X(8, 16) X(10, 16) X(12, 16) X(16, 16) X(20, 16) X(24, 16) \
    X(4, 32) X(5, 32) X(6, 32) X(8, 32) X(10, 32) X(12, 32) X(16, 32) X(20, 32) X(24, 32)

// Forward variants that read the cell coefficients from a field computed
// beforehand on the matrix cores (channel bucket 0: any d, used for d > 32).
#define SIGK_FWDG_VARIANTS(X) \
    X(4, 0) X(5, 0) X(6, 0) X(8, 0) X(10, 0) X(12, 0) X(16, 0) X(20, 0) X(24, 0)

// Steps per strip stored in a cell-coefficient field (a multiple of the
// chunk width of the channel-bucket-0 sweep).
__host__ __device__ constexpr int64_t delta_steps(int64_t m) {
    return (m + 63 + 31) / 32 * 32;
}

// Square-truncation forward variants (SIGK_FLAG_SQUARE): the paper's default
// fixed order N = 7, i.e. P = 8.
#define SIGK_FWDSQ_VARIANTS(X) X(8, 8) X(8, 16) X(8, 32)

// Variants of the adjoint kernels.
#define SIGK_BWD_VARIANTS(X) \
    X(4, 8) X(5, 8) X(6, 8) X(8, 8) X(10, 8) X(12, 8) X(16, 8) X(20, 8) X(24, 8) \
    X(4, 16) X(5, 16) X(6, 16) X(8, 16) X(10, 16) X(12, 16) X(16, 16) X(20, 16) X(24, 16) \
    X(4, 32) X(5, 32) X(6, 32) X(8, 32) X(10, 32) X(12, 32) X(16, 32) X(20, 32) X(24, 32)

// Frontier chunk (columns per progress flag) of the checkpointing forward
// sweep and of the adjoint, for edge order P.
__host__ __device__ constexpr int chunk_cols(int P) { return 32; }
// Frontier chunk of the plain forward sweep, for edge order P and channel
// bucket D.  Wider chunks halve the flag waits and frontier loads per column
// but lengthen the start lag between strips and take LDS (a wave less per
// CU at D = 8); 64 columns (the most a 128-column ring allows: it holds
// [c0-63, c0+chunk)) pay off at orders 4 and 5 with D = 8 (5-6% faster on
// the long pair, order 6 ran 6% slower: a wave less per CU) and at orders
// 10-20 with D <= 16, which run one wave per SIMD anyway (Gram workloads
// 6-9% faster).  (The adjoint path keeps 32: there the wider buffers cost
// more waves than the exchange saves.)
__host__ __device__ constexpr int fwd_chunk_cols(int P, int D) {
    return D == 0 ? 32 : (P <= 5 && D <= 8) || (P >= 10 && P <= 20 && D <= 16) ? 64 : 32;
}
// Columns of the increment ring in LDS: it holds [c0-63, c0+chunk) while the
// steps of chunk c0 run.  ring_cols: the checkpointing sweep and the adjoint;
// fwd_ring_cols: the plain forward sweep, 128 wherever its chunks are 64
// columns wide.
__host__ __device__ constexpr int ring_cols(int P) { return P <= 8 ? 128 : 96; }
__host__ __device__ constexpr int fwd_ring_cols(int P, int D) {
    return fwd_chunk_cols(P, D) == 64 ? 128 : ring_cols(P);
}
// The other compiled frontier chunk of a (P, D > 0) forward variant: the
// work-tile width (64 rows x chunk columns) an autotuner may pick instead of
// the default, 32 where the default is 64 and 64 where it is 32.  The same
// (P, D) list as SIGK_FWD_VARIANTS is compiled with it (launch_fwdt_P_D).
__host__ __device__ constexpr int alt_chunk_cols(int P, int D) {
    return fwd_chunk_cols(P, D) == 64 ? 32 : 64;
}

// Per-pair geometry for table mode (ragged batches).  Offsets in elements.
struct PairDesc {
    int64_t x_off;      // first double of path x in the pool
    int64_t y_off;      // first double of path y in the pool
    int64_t front_off;  // first double of this pair's frontier row ([m][P])
    int64_t ckpt_off;   // first double of this pair's adjoint checkpoints
    int64_t snap_off;   // first double of this pair's frontier snapshots ([S][m][P])
    int32_t lx, ly;     // points
    int32_t prog_off;   // first progress counter (one per strip)
    int32_t out_idx;    // output slot
    int32_t out_idx2;   // mirror output slot or -1
    int32_t pad;
};
static_assert(sizeof(PairDesc) == 64, "descriptor size");

// Adjoint checkpointing: wave state every kCkptEvery steps; per strip
// ckpt_states(m) states of 2P x 64 doubles followed by the Neumann depth of
// every frontier chunk (stored as doubles, padded to 64).
constexpr int kCkptEvery = 16;
// Per-chunk depth record of the checkpointing sweep: the depth plus
// kRoughFlag where the chunk's bound of |c|^2 exceeds kRoughC2 (the adjoint
// then keeps left edges in its scratch instead of recovering them).
constexpr int kRoughFlag = 64;
constexpr double kRoughC2 = 0.25;
__host__ __device__ constexpr int64_t ckpt_states(int64_t m) {
    return (m + kWave + kCkptEvery - 1) / kCkptEvery + 1;
}
__host__ __device__ constexpr int64_t ckpt_strip_doubles(int64_t m, int P) {
    return ckpt_states(m) * 2 * P * kWave +
           ((m + chunk_cols(P) - 1) / chunk_cols(P) + kWave - 1) / kWave * kWave;
}

struct Ticket {
    int32_t pair;
    int32_t strip;
};

// Header at the start of every workspace.
struct WsHeader {
    unsigned status;           // SIGK_WARN_* / SIGK_ERR_* bits
    unsigned ticket;           // next ticket (forward)
    unsigned long long cells;  // cells evaluated
    unsigned long long flops;  // algorithmic flops
    unsigned order;            // compiled edge order used
    unsigned ticket2;          // next ticket (adjoint)
    double trunc_max;          // largest per-pair truncation estimate
    unsigned long long bwd_cells;  // cells of the adjoint sweep
    unsigned long long bwd_flops;  // algorithmic flops of the adjoint sweep
                                   // (adjoint maps + recomputed forward maps)
    unsigned pad[50];
};
static_assert(sizeof(WsHeader) == 256, "header size");

enum { kModeGram = 0, kModeTable = 1, kModeLines = 2, kModeBlock = 3 };

// Two-level (block) checkpointing of one long pair for its gradient.  The
// grid of m x n cells is cut into blocks of rb rows (a multiple of 64) and cb
// columns.  A first forward sweep over the whole pair (kModeLines) keeps the
// edge series on the block boundaries: the top edges of the last row of every
// block row but the top one (hline, [ni-1][m][P]) and the right edges of the
// last column of every block column but the last one (vline, [nj-1][n][P]).
// Then, block anti-diagonal by anti-diagonal from the top-right corner down,
// each block is a small pair of its own (kModeBlock): its forward sweep is
// recomputed from its bottom and left lines into per-slot checkpoints, and
// its adjoint takes the cotangents of its top and right edges from the blocks
// above and to its right (lam_h: one row of [m][P], shared down each block
// column; lam_v: one column of [n][P], shared along each block row) and
// leaves those of its bottom and left edges in the same places.
struct BlockGeo {
    int64_t m, n;       // cells of the pair
    int rb, cb;         // rows (multiple of 64) and columns per block
    int ni, nj;         // blocks along the rows (y) and the columns (x)
    int kb;             // strips per block, rb / 64
    int diag;           // block anti-diagonal I + J of a kModeBlock launch
    int j_lo, nb;       // its first block column and number of blocks
    double* hline;
    double* vline;
    int64_t slot_snap;  // doubles of frontier snapshots per block slot
    int64_t slot_ckpt;  // doubles of wave-state checkpoints per block slot
    int slot_prog;      // progress counters per slot (kb + 2: a sentinel on
                        // either side, always complete)
    int64_t y_gdx;      // first double of y's increment gradients in gdx
};

struct FwdArgs {
    int mode;
    int symmetric;
    int d;
    int strips;        // strips per pair (gram mode)
    const double* X;   // gram: X batch; table: pool
    const double* Y;   // gram: Y batch; table: pool
    int64_t nx, ny, lx, ly;
    int64_t npairs;
    int64_t ntickets;
    const PairDesc* desc;
    const Ticket* tickets;
    double* out;
    double* frontier;
    int* progress;
    WsHeader* hdr;
    double* ckpt;      // adjoint checkpoints (null: forward only)
    double tau2[kMaxP];  // Neumann term n is needed where |c|^2 > tau2[n]
                         // (|c|^n/(n!)^2 > tol); all < 0 for the fixed depth
    double* trunc_est;   // [npairs] truncation estimate per pair (strips add)
    double* delta;       // channel bucket 0: cell coefficients, per pair
                         // [strips][delta_steps(m)][64] (gram mode)
    int64_t delta_pair;  // doubles per pair in delta
    int ckpt_every;    // steps between wave-state checkpoints (adjoint)
    BlockGeo blk;      // kModeLines / kModeBlock
    long long watchdog_ticks;  // 100 MHz ticks before a wait is abandoned
};

struct BwdArgs {
    FwdArgs f;               // geometry (table mode), depth thresholds
    const Ticket* tickets;   // adjoint order (a pair's strips top-down, producers first)
    int64_t ntickets;
    const double* grad_out;  // [npairs] weights of the kernel values
    double* snap;            // frontier snapshots written by the checkpoint pass
    double* ckpt;            // wave-state checkpoints + per-chunk depths
    double* lam_front;       // adjoint frontier (one row per pair, [m][P])
    double* lam_v;           // kModeBlock: right/left edge cotangents, [n][P]
    int* lam_prog;           // adjoint progress counters (columns done from the right)
    double* gdx;             // [sum len][d]: dL/d(increment) at the increment's first point
    double* scratch;         // per workgroup: kCkptEvery x P x 64 recomputed bottom edges,
                             // then as many left edges (rough segments)
};

// Records the HIP error string for sigk_strerror and returns SIGK_EDEVICE.
int device_error(hipError_t e);

// Launchers implemented per variant (one translation unit each).
#define SIGK_DECL_FWD(P, D) \
    hipError_t launch_fwd_##P##_##D(const FwdArgs& a, int grid, hipStream_t s); \
    int occupancy_fwd_##P##_##D();
SIGK_FWD_VARIANTS(SIGK_DECL_FWD)
SIGK_FWDG_VARIANTS(SIGK_DECL_FWD)
#undef SIGK_DECL_FWD
#define SIGK_DECL_FWDT(P, D) \
    hipError_t launch_fwdt_##P##_##D(const FwdArgs& a, int grid, hipStream_t s); \
    int occupancy_fwdt_##P##_##D();
SIGK_FWD_VARIANTS(SIGK_DECL_FWDT)
#undef SIGK_DECL_FWDT
#define SIGK_DECL_FWDSQ(P, D) \
    hipError_t launch_fwdsq_##P##_##D(const FwdArgs& a, int grid, hipStream_t s); \
    int occupancy_fwdsq_##P##_##D();
SIGK_FWDSQ_VARIANTS(SIGK_DECL_FWDSQ)
#undef SIGK_DECL_FWDSQ

// The cell-coefficient field of every pair of a Gram call (FwdArgs in gram
// mode with delta set), on the matrix cores.
hipError_t launch_delta_gemm(const FwdArgs& a, hipStream_t s);
#define SIGK_DECL_BWD(P, D) \
    hipError_t launch_lines_##P##_##D(const FwdArgs& a, int grid, hipStream_t s); \
    int occupancy_lines_##P##_##D(); \
    hipError_t launch_ckpt_##P##_##D(const FwdArgs& a, int grid, hipStream_t s); \
    hipError_t launch_bwd_##P##_##D(const BwdArgs& a, int grid, hipStream_t s); \
    int occupancy_ckpt_##P##_##D(); \
    int occupancy_bwd_##P##_##D();
SIGK_BWD_VARIANTS(SIGK_DECL_BWD)
#undef SIGK_DECL_BWD

}  // namespace sigk
