// sigk_api.hip -- host side of libsigk: the C ABI declared in include/sigk.h.
//
// Validation, workspace layout, plan construction (ragged batches), variant
// dispatch over the compiled (edge order P, channel bucket D) kernels, and
// the small reset kernel that precedes every persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/sigk.h"
#include "sigk_internal.h"

using namespace sigk;

namespace {

constexpr int kOrders[] = {4, 5, 6, 8, 10, 12, 16, 20, 24};
constexpr int kDims[] = {8, 16, 32};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Variant {
    int P, D;
    hipError_t (*fwd)(const FwdArgs&, int, hipStream_t);
    int (*occ_fwd)();
    hipError_t (*ckpt)(const FwdArgs&, int, hipStream_t);
    hipError_t (*bwd)(const BwdArgs&, int, hipStream_t);
    int (*occ_ckpt)();
    int (*occ_bwd)();
};

#define SIGK_V_FWD(P, D) {P, D, launch_fwd_##P##_##D, occupancy_fwd_##P##_##D, nullptr, nullptr, nullptr, nullptr},
const Variant kFwdTable[] = {SIGK_FWD_VARIANTS(SIGK_V_FWD)};
#undef SIGK_V_FWD
// (the adjoint variants' fwd slot is the first sweep of a long pair's
// gradient, the lines kernel)
#define SIGK_V_BWD(P, D) {P, D, launch_lines_##P##_##D, occupancy_lines_##P##_##D, launch_ckpt_##P##_##D, launch_bwd_##P##_##D, occupancy_ckpt_##P##_##D, occupancy_bwd_##P##_##D},
const Variant kBwdTable[] = {SIGK_BWD_VARIANTS(SIGK_V_BWD)};
#undef SIGK_V_BWD
#define SIGK_V_FWDT(P, D) {P, D, launch_fwdt_##P##_##D, occupancy_fwdt_##P##_##D, nullptr, nullptr, nullptr, nullptr},
const Variant kFwdTTable[] = {SIGK_FWD_VARIANTS(SIGK_V_FWDT)};
#undef SIGK_V_FWDT
#define SIGK_V_FWDSQ(P, D) {P, D, launch_fwdsq_##P##_##D, occupancy_fwdsq_##P##_##D, nullptr, nullptr, nullptr, nullptr},
const Variant kFwdSqTable[] = {SIGK_FWDSQ_VARIANTS(SIGK_V_FWDSQ)};
#undef SIGK_V_FWDSQ
#define SIGK_V_FWDG(P, D) {P, D, launch_fwd_##P##_##D, occupancy_fwd_##P##_##D, nullptr, nullptr, nullptr, nullptr},
const Variant kFwdGTable[] = {SIGK_FWDG_VARIANTS(SIGK_V_FWDG)};
#undef SIGK_V_FWDG

int round_order(int order) {
    if (order <= 0) order = 12;
    for (int p : kOrders)
        if (p >= order) return p;
    return 0;
}
int round_dim(int64_t d) {
    for (int v : kDims)
        if (d <= v) return v;
    return 0;
}
// Channel bucket of a Gram / pair call: 0 (coefficients from the matrix-core
// field stage) for d > 32 or on request, else the compiled bucket.
int bucket_of(int64_t d, uint32_t flags) {
    return (d > 32 || (flags & SIGK_FLAG_FIELD)) ? 0 : round_dim(d);
}

// Work-tile (frontier chunk) choice of a forward call: 0 or the compiled
// default chunk of (P, D), or the alternative one (channel buckets > 0,
// without square truncation).
bool tile_valid(int P, int D, uint32_t flags, int tile) {
    if (tile == 0 || tile == fwd_chunk_cols(P, D)) return true;
    return D > 0 && !(flags & SIGK_FLAG_SQUARE) && tile == alt_chunk_cols(P, D);
}
bool alt_tile(int P, int D, int tile) { return D > 0 && tile != 0 && tile != fwd_chunk_cols(P, D); }
int chunk_of(int P, int D, int tile) { return alt_tile(P, D, tile) ? tile : fwd_chunk_cols(P, D); }

const Variant* find_fwd(int P, int D, uint32_t flags = 0, int tile = 0) {
    if (!tile_valid(P, D, flags, tile)) return nullptr;
    if (alt_tile(P, D, tile)) {
        for (const Variant& v : kFwdTTable)
            if (v.P == P && v.D == D) return &v;
        return nullptr;
    }
    if (D == 0) {
        if (flags & SIGK_FLAG_SQUARE) return nullptr;
        for (const Variant& v : kFwdGTable)
            if (v.P == P) return &v;
        return nullptr;
    }
    if (flags & SIGK_FLAG_SQUARE) {
        for (const Variant& v : kFwdSqTable)
            if (v.P == P && v.D == D) return &v;
        return nullptr;
    }
    for (const Variant& v : kFwdTable)
        if (v.P == P && v.D == D) return &v;
    return nullptr;
}
const Variant* find_bwd(int P, int D, uint32_t flags = 0) {
    if (flags & SIGK_FLAG_SQUARE) return nullptr;  // forward-only mode
    for (const Variant& v : kBwdTable)
        if (v.P == P && v.D == D) return &v;
    return nullptr;
}

std::mutex g_mu;
struct OccKey {
    int dev, P, D, kind;
    int value;
};
std::vector<OccKey> g_occ;
int g_cus[64] = {0};

// resident workgroups per device for a variant's forward, adjoint or
// checkpoint kernel (their register and LDS footprints differ)
enum {
    kKernelFwd = 0,
    kKernelBwd = 1,
    kKernelCkpt = 2,
    kKernelFwdSq = 3,
    kKernelLines = 4,
    kKernelFwdT = 5  // forward with the alternative work tile
};

int fwd_kind(int P, int D, uint32_t flags, int tile) {
    return (flags & SIGK_FLAG_SQUARE) ? kKernelFwdSq
                                      : (alt_tile(P, D, tile) ? kKernelFwdT : kKernelFwd);
}

int device_wgs(int P, int D, int kind) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& k : g_occ)
        if (k.dev == dev && k.P == P && k.D == D && k.kind == kind) return k.value;
    if (dev < 64 && g_cus[dev] == 0) {
        int cus = 0;
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        g_cus[dev] = cus;
    }
    int occ = 0;
    if (kind == kKernelFwd || kind == kKernelFwdSq || kind == kKernelFwdT) {
        const Variant* v = find_fwd(P, D, kind == kKernelFwdSq ? SIGK_FLAG_SQUARE : 0,
                                    kind == kKernelFwdT ? alt_chunk_cols(P, D) : 0);
        occ = v ? v->occ_fwd() : 0;
    } else {
        const Variant* v = find_bwd(P, D);
        occ = v ? (kind == kKernelBwd    ? v->occ_bwd()
                   : kind == kKernelLines ? v->occ_fwd()
                                          : v->occ_ckpt())
                : 0;
    }
    if (occ < 1) occ = 1;
    int value = occ * (dev < 64 ? g_cus[dev] : 256);
    g_occ.push_back({dev, P, D, kind, value});
    return value;
}

// Per-cell Neumann tolerance.  A dropped term n is bounded by |c|^n/(n!)^2
// relative to the edge data, and since the kernel value is a linear function
// of every cell's local error with O(1) weights, these bounds add up over all
// cells of a pair.  The default therefore scales with the largest pair:
// tol = min(2^-53, 2^-36 / cells), an accumulated bound of about 1.5e-11.
double default_tol(int64_t max_cells) {
    double t = std::ldexp(1.0, -53);
    if (max_cells > 0) t = std::min(t, std::ldexp(1.0, -36) / (double)max_cells);
    return t;
}

void fill_common(FwdArgs& a, const sigk_opts& o, int P, int64_t d, int64_t max_cells) {
    const double tol = o.tol > 0 ? o.tol : default_tol(max_cells);
    // Neumann term n bounded by |c|^n/(n!)^2 relative to the edge data; it is
    // applied where |c| > tau_n = (tol (n!)^2)^(1/n).  Fixed depth: tau < 0.
    double lf = 0.0;  // log n!
    for (int n = 0; n < kMaxP; ++n) {
        if (n > 0) lf += std::log((double)n);
        double tau = n == 0 ? 0.0 : std::exp((std::log(tol) + 2.0 * lf) / (double)n);
        tau *= 1.0 - 1e-12;  // round the bound outward
        a.tau2[n] = (o.flags & SIGK_FLAG_FIXED_DEPTH) ? -1.0 : tau * tau;
    }
    a.d = (int)d;
    a.watchdog_ticks = 2000000000LL;  // 20 s of the 100 MHz counter
    (void)P;
}

// Budget of a pair's estimated relative truncation error (sum of the cells'
// local estimates, see the strip kernel): the Neumann tolerance's accumulated
// bound, 2^-36 (about 1.5e-11).
double default_budget() { return std::ldexp(1.0, -36); }
double budget_of(const sigk_opts& o) { return o.tail_tol > 0 ? o.tail_tol : default_budget(); }

__global__ void reset_kernel(WsHeader* h, int* prog, int64_t nprog, double* out, int64_t nout,
                             double* est, int64_t nest, unsigned order) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i0 == 0) {
        h->status = 0;
        h->ticket = 0;
        h->ticket2 = 0;
        h->cells = 0;
        h->flops = 0;
        h->order = order;
        h->trunc_max = 0.0;
        h->bwd_cells = 0;
        h->bwd_flops = 0;
    }
    for (int64_t i = i0; i < nprog; i += stride) prog[i] = 0;
    // pairs without cells keep k = 1 (K = 1 on the axes)
    for (int64_t i = i0; i < nout; i += stride) out[i] = 1.0;
    for (int64_t i = i0; i < nest; i += stride) est[i] = 0.0;
}

hipError_t launch_reset(WsHeader* h, int* prog, int64_t nprog, double* out, int64_t nout,
                        double* est, int64_t nest, unsigned order, hipStream_t s) {
    int64_t n = std::max<int64_t>(std::max(std::max(nprog, nout), nest), 1);
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, h, prog, nprog, out, nout,
                       est, nest, order);
    return hipGetLastError();
}

// After a forward sweep: compare every pair's truncation estimate with the
// budget (SIGK_WARN_TRUNC above it, SIGK_WARN_NONFINITE if not finite) and
// record the largest finite one.  One block.
__global__ void finalize_kernel(WsHeader* h, const double* est, int64_t npairs, double budget) {
    __shared__ double smax[256];
    __shared__ unsigned sbits[256];
    double mx = 0.0;
    unsigned bits = 0;
    for (int64_t p = threadIdx.x; p < npairs; p += blockDim.x) {
        const double v = est[p];
        if (!isfinite(v)) bits |= SIGK_WARN_NONFINITE;
        else if (v > budget) bits |= SIGK_WARN_TRUNC;
        if (isfinite(v)) mx = fmax(mx, v);
    }
    smax[threadIdx.x] = mx;
    sbits[threadIdx.x] = bits;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbits[threadIdx.x] |= sbits[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        h->trunc_max = smax[0];
        if (sbits[0]) h->status |= sbits[0];
    }
}

hipError_t launch_finalize(WsHeader* h, const double* est, int64_t npairs, double budget,
                           hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, h, est, npairs, budget);
    return hipGetLastError();
}

thread_local char g_errbuf[256];

// ---------------------------------------------------------------- gram layout
struct GramLayout {
    size_t hdr = 0, prog = 0, est = 0, front = 0, field = 0, total = 0;
    int64_t strips = 0, npairs = 0, nprog = 0, field_pair = 0;
};

GramLayout gram_layout(int64_t nx, int64_t ny, int64_t lx, int64_t ly, int symmetric, int P,
                       bool field = false) {
    GramLayout L;
    L.npairs = symmetric ? nx * (nx + 1) / 2 : nx * ny;
    const int64_t m = std::max<int64_t>(lx - 1, 0), n = std::max<int64_t>(ly - 1, 0);
    L.strips = (n + kWave - 1) / kWave;
    L.nprog = L.npairs * L.strips;
    L.hdr = 0;
    L.prog = align256(sizeof(WsHeader));
    L.est = align256(L.prog + sizeof(int) * (size_t)std::max<int64_t>(L.nprog, 1));
    L.front = align256(L.est + sizeof(double) * (size_t)std::max<int64_t>(L.npairs, 1));
    L.field = align256(L.front + sizeof(double) * (size_t)(L.npairs * m * P));
    // the cell-coefficient field: per pair [strips][delta_steps(m)][64]
    L.field_pair = field && m > 0 && n > 0 ? L.strips * delta_steps(m) * kWave : 0;
    L.total = align256(L.field + sizeof(double) * (size_t)(L.npairs * L.field_pair));
    return L;
}

}  // namespace

namespace sigk {
int device_error(hipError_t e) {
    std::snprintf(g_errbuf, sizeof g_errbuf, "HIP error: %s", hipGetErrorString(e));
    return SIGK_EDEVICE;
}
}  // namespace sigk

// ===================================================================== plan
struct sigk_plan {
    int P = 0, D = 0;
    int64_t d = 0, npaths = 0, npairs = 0;
    std::vector<PairDesc> desc;
    std::vector<Ticket> tickets;      // forward order (longest remaining chain first)
    std::vector<Ticket> tickets_rev;  // adjoint order (the same, top-down)
    int64_t ntk = 0;                  // ticket slots (forward and adjoint tables)
    int64_t nprog = 0;
    int64_t front_doubles = 0;        // forward frontier (one row per pair)
    int64_t snap_doubles = 0;         // adjoint: per-strip frontier snapshots
    int64_t ckpt_doubles = 0;         // adjoint: wave-state checkpoints
    int64_t pool_points = 0;
    int bwd_grid = 0;                 // workgroups the adjoint scratch is sized for
    uint64_t cells = 0;
    int64_t max_cells = 0;            // cells of the largest pair
    sigk_opts opts;
    // workspace offsets (bytes)
    size_t o_desc = 0, o_tk = 0, o_tkr = 0, o_prog = 0, o_est = 0, o_front = 0, fwd_total = 0;
    size_t o_snap = 0, o_ckpt = 0, o_lfront = 0, o_lprog = 0, o_gdx = 0, o_scr = 0,
           bwd_total = 0;
    // tables built on the device (one-call forms): every pair is laid out at
    // fixed strides for paths of up to max_len points; bucket counters of the
    // forward and adjoint ticket orders
    bool dev_tables = false;
    int64_t max_len = 0, M = 0, S_max = 0, nbk_f = 0, nbk_b = 0;
    int lag_f = 0, lag_b = 0;
    size_t o_hist = 0, o_histr = 0;
    // output slots set by sigk_plan_set_outputs (default: out[p] for pair p)
    bool custom_out = false;
};

namespace {

constexpr int kBwdMaxGrid = 2048;

// Workgroups the adjoint's recompute scratch is sized for: those of the
// adjoint launch on the current device (no more than `tickets`), or
// kBwdMaxGrid where no device can be queried (workspace sizes asked for on a
// host without one).  The launch never exceeds it.
int bwd_scratch_grid(int P, int D, int64_t tickets) {
    const int g = device_wgs(P, D, kKernelBwd);
    const int64_t n = g > 0 ? std::min(g, kBwdMaxGrid) : kBwdMaxGrid;
    return (int)std::max<int64_t>(std::min<int64_t>(n, tickets), 1);
}

void plan_layout(sigk_plan& p) {
    size_t o = align256(sizeof(WsHeader));
    p.o_desc = o;
    o = align256(o + sizeof(PairDesc) * (size_t)std::max<int64_t>(p.npairs, 1));
    p.o_tk = o;
    o = align256(o + sizeof(Ticket) * (size_t)std::max<int64_t>(p.ntk, 1));
    p.o_tkr = o;
    o = align256(o + sizeof(Ticket) * (size_t)std::max<int64_t>(p.ntk, 1));
    p.o_prog = o;
    o = align256(o + sizeof(int) * (size_t)std::max<int64_t>(p.nprog, 1));
    p.o_est = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.npairs, 1));
    p.o_front = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.front_doubles, 1));
    p.o_hist = o;
    o = align256(o + sizeof(int) * (size_t)p.nbk_f);
    p.o_histr = o;
    o = align256(o + sizeof(int) * (size_t)p.nbk_b);
    p.fwd_total = o;
    // adjoint extension
    p.o_snap = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.snap_doubles, 1));
    p.o_ckpt = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.ckpt_doubles, 1));
    p.o_lfront = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.front_doubles, 1));
    p.o_lprog = o;
    o = align256(o + sizeof(int) * (size_t)std::max<int64_t>(p.nprog, 1));
    p.o_gdx = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.pool_points * p.d, 1));
    p.o_scr = o;
    p.bwd_grid = bwd_scratch_grid(p.P, p.D, p.ntk);
    o = align256(o + sizeof(double) * (size_t)p.bwd_grid * 2 * kCkptEvery * p.P * kWave);
    p.bwd_total = o;
}

bool valid_opts(const sigk_opts* o) { return o == nullptr || (std::isfinite(o->tol) && std::isfinite(o->tail_tol)); }

// k = 1 in the output slot of every pair without cells (plans whose pairs
// write chosen slots of a shared output: the other slots are not touched).
__global__ void unit_out_kernel(const PairDesc* desc, int64_t npairs, double* out) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t p = i0; p < npairs; p += (int64_t)gridDim.x * blockDim.x)
        if (desc[p].lx < 2 || desc[p].ly < 2) out[desc[p].out_idx] = 1.0;
}

// Reset of a plan's workspace before a forward sweep: header, progress flags,
// truncation estimates and the outputs (k = 1 where a pair has no cells).
hipError_t plan_reset(const sigk_plan* plan, double* out, char* base, hipStream_t s) {
    hipError_t e = launch_reset((WsHeader*)base, (int*)(base + plan->o_prog), plan->nprog, out,
                                out && !plan->custom_out ? plan->npairs : 0,
                                (double*)(base + plan->o_est), plan->npairs, (unsigned)plan->P,
                                s);
    if (e == hipSuccess && out && plan->custom_out && plan->npairs > 0) {
        const int blocks = (int)std::min<int64_t>((plan->npairs + 255) / 256, 1024);
        hipLaunchKernelGGL(unit_out_kernel, dim3(blocks), dim3(256), 0, s,
                           (const PairDesc*)(base + plan->o_desc), plan->npairs, out);
        e = hipGetLastError();
    }
    return e;
}

// The forward sweep of a plan (after plan_reset): one persistent launch, then
// the truncation-estimate check.
int fwd_pass(const sigk_plan* plan, const double* pool, double* out, char* base, hipStream_t s) {
    if (plan->ntk == 0) return SIGK_OK;
    WsHeader* hdr = (WsHeader*)base;
    double* est = (double*)(base + plan->o_est);
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, plan->opts, plan->P, plan->d, plan->max_cells);
    a.mode = kModeTable;
    a.X = pool;
    a.Y = pool;
    a.npairs = plan->npairs;
    a.ntickets = plan->ntk;
    a.desc = (const PairDesc*)(base + plan->o_desc);
    a.tickets = (const Ticket*)(base + plan->o_tk);
    a.out = out;
    a.frontier = (double*)(base + plan->o_front);
    a.progress = (int*)(base + plan->o_prog);
    a.hdr = hdr;
    a.trunc_est = est;
    const Variant* v = find_fwd(plan->P, plan->D, plan->opts.flags, plan->opts.tile_cols);
    if (!v) return SIGK_EUNSUPPORTED;
    int grid = plan->opts.grid > 0
                   ? plan->opts.grid
                   : device_wgs(plan->P, plan->D,
                                fwd_kind(plan->P, plan->D, plan->opts.flags, plan->opts.tile_cols));
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    hipError_t e = v->fwd(a, std::max(grid, 1), s);
    if (e == hipSuccess) e = launch_finalize(hdr, est, plan->npairs, budget_of(plan->opts), s);
    if (e != hipSuccess) return device_error(e);
    return SIGK_OK;
}

sigk_opts opts_or_default(const sigk_opts* o) {
    sigk_opts r;
    sigk_default_opts(&r);
    if (o) r = *o;
    return r;
}

}  // namespace

extern "C" {

void sigk_default_opts(sigk_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->tol = 0.0;  // chosen by size at launch
    o->tail_tol = default_budget();
    o->order = 12;
}

int sigk_supported_order(int order) { return round_order(order); }

int sigk_tile_cols(int order, int64_t d, int alternative) {
    const int P = round_order(order);
    const int D = bucket_of(d, 0);
    if (!P || D == 0) return alternative ? 0 : (P ? fwd_chunk_cols(P, 0) : 0);
    return alternative ? alt_chunk_cols(P, D) : fwd_chunk_cols(P, D);
}

int sigk_device_grid(int order, int64_t d, int backward) {
    const int P = round_order(order);
    const int D = backward ? round_dim(d) : bucket_of(d, 0);
    if (!P || (backward && !D) || (!backward && !find_fwd(P, D))) return 0;
    if (backward && !find_bwd(P, D)) return 0;
    return device_wgs(P, D, backward != 0 ? kKernelBwd : kKernelFwd);
}

const char* sigk_strerror(int code) {
    switch (code) {
        case SIGK_OK: return "ok";
        case SIGK_EINVAL: return "invalid argument";
        case SIGK_EWORKSPACE: return "workspace too small";
        case SIGK_EDEVICE: return g_errbuf[0] ? g_errbuf : "HIP runtime error";
        case SIGK_EUNSUPPORTED: return "order or dimension outside the compiled range";
        default: return "unknown error";
    }
}

// ------------------------------------------------------------------ pair/gram
int sigk_gram_workspace_size(int64_t nx, int64_t ny, int64_t lx, int64_t ly, int64_t d,
                             int symmetric, const sigk_opts* o, size_t* bytes) {
    if (!bytes || nx < 0 || ny < 0 || lx < 0 || ly < 0 || d < 1 || !valid_opts(o))
        return SIGK_EINVAL;
    if (symmetric && (nx != ny || lx != ly)) return SIGK_EINVAL;
    const sigk_opts op = opts_or_default(o);
    const int P = round_order(op.order);
    const int D = bucket_of(d, op.flags);
    if (!P || !find_fwd(P, D, op.flags, op.tile_cols)) return SIGK_EUNSUPPORTED;
    *bytes = gram_layout(nx, ny, lx, ly, symmetric, P, D == 0).total;
    return SIGK_OK;
}

int sigk_gram(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t lx, int64_t ly,
              int64_t d, int symmetric, const sigk_opts* o, double* G, void* ws, size_t ws_bytes,
              void* stream) {
    if (nx < 0 || ny < 0 || lx < 0 || ly < 0 || d < 1 || !valid_opts(o)) return SIGK_EINVAL;
    if (nx * ny == 0) return SIGK_OK;
    if (!G || !ws || (lx > 0 && !X) || (ly > 0 && !Y)) return SIGK_EINVAL;
    if (symmetric && (nx != ny || lx != ly || X != Y)) return SIGK_EINVAL;
    if (lx > INT32_MAX / 2 || ly > INT32_MAX / 2 || nx * ny > INT32_MAX) return SIGK_EINVAL;
    const sigk_opts op = opts_or_default(o);
    const int P = round_order(op.order);
    const int D = bucket_of(d, op.flags);
    const Variant* v = P ? find_fwd(P, D, op.flags, op.tile_cols) : nullptr;
    if (!v) return SIGK_EUNSUPPORTED;
    const GramLayout L = gram_layout(nx, ny, lx, ly, symmetric, P, D == 0);
    if (L.nprog > INT32_MAX) return SIGK_EINVAL;  // progress slots are indexed in 32 bits
    // the field stage's grid: strips in y, pairs in z
    if (D == 0 && (L.strips > 65535 || L.npairs > 65535)) return SIGK_EUNSUPPORTED;
    if (ws_bytes < L.total) return SIGK_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    WsHeader* hdr = (WsHeader*)(base + L.hdr);
    int* prog = (int*)(base + L.prog);
    double* est = (double*)(base + L.est);
    hipError_t e = launch_reset(hdr, prog, L.nprog, G, nx * ny, est, L.npairs, (unsigned)P, s);
    if (e != hipSuccess) return device_error(e);
    if (lx < 2 || ly < 2) return SIGK_OK;
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, op, P, d, std::max<int64_t>(lx - 1, 0) * std::max<int64_t>(ly - 1, 0));
    a.mode = kModeGram;
    a.symmetric = symmetric ? 1 : 0;
    a.strips = (int)L.strips;
    a.X = X;
    a.Y = Y;
    a.nx = nx;
    a.ny = ny;
    a.lx = lx;
    a.ly = ly;
    a.npairs = L.npairs;
    a.ntickets = L.npairs * L.strips;
    a.out = G;
    a.frontier = (double*)(base + L.front);
    a.progress = prog;
    a.hdr = hdr;
    a.ckpt = nullptr;
    a.trunc_est = est;
    if (D == 0) {
        a.delta = (double*)(base + L.field);
        a.delta_pair = L.field_pair;
        e = launch_delta_gemm(a, s);
        if (e != hipSuccess) return device_error(e);
    }
    int grid = op.grid > 0 ? op.grid : device_wgs(P, D, fwd_kind(P, D, op.flags, op.tile_cols));
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    e = v->fwd(a, std::max(grid, 1), s);
    if (e == hipSuccess) e = launch_finalize(hdr, est, L.npairs, budget_of(op), s);
    if (e != hipSuccess) return device_error(e);
    return SIGK_OK;
}

int sigk_pair_workspace_size(int64_t lx, int64_t ly, int64_t d, const sigk_opts* o,
                             size_t* bytes) {
    return sigk_gram_workspace_size(1, 1, lx, ly, d, 0, o, bytes);
}

int sigk_pair(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
              const sigk_opts* o, double* k_out, void* ws, size_t ws_bytes, void* stream) {
    return sigk_gram(x, 1, y, 1, lx, ly, d, 0, o, k_out, ws, ws_bytes, stream);
}

// ------------------------------------------------------------------ plans
int sigk_plan_ragged(const int64_t* offsets, int64_t npaths, int64_t d, const int32_t* pairs,
                     int64_t npairs, const sigk_opts* o, sigk_plan** plan) {
    if (!plan) return SIGK_EINVAL;
    *plan = nullptr;
    if (!offsets || npaths < 0 || d < 1 || npairs < 0 || (npairs > 0 && !pairs) || !valid_opts(o))
        return SIGK_EINVAL;
    if (npairs > INT32_MAX / 2) return SIGK_EINVAL;
    const sigk_opts op = opts_or_default(o);
    const int P = round_order(op.order);
    const int D = round_dim(d);
    if (!P || !D || !tile_valid(P, D, op.flags, op.tile_cols)) return SIGK_EUNSUPPORTED;
    if (offsets[0] < 0) return SIGK_EINVAL;
    for (int64_t i = 0; i < npaths; ++i)
        if (offsets[i + 1] < offsets[i] || offsets[i + 1] - offsets[i] > INT32_MAX / 2)
            return SIGK_EINVAL;
    for (int64_t p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= npaths || pairs[2 * p + 1] < 0 ||
            pairs[2 * p + 1] >= npaths)
            return SIGK_EINVAL;
    sigk_plan* pl = new (std::nothrow) sigk_plan();
    if (!pl) return SIGK_EINVAL;
    pl->P = P;
    pl->D = D;
    pl->d = d;
    pl->npaths = npaths;
    pl->npairs = npairs;
    pl->opts = op;
    pl->pool_points = offsets[npaths];
    pl->desc.resize((size_t)npairs);
    std::vector<int> strips((size_t)npairs, 0);
    int64_t prog = 0, front = 0, snap = 0, ck = 0;
    int max_strips = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        PairDesc& q = pl->desc[(size_t)p];
        const int32_t px = pairs[2 * p], py = pairs[2 * p + 1];
        q.x_off = offsets[px] * d;
        q.y_off = offsets[py] * d;
        q.lx = (int32_t)(offsets[px + 1] - offsets[px]);
        q.ly = (int32_t)(offsets[py + 1] - offsets[py]);
        q.out_idx = (int32_t)p;
        q.out_idx2 = -1;
        const int64_t m = std::max(q.lx - 1, 0), n = std::max(q.ly - 1, 0);
        const int S = (m > 0 && n > 0) ? (int)((n + kWave - 1) / kWave) : 0;
        strips[(size_t)p] = S;
        max_strips = std::max(max_strips, S);
        q.prog_off = (int32_t)prog;
        prog += S;
        q.front_off = front;
        front += m * P;
        // adjoint: frontier snapshot per strip and wave-state checkpoints
        q.ckpt_off = ck;
        ck += (int64_t)S * ckpt_strip_doubles(m, P);
        q.snap_off = snap;
        snap += (int64_t)S * m * P;
        pl->cells += (uint64_t)(m * n);
        pl->max_cells = std::max<int64_t>(pl->max_cells, m * n);
    }
    if (prog > INT32_MAX) {
        delete pl;
        return SIGK_EINVAL;
    }
    pl->nprog = prog;
    pl->front_doubles = front;
    pl->snap_doubles = snap;
    pl->ckpt_doubles = ck;
    // Work order: longest remaining chain first.  The strips of a pair form a
    // chain (each starts about one chunk plus the strip height behind its
    // producer and sweeps all the pair's columns), so a ticket's remaining
    // chain is its own sweep plus one such lag per strip still to follow it.
    // Issuing long chains first keeps the deep strips of the largest pairs
    // off the end of the launch.  Within a pair the producer always ranks
    // first (its chain is one lag longer), so every wave waits on a wave that
    // is already running.  Ties: more cells first, then pair index.
    const int64_t lag_fwd = chunk_of(P, D, op.tile_cols) + kWave - 1,
                  lag_adj = chunk_cols(P) + kWave - 1;
    auto chain_order = [&](bool reverse) {
        struct Key {
            int64_t chain, cells;
            int32_t p, s;
        };
        std::vector<Key> keys;
        keys.reserve((size_t)prog);
        for (int64_t p = 0; p < npairs; ++p) {
            const PairDesc& q = pl->desc[(size_t)p];
            const int S = strips[(size_t)p];
            const int64_t m = std::max(q.lx - 1, 0), n = std::max(q.ly - 1, 0);
            for (int s = 0; s < S; ++s) {
                // forward: strips s+1.. follow; adjoint (top-down): strips ..s-1
                const int64_t after = reverse ? s : S - 1 - s;
                keys.push_back({after * (reverse ? lag_adj : lag_fwd) + m + kWave - 1, m * n,
                                (int32_t)p, s});
            }
        }
        std::stable_sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
            if (a.chain != b.chain) return a.chain > b.chain;
            if (a.cells != b.cells) return a.cells > b.cells;
            return a.p < b.p;
        });
        std::vector<Ticket> t;
        t.reserve(keys.size());
        for (const Key& k : keys) t.push_back({k.p, k.s});
        return t;
    };
    pl->tickets = chain_order(false);
    pl->tickets_rev = chain_order(true);
    pl->ntk = (int64_t)pl->tickets.size();
    plan_layout(*pl);
    *plan = pl;
    return SIGK_OK;
}

namespace {

// Adjoint ticket counter (the adjoint may run long after the checkpoint pass
// that reset the header).
__global__ void zero_tickets_kernel(WsHeader* h) {
    h->ticket2 = 0;
    h->bwd_cells = 0;
    h->bwd_flops = 0;
}

__global__ void zero_kernel(int* ip, int64_t ni, double* dp, int64_t nd) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < ni; i += stride) ip[i] = 0;
    for (int64_t i = i0; i < nd; i += stride) dp[i] = 0.0;
}

// dL/dz_p = dL/d(dz_{p-1}) - dL/d(dz_p): increments dz_p = z_{p+1} - z_p are
// stored at their first point; the last point of every path holds zero, so
// the rule needs no path boundaries.
__global__ void chain_kernel(const double* gdx, double* gpool, int64_t npts, int d) {
    const int64_t n = npts * d;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < n; i += stride) {
        const double prev = i >= d ? gdx[i - d] : 0.0;
        gpool[i] += prev - gdx[i];
    }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

}  // namespace

void sigk_plan_destroy(sigk_plan* plan) { delete plan; }

int sigk_plan_set_outputs(sigk_plan* plan, const int64_t* out_index) {
    if (!plan || (plan->npairs > 0 && !out_index) || plan->dev_tables) return SIGK_EINVAL;
    std::vector<int64_t> sorted(out_index, out_index + plan->npairs);
    std::sort(sorted.begin(), sorted.end());
    for (size_t i = 0; i < sorted.size(); ++i)
        if (sorted[i] < 0 || sorted[i] > INT32_MAX / 2 || (i > 0 && sorted[i] == sorted[i - 1]))
            return SIGK_EINVAL;
    for (int64_t p = 0; p < plan->npairs; ++p) {
        plan->desc[(size_t)p].out_idx = (int32_t)out_index[p];
        plan->desc[(size_t)p].out_idx2 = -1;
    }
    plan->custom_out = true;
    return SIGK_OK;
}

size_t sigk_plan_estimates_offset(const sigk_plan* plan) { return plan ? plan->o_est : 0; }

int sigk_plan_tickets(const sigk_plan* plan, int adjoint, int32_t* out, int64_t cap,
                      int64_t* n_out) {
    if (!plan || !n_out || plan->dev_tables) return SIGK_EINVAL;
    const std::vector<Ticket>& t = adjoint ? plan->tickets_rev : plan->tickets;
    *n_out = (int64_t)t.size();
    if (!out) return SIGK_OK;
    if (cap < (int64_t)t.size()) return SIGK_EINVAL;
    for (size_t i = 0; i < t.size(); ++i) {
        out[2 * i] = t[i].pair;
        out[2 * i + 1] = t[i].strip;
    }
    return SIGK_OK;
}

size_t sigk_plan_workspace_size(const sigk_plan* plan) { return plan ? plan->fwd_total : 0; }
size_t sigk_plan_backward_workspace_size(const sigk_plan* plan) {
    return plan ? plan->bwd_total : 0;
}
uint64_t sigk_plan_cells(const sigk_plan* plan) { return plan ? plan->cells : 0; }

int sigk_plan_upload(const sigk_plan* plan, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !ws) return SIGK_EINVAL;
    if (ws_bytes < plan->fwd_total) return SIGK_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    hipError_t e = hipSuccess;
    if (!plan->desc.empty())
        e = hipMemcpyAsync(base + plan->o_desc, plan->desc.data(),
                           plan->desc.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !plan->tickets.empty())
        e = hipMemcpyAsync(base + plan->o_tk, plan->tickets.data(),
                           plan->tickets.size() * sizeof(Ticket), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !plan->tickets_rev.empty())
        e = hipMemcpyAsync(base + plan->o_tkr, plan->tickets_rev.data(),
                           plan->tickets_rev.size() * sizeof(Ticket), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_error(e);
    return SIGK_OK;
}

int sigk_plan_run(const sigk_plan* plan, const double* pool, double* out, void* ws,
                  size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !out))) return SIGK_EINVAL;
    if (ws_bytes < plan->fwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0) return SIGK_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = plan_reset(plan, out, (char*)ws, s);
    if (e != hipSuccess) return device_error(e);
    return fwd_pass(plan, pool, out, (char*)ws, s);
}

// ------------------------------------------------------------------ status
int sigk_read_counters(const void* ws, sigk_counters* out, void* stream) {
    if (!ws || !out) return SIGK_EINVAL;
    WsHeader h;
    hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return device_error(e);
    out->cells = h.cells;
    out->flops = h.flops;
    out->status = h.status;
    out->order = h.order;
    out->trunc_est = h.trunc_max;
    out->bwd_cells = h.bwd_cells;
    out->bwd_flops = h.bwd_flops;
    return SIGK_OK;
}

int sigk_read_status(const void* ws, uint32_t* status_bits, void* stream) {
    if (!status_bits) return SIGK_EINVAL;
    sigk_counters c;
    int rc = sigk_read_counters(ws, &c, stream);
    if (!rc) *status_bits = c.status;
    return rc;
}

}  // extern "C"

namespace {

// Checkpoint pass: the forward sweep of every strip (64-row strips), keeping
// the frontier row each strip reads, the wave state every kCkptEvery steps and
// the depth of every chunk; writes the kernel values to out when out != null.
int checkpoint_pass(const sigk_plan* plan, const Variant* v, const double* pool, double* out,
                    char* base, hipStream_t s, bool reset = true) {
    WsHeader* hdr = (WsHeader*)base;
    int* prog = (int*)(base + plan->o_prog);
    double* est = (double*)(base + plan->o_est);
    hipError_t e = reset ? plan_reset(plan, out, base, s) : hipSuccess;
    if (e != hipSuccess) return device_error(e);
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, plan->opts, plan->P, plan->d, plan->max_cells);
    a.mode = kModeTable;
    a.X = pool;
    a.Y = pool;
    a.npairs = plan->npairs;
    a.ntickets = plan->ntk;
    a.desc = (const PairDesc*)(base + plan->o_desc);
    a.tickets = (const Ticket*)(base + plan->o_tk);
    a.out = out;
    a.frontier = (double*)(base + plan->o_snap);
    a.progress = prog;
    a.hdr = hdr;
    a.ckpt = (double*)(base + plan->o_ckpt);
    a.trunc_est = est;
    int grid = plan->opts.grid > 0 ? plan->opts.grid : device_wgs(plan->P, plan->D, kKernelCkpt);
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    e = v->ckpt(a, std::max(grid, 1), s);
    if (e == hipSuccess) e = launch_finalize(hdr, est, plan->npairs, budget_of(plan->opts), s);
    if (e != hipSuccess) return device_error(e);
    return SIGK_OK;
}

// Adjoint pass over the checkpoints in base, then the chain to the points.
int adjoint_pass(const sigk_plan* plan, const Variant* v, const double* pool,
                 const double* grad_out, double* grad_pool, char* base, hipStream_t s) {
    WsHeader* hdr = (WsHeader*)base;
    int* lprog = (int*)(base + plan->o_lprog);
    double* gdx = (double*)(base + plan->o_gdx);
    const int64_t ngdx = plan->pool_points * plan->d;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(std::max(plan->nprog, ngdx))), dim3(256), 0,
                       s, lprog, plan->nprog, gdx, ngdx);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    hipLaunchKernelGGL(zero_tickets_kernel, dim3(1), dim3(1), 0, s, hdr);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    BwdArgs b;
    std::memset(&b, 0, sizeof b);
    fill_common(b.f, plan->opts, plan->P, plan->d, plan->max_cells);
    b.f.mode = kModeTable;
    b.f.X = pool;
    b.f.Y = pool;
    b.f.npairs = plan->npairs;
    b.f.desc = (const PairDesc*)(base + plan->o_desc);
    b.f.hdr = hdr;
    b.tickets = (const Ticket*)(base + plan->o_tkr);
    b.ntickets = plan->ntk;
    b.grad_out = grad_out;
    b.snap = (double*)(base + plan->o_snap);
    b.ckpt = (double*)(base + plan->o_ckpt);
    b.lam_front = (double*)(base + plan->o_lfront);
    b.lam_prog = lprog;
    b.gdx = gdx;
    b.scratch = (double*)(base + plan->o_scr);
    int bgrid = plan->opts.grid > 0 ? plan->opts.grid : device_wgs(plan->P, plan->D, kKernelBwd);
    bgrid = (int)std::min<int64_t>(std::min(bgrid, plan->bwd_grid), b.ntickets);
    e = v->bwd(b, std::max(bgrid, 1), s);
    if (e != hipSuccess) return device_error(e);
    hipLaunchKernelGGL(chain_kernel, dim3(blocks_for(ngdx)), dim3(256), 0, s, gdx, grad_pool,
                       plan->pool_points, (int)plan->d);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    return SIGK_OK;
}

}  // namespace

extern "C" {

int sigk_plan_run_checkpointed(const sigk_plan* plan, const double* pool, double* out, void* ws,
                               size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !out))) return SIGK_EINVAL;
    if (ws_bytes < plan->bwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0) return SIGK_OK;
    hipStream_t s = (hipStream_t)stream;
    if (plan->ntk == 0) {
        hipError_t e = launch_reset((WsHeader*)ws, (int*)((char*)ws + plan->o_prog), plan->nprog,
                                    out, plan->npairs, (double*)((char*)ws + plan->o_est),
                                    plan->npairs, (unsigned)plan->P, s);
        return e == hipSuccess ? SIGK_OK : device_error(e);
    }
    const Variant* v = find_bwd(plan->P, plan->D, plan->opts.flags);
    if (!v) return SIGK_EUNSUPPORTED;
    return checkpoint_pass(plan, v, pool, out, (char*)ws, s);
}

int sigk_plan_backward_checkpointed(const sigk_plan* plan, const double* pool,
                                    const double* grad_out, double* grad_pool, void* ws,
                                    size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !grad_out || !grad_pool)))
        return SIGK_EINVAL;
    if (ws_bytes < plan->bwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0 || plan->ntk == 0) return SIGK_OK;
    const Variant* v = find_bwd(plan->P, plan->D, plan->opts.flags);
    if (!v) return SIGK_EUNSUPPORTED;
    return adjoint_pass(plan, v, pool, grad_out, grad_pool, (char*)ws, (hipStream_t)stream);
}

int sigk_plan_backward(const sigk_plan* plan, const double* pool, const double* grad_out,
                       double* grad_pool, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !grad_out || !grad_pool)))
        return SIGK_EINVAL;
    if (ws_bytes < plan->bwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0 || plan->ntk == 0) return SIGK_OK;
    const Variant* v = find_bwd(plan->P, plan->D, plan->opts.flags);
    if (!v) return SIGK_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    int rc = checkpoint_pass(plan, v, pool, nullptr, (char*)ws, s);
    if (rc) return rc;
    return adjoint_pass(plan, v, pool, grad_out, grad_pool, (char*)ws, s);
}

}  // extern "C"

// ===================================================================== device tables
//
// One-call ragged batches (sigk_gram_ragged, sigk_backward) whose offsets and
// pair table are device arrays: the tables the kernels need are built on the
// device by a few small kernels, so the calls are asynchronous and can be
// captured in a HIP graph.  Every pair is laid out at fixed strides for paths
// of up to max_len points.  Tickets are ordered by a counting sort on the
// strip's remaining chain (its own sweep plus one start lag per strip still to
// follow it in its pair), in buckets one lag wide: a producer's chain is one
// lag longer than its consumer's, so it always lands in an earlier bucket and
// takes a smaller ticket (no wave ever waits on a ticket not yet claimed).
namespace {

__global__ void dt_desc_kernel(const int64_t* offsets, int64_t npaths, const int32_t* pairs,
                               int64_t npairs, int64_t max_len, int64_t pool_points, int64_t d,
                               int64_t front_stride, int64_t snap_stride, int64_t ckpt_stride,
                               int64_t S_max, PairDesc* desc, double* out, WsHeader* h) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = i0; p < npairs; p += stride) {
        const int32_t px = pairs[2 * p], py = pairs[2 * p + 1];
        bool ok = px >= 0 && px < npaths && py >= 0 && py < npaths;
        int64_t x0 = 0, x1 = 0, y0 = 0, y1 = 0;
        if (ok) {
            x0 = offsets[px];
            x1 = offsets[px + 1];
            y0 = offsets[py];
            y1 = offsets[py + 1];
            ok = x0 >= 0 && x0 <= x1 && x1 - x0 <= max_len && x1 <= pool_points && y0 >= 0 &&
                 y0 <= y1 && y1 - y0 <= max_len && y1 <= pool_points;
        }
        PairDesc q;
        q.x_off = ok ? x0 * d : 0;
        q.y_off = ok ? y0 * d : 0;
        q.lx = ok ? (int32_t)(x1 - x0) : 0;
        q.ly = ok ? (int32_t)(y1 - y0) : 0;
        q.front_off = p * front_stride;
        q.snap_off = p * snap_stride;
        q.ckpt_off = p * ckpt_stride;
        q.prog_off = (int32_t)(p * S_max);
        q.out_idx = (int32_t)p;
        q.out_idx2 = -1;
        q.pad = 0;
        desc[p] = q;
        if (!ok) {
            if (out) out[p] = __builtin_nan("");
            atomicOr(&h->status, SIGK_ERR_TABLE);
        }
    }
}

__global__ void dt_clear_kernel(Ticket* tk, Ticket* tkr, int64_t nt, int* hist, int64_t nh,
                                int* histr, int64_t nhr) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < nt; i += stride) {
        tk[i] = Ticket{-1, -1};
        if (tkr) tkr[i] = Ticket{-1, -1};
    }
    for (int64_t i = i0; i < nh; i += stride) hist[i] = 0;
    for (int64_t i = i0; i < nhr; i += stride) histr[i] = 0;
}

// Bucket (ascending = issued first) of strip s of a pair with m columns and S
// strips: forward chains run upwards (strips s+1.. follow), adjoint chains
// downwards (strips ..s-1 follow).
__device__ __forceinline__ int64_t dt_bucket(int64_t m, int64_t S, int64_t s, int lag,
                                             int64_t nbk, bool adjoint) {
    const int64_t after = adjoint ? s : S - 1 - s;
    return nbk - 1 - (after * lag + m + kWave - 1) / lag;
}

// Counting sort of the tickets: count (scatter == false) or place.
__global__ void dt_tickets_kernel(const PairDesc* desc, int64_t S_max, int64_t nt, int lag_f,
                                  int64_t nbf, int* hist, Ticket* tk, int lag_b, int64_t nbb,
                                  int* histr, Ticket* tkr, int scatter) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = i0; t < nt; t += stride) {
        const int64_t p = t / S_max, s = t % S_max;
        const PairDesc q = desc[p];
        const int64_t m = q.lx > 1 ? q.lx - 1 : 0, n = q.ly > 1 ? q.ly - 1 : 0;
        const int64_t S = (m > 0 && n > 0) ? (n + kWave - 1) / kWave : 0;
        if (s >= S) continue;
        const int64_t bf = dt_bucket(m, S, s, lag_f, nbf, false);
        if (!scatter) {
            atomicAdd(&hist[bf], 1);
        } else {
            const int slot = atomicAdd(&hist[bf], 1);
            tk[slot] = Ticket{(int32_t)p, (int32_t)s};
        }
        if (histr) {
            const int64_t bb = dt_bucket(m, S, s, lag_b, nbb, true);
            if (!scatter) {
                atomicAdd(&histr[bb], 1);
            } else {
                const int slot = atomicAdd(&histr[bb], 1);
                tkr[slot] = Ticket{(int32_t)p, (int32_t)s};
            }
        }
    }
}

// Exclusive prefix sum in place, one block of 1024 threads (bucket counts
// -> first ticket of each bucket); histr may be null.
__global__ void dt_scan_kernel(int* hist, int64_t nh, int* histr, int64_t nhr) {
    __shared__ int sv[1024];
    __shared__ int carry;
    for (int which = 0; which < 2; ++which) {
        int* a = which ? histr : hist;
        const int64_t n = which ? nhr : nh;
        if (!a) continue;
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int64_t base = 0; base < n; base += 1024) {
            const int64_t i = base + threadIdx.x;
            const int v = i < n ? a[i] : 0;
            sv[threadIdx.x] = v;
            __syncthreads();
            for (int o = 1; o < 1024; o <<= 1) {
                const int w = (int)threadIdx.x >= o ? sv[threadIdx.x - o] : 0;
                __syncthreads();
                sv[threadIdx.x] += w;
                __syncthreads();
            }
            if (i < n) a[i] = carry + sv[threadIdx.x] - v;
            __syncthreads();
            if (threadIdx.x == 1023) carry += sv[1023];
            __syncthreads();
        }
    }
}

// Layout of a one-call batch (host only): bounds from the scalar arguments.
int dev_plan(int64_t npaths, int64_t npairs, int64_t max_len, int64_t pool_points, int64_t d,
             const sigk_opts* o, bool backward, sigk_plan& pl) {
    if (npaths < 0 || npairs < 0 || max_len < 0 || pool_points < 0 || d < 1 || !valid_opts(o))
        return SIGK_EINVAL;
    if (max_len > INT32_MAX / 2 || npairs > INT32_MAX / 2) return SIGK_EINVAL;
    const sigk_opts op = opts_or_default(o);
    const int P = round_order(op.order);
    const int D = round_dim(d);
    if (!P || !D || !tile_valid(P, D, op.flags, op.tile_cols)) return SIGK_EUNSUPPORTED;
    if (backward && !find_bwd(P, D, op.flags)) return SIGK_EUNSUPPORTED;
    pl.P = P;
    pl.D = D;
    pl.d = d;
    pl.npaths = npaths;
    pl.npairs = npairs;
    pl.opts = op;
    pl.pool_points = pool_points;
    pl.dev_tables = true;
    pl.max_len = max_len;
    pl.M = std::max<int64_t>(max_len - 1, 0);
    pl.S_max = (pl.M + kWave - 1) / kWave;
    pl.ntk = npairs * pl.S_max;
    if (pl.ntk > INT32_MAX) return SIGK_EINVAL;  // tickets and progress slots are 32-bit
    pl.nprog = pl.ntk;
    pl.max_cells = pl.M * pl.M;  // the default Neumann tolerance, for the largest pair
    pl.front_doubles = npairs * pl.M * P;
    pl.snap_doubles = backward ? pl.ntk * pl.M * P : 0;
    pl.ckpt_doubles = backward ? pl.ntk * ckpt_strip_doubles(pl.M, P) : 0;
    pl.lag_f = chunk_of(P, D, op.tile_cols) + kWave - 1;
    pl.lag_b = chunk_cols(P) + kWave - 1;
    const int64_t chain_max = std::max<int64_t>(pl.S_max - 1, 0) * std::max(pl.lag_f, pl.lag_b) +
                              pl.M + kWave - 1;
    pl.nbk_f = chain_max / pl.lag_f + 1;
    pl.nbk_b = backward ? chain_max / pl.lag_b + 1 : 0;
    plan_layout(pl);
    if (!backward) pl.bwd_total = pl.fwd_total;
    return SIGK_OK;
}

int blocks_of(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

// Reset, then the device tables (descriptors, ticket orders) of a one-call
// batch.  out: kernel values (NaN for invalid pairs) or null.
int dev_tables(const sigk_plan& pl, const int64_t* offsets, const int32_t* pairs, double* out,
               char* base, bool backward, hipStream_t s) {
    hipError_t e = plan_reset(&pl, out, base, s);
    if (e != hipSuccess) return device_error(e);
    PairDesc* desc = (PairDesc*)(base + pl.o_desc);
    Ticket* tk = (Ticket*)(base + pl.o_tk);
    Ticket* tkr = backward ? (Ticket*)(base + pl.o_tkr) : nullptr;
    int* hist = (int*)(base + pl.o_hist);
    int* histr = backward ? (int*)(base + pl.o_histr) : nullptr;
    const int64_t ckpt_stride = pl.S_max * ckpt_strip_doubles(pl.M, pl.P);
    hipLaunchKernelGGL(dt_desc_kernel, dim3(blocks_of(pl.npairs)), dim3(256), 0, s, offsets,
                       pl.npaths, pairs, pl.npairs, pl.max_len, pl.pool_points, pl.d,
                       pl.M * pl.P, pl.S_max * pl.M * pl.P, ckpt_stride, pl.S_max, desc, out,
                       (WsHeader*)base);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    const int64_t nclear = std::max(pl.ntk, std::max(pl.nbk_f, pl.nbk_b));
    hipLaunchKernelGGL(dt_clear_kernel, dim3(blocks_of(nclear)), dim3(256), 0, s, tk, tkr, pl.ntk,
                       hist, pl.nbk_f, histr, pl.nbk_b);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    for (int scatter = 0; scatter < 2; ++scatter) {
        hipLaunchKernelGGL(dt_tickets_kernel, dim3(blocks_of(pl.ntk)), dim3(256), 0, s, desc,
                           pl.S_max, pl.ntk, pl.lag_f, pl.nbk_f, hist, tk, pl.lag_b, pl.nbk_b,
                           histr, tkr, scatter);
        if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
        if (!scatter) {
            hipLaunchKernelGGL(dt_scan_kernel, dim3(1), dim3(1024), 0, s, hist, pl.nbk_f, histr,
                               pl.nbk_b);
            if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
        }
    }
    return SIGK_OK;
}

}  // namespace

extern "C" {

int sigk_gram_ragged_workspace_size(int64_t npaths, int64_t npairs, int64_t max_len,
                                    int64_t pool_points, int64_t d, const sigk_opts* o,
                                    size_t* bytes) {
    if (!bytes) return SIGK_EINVAL;
    sigk_plan pl;
    const int rc = dev_plan(npaths, npairs, max_len, pool_points, d, o, false, pl);
    if (rc) return rc;
    *bytes = pl.fwd_total;
    return SIGK_OK;
}

int sigk_gram_ragged(const double* pool, int64_t pool_points, const int64_t* offsets,
                     int64_t npaths, int64_t d, const int32_t* pairs, int64_t npairs,
                     int64_t max_len, const sigk_opts* o, double* out, void* ws, size_t ws_bytes,
                     void* stream) {
    sigk_plan pl;
    int rc = dev_plan(npaths, npairs, max_len, pool_points, d, o, false, pl);
    if (rc) return rc;
    if (npairs == 0) return SIGK_OK;
    if (!pool || !offsets || !pairs || !out || !ws) return SIGK_EINVAL;
    if (ws_bytes < pl.fwd_total) return SIGK_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    rc = dev_tables(pl, offsets, pairs, out, (char*)ws, false, s);
    if (rc) return rc;
    return fwd_pass(&pl, pool, out, (char*)ws, s);
}

int sigk_ragged_tables(int64_t npaths, int64_t npairs, int64_t max_len, int64_t pool_points,
                       int64_t d, const sigk_opts* o, int adjoint, size_t* tickets_offset,
                       int64_t* ntickets) {
    if (!tickets_offset || !ntickets) return SIGK_EINVAL;
    sigk_plan pl;
    const int rc = dev_plan(npaths, npairs, max_len, pool_points, d, o, adjoint != 0, pl);
    if (rc) return rc;
    *tickets_offset = adjoint ? pl.o_tkr : pl.o_tk;
    *ntickets = pl.ntk;
    return SIGK_OK;
}

int sigk_backward_workspace_size(int64_t npaths, int64_t npairs, int64_t max_len,
                                 int64_t pool_points, int64_t d, const sigk_opts* o,
                                 size_t* bytes) {
    if (!bytes) return SIGK_EINVAL;
    sigk_plan pl;
    const int rc = dev_plan(npaths, npairs, max_len, pool_points, d, o, true, pl);
    if (rc) return rc;
    *bytes = pl.bwd_total;
    return SIGK_OK;
}

int sigk_backward(const double* pool, int64_t pool_points, const int64_t* offsets,
                  int64_t npaths, int64_t d, const int32_t* pairs, int64_t npairs,
                  int64_t max_len, const double* grad_out, const sigk_opts* o, double* grad_pool,
                  void* ws, size_t ws_bytes, void* stream) {
    sigk_plan pl;
    int rc = dev_plan(npaths, npairs, max_len, pool_points, d, o, true, pl);
    if (rc) return rc;
    if (npairs == 0) return SIGK_OK;
    if (!pool || !offsets || !pairs || !grad_out || !grad_pool || !ws) return SIGK_EINVAL;
    if (ws_bytes < pl.bwd_total) return SIGK_EWORKSPACE;
    const Variant* v = find_bwd(pl.P, pl.D);
    hipStream_t s = (hipStream_t)stream;
    rc = dev_tables(pl, offsets, pairs, nullptr, (char*)ws, true, s);
    if (!rc) rc = checkpoint_pass(&pl, v, pool, nullptr, (char*)ws, s, false);
    if (!rc) rc = adjoint_pass(&pl, v, pool, grad_out, grad_pool, (char*)ws, s);
    return rc;
}

}  // extern "C"

// ============================================================ long pair gradient
namespace {

struct LongLayout {
    int P = 0, D = 0;
    int64_t lx = 0, ly = 0, d = 0, m = 0, n = 0;
    int rb = 0, cb = 0, ni = 0, nj = 0, kb = 0, nslots = 0, S = 0, bwd_grid = 0;
    int64_t slot_snap = 0, slot_ckpt = 0;
    int slot_prog = 0;
    size_t o_est = 0, o_prog = 0, o_front = 0, o_hline = 0, o_vline = 0, o_snap = 0, o_ckpt = 0,
           o_bprog = 0, o_lprog = 0, o_lamh = 0, o_lamv = 0, o_gdx = 0, o_scr = 0, total = 0;
};

// Square blocks of side b cost about 16 m n P / b bytes of lines and, per
// anti-diagonal, min(m, n) b (9P/8) bytes of checkpoints and snapshots; the
// sum is least near b = sqrt(14.2 max(m, n)).  Rows are rounded to whole
// strips.
int auto_block(int64_t m, int64_t n) {
    const double b = std::sqrt(14.2 * (double)std::max(m, n));
    const int r = (int)std::lround(b / 64.0) * 64;
    return std::min(std::max(r, 64), 16384);
}

int long_layout(int64_t lx, int64_t ly, int64_t d, int64_t brows, int64_t bcols,
                const sigk_opts& op, LongLayout& L) {
    if (lx < 0 || ly < 0 || d < 1 || brows < 0 || bcols < 0 || (brows % kWave) != 0)
        return SIGK_EINVAL;
    if (lx > INT32_MAX / 2 || ly > INT32_MAX / 2 || brows > INT32_MAX / 2 ||
        bcols > INT32_MAX / 2)
        return SIGK_EINVAL;
    L.P = round_order(op.order);
    L.D = round_dim(d);
    if (!L.P || !L.D || !find_bwd(L.P, L.D, op.flags)) return SIGK_EUNSUPPORTED;
    const int P = L.P;
    L.lx = lx;
    L.ly = ly;
    L.d = d;
    L.m = std::max<int64_t>(lx - 1, 0);
    L.n = std::max<int64_t>(ly - 1, 0);
    const int64_t m = L.m, n = L.n;
    const int64_t n64 = std::max<int64_t>((n + kWave - 1) / kWave * kWave, kWave);
    L.rb = (int)std::min<int64_t>(brows ? brows : auto_block(m, n), n64);
    L.cb = (int)std::max<int64_t>(std::min<int64_t>(bcols ? bcols : L.rb, std::max<int64_t>(m, 1)), 1);
    L.ni = (int)std::max<int64_t>((n + L.rb - 1) / L.rb, 1);
    L.nj = (int)std::max<int64_t>((m + L.cb - 1) / L.cb, 1);
    L.kb = L.rb / kWave;
    L.nslots = std::min(L.ni, L.nj);
    L.S = (int)((n + kWave - 1) / kWave);
    L.slot_snap = (int64_t)L.kb * L.cb * P;
    L.slot_ckpt = (int64_t)L.kb * ckpt_strip_doubles(L.cb, P);
    L.slot_prog = L.kb + 2;
    if ((int64_t)L.nslots * L.kb > INT32_MAX || (int64_t)L.nslots * L.slot_prog > INT32_MAX)
        return SIGK_EINVAL;
    size_t o = align256(sizeof(WsHeader));
    auto take = [&o](size_t& at, size_t bytes) {
        at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
    };
    take(L.o_est, sizeof(double));
    take(L.o_prog, sizeof(int) * (size_t)L.S);
    take(L.o_front, sizeof(double) * (size_t)(m * P));
    take(L.o_hline, sizeof(double) * (size_t)((L.ni - 1) * m * P));
    take(L.o_vline, sizeof(double) * (size_t)((L.nj - 1) * n * P));
    take(L.o_snap, sizeof(double) * (size_t)(L.nslots * L.slot_snap));
    take(L.o_ckpt, sizeof(double) * (size_t)(L.nslots * L.slot_ckpt));
    take(L.o_bprog, sizeof(int) * (size_t)L.nslots * L.slot_prog);
    take(L.o_lprog, sizeof(int) * (size_t)L.nslots * L.slot_prog);
    take(L.o_lamh, sizeof(double) * (size_t)(m * P));
    take(L.o_lamv, sizeof(double) * (size_t)(n * P));
    take(L.o_gdx, sizeof(double) * (size_t)((lx + ly) * d));
    L.bwd_grid = bwd_scratch_grid(P, L.D, (int64_t)L.nslots * L.kb);
    take(L.o_scr, sizeof(double) * (size_t)L.bwd_grid * 2 * kCkptEvery * P * kWave);
    L.total = o;
    return SIGK_OK;
}

// Before the blocks of one anti-diagonal: both ticket counters, and per slot
// the progress counters of the checkpointing sweep and of the adjoint, each
// between two sentinels that count as complete (strip 0 reads a bottom line,
// the top strip a cotangent row, with no producer in the launch).
__global__ void blk_diag_reset_kernel(WsHeader* h, int* bprog, int* lprog, int n, int per) {
    const int i0 = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 == 0) {
        h->ticket = 0;
        h->ticket2 = 0;
    }
    for (int i = i0; i < n; i += (int)(gridDim.x * blockDim.x)) {
        const int k = i % per;
        const int v = (k == 0 || k == per - 1) ? INT32_MAX : 0;
        bprog[i] = v;
        lprog[i] = v;
    }
}

// dL/dz from dL/d(dz) for the two paths stored back to back in gdx (x's
// increments at its points 0..lx-2, y's after lx points), accumulated.
__global__ void chain2_kernel(const double* gdx, int64_t lx, int64_t ly, int d, double* gx,
                              double* gy) {
    const int64_t nx = lx * d, n = (lx + ly) * d;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < n; i += stride) {
        const bool isx = i < nx;
        const int64_t j = isx ? i : i - nx;  // index within the path
        const double prev = j >= d ? gdx[i - d] : 0.0;
        const double last = (isx ? j >= nx - d : j >= n - nx - d) ? 0.0 : gdx[i];
        double* g = isx ? gx : gy;
        g[j] += prev - last;
    }
}

}  // namespace

extern "C" {

int sigk_pair_backward_workspace_size(int64_t lx, int64_t ly, int64_t d, int64_t block_rows,
                                      int64_t block_cols, const sigk_opts* o, size_t* bytes) {
    if (!bytes || !valid_opts(o)) return SIGK_EINVAL;
    LongLayout L;
    const int rc = long_layout(lx, ly, d, block_rows, block_cols, opts_or_default(o), L);
    if (rc) return rc;
    *bytes = L.total;
    return SIGK_OK;
}

int sigk_pair_backward_blocks(int64_t lx, int64_t ly, int64_t d, int64_t block_rows,
                              int64_t block_cols, const sigk_opts* o, int64_t* rows_out,
                              int64_t* cols_out) {
    if (!rows_out || !cols_out || !valid_opts(o)) return SIGK_EINVAL;
    LongLayout L;
    const int rc = long_layout(lx, ly, d, block_rows, block_cols, opts_or_default(o), L);
    if (rc) return rc;
    *rows_out = L.rb;
    *cols_out = L.cb;
    return SIGK_OK;
}

int sigk_pair_backward(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                       const double* grad_out, int64_t block_rows, int64_t block_cols,
                       const sigk_opts* o, double* k_out, double* grad_x, double* grad_y,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!valid_opts(o)) return SIGK_EINVAL;
    const sigk_opts op = opts_or_default(o);
    LongLayout L;
    int rc = long_layout(lx, ly, d, block_rows, block_cols, op, L);
    if (rc) return rc;
    if (!ws || !grad_out || (lx > 0 && (!x || !grad_x)) || (ly > 0 && (!y || !grad_y)))
        return SIGK_EINVAL;
    if (ws_bytes < L.total) return SIGK_EWORKSPACE;
    const Variant* v = find_bwd(L.P, L.D);
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    WsHeader* hdr = (WsHeader*)base;
    int* prog = (int*)(base + L.o_prog);
    double* est = (double*)(base + L.o_est);
    hipError_t e = launch_reset(hdr, prog, L.S, k_out, k_out ? 1 : 0, est, 1, (unsigned)L.P, s);
    if (e != hipSuccess) return device_error(e);
    if (L.m == 0 || L.n == 0) return SIGK_OK;  // k = 1 for every path: no gradient
    double* gdx = (double*)(base + L.o_gdx);
    const int64_t ngdx = (lx + ly) * d;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(ngdx)), dim3(256), 0, s, nullptr, 0, gdx,
                       ngdx);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);

    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, op, L.P, d, L.m * L.n);
    a.X = x;
    a.Y = y;
    a.npairs = 1;
    a.hdr = hdr;
    BlockGeo& k = a.blk;
    k.m = L.m;
    k.n = L.n;
    k.rb = L.rb;
    k.cb = L.cb;
    k.ni = L.ni;
    k.nj = L.nj;
    k.kb = L.kb;
    k.hline = (double*)(base + L.o_hline);
    k.vline = (double*)(base + L.o_vline);
    k.slot_snap = L.slot_snap;
    k.slot_ckpt = L.slot_ckpt;
    k.slot_prog = L.slot_prog;
    k.y_gdx = lx * d;
    const int cgrid = std::max(device_wgs(L.P, L.D, kKernelCkpt), 1);
    const int bgrid = L.bwd_grid;

    // 1. the whole pair once: k(x, y), its truncation estimate and the lines
    a.mode = kModeLines;
    a.ntickets = L.S;
    a.out = k_out;
    a.frontier = (double*)(base + L.o_front);
    a.progress = prog;
    a.trunc_est = est;
    const int lgrid = std::max(device_wgs(L.P, L.D, kKernelLines), 1);
    e = v->fwd(a, (int)std::min<int64_t>(lgrid, L.S), s);
    if (e == hipSuccess) e = launch_finalize(hdr, est, 1, budget_of(op), s);
    if (e != hipSuccess) return device_error(e);

    // 2. block anti-diagonals from the top-right corner down: checkpoints of
    // the blocks, then their adjoint
    a.mode = kModeBlock;
    a.out = nullptr;
    a.trunc_est = nullptr;
    a.frontier = (double*)(base + L.o_snap);
    a.ckpt = (double*)(base + L.o_ckpt);
    a.progress = (int*)(base + L.o_bprog);
    BwdArgs b;
    std::memset(&b, 0, sizeof b);
    b.grad_out = grad_out;
    b.snap = a.frontier;
    b.ckpt = a.ckpt;
    b.lam_front = (double*)(base + L.o_lamh);
    b.lam_v = (double*)(base + L.o_lamv);
    b.lam_prog = (int*)(base + L.o_lprog);
    b.gdx = gdx;
    b.scratch = (double*)(base + L.o_scr);
    for (int diag = L.ni + L.nj - 2; diag >= 0; --diag) {
        const int j_lo = std::max(0, diag - (L.ni - 1));
        const int j_hi = std::min(diag, L.nj - 1);
        k.diag = diag;
        k.j_lo = j_lo;
        k.nb = j_hi - j_lo + 1;
        const int nprog = k.nb * L.slot_prog;
        hipLaunchKernelGGL(blk_diag_reset_kernel, dim3((nprog + 255) / 256), dim3(256), 0, s, hdr,
                           a.progress, b.lam_prog, nprog, L.slot_prog);
        if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
        a.ntickets = (int64_t)k.nb * L.kb;
        e = v->ckpt(a, (int)std::min<int64_t>(cgrid, a.ntickets), s);
        if (e != hipSuccess) return device_error(e);
        b.f = a;
        b.ntickets = a.ntickets;
        e = v->bwd(b, (int)std::min<int64_t>(bgrid, b.ntickets), s);
        if (e != hipSuccess) return device_error(e);
    }
    hipLaunchKernelGGL(chain2_kernel, dim3(blocks_for(ngdx)), dim3(256), 0, s, gdx, lx, ly,
                       (int)d, grad_x, grad_y);
    if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
    return SIGK_OK;
}

}  // extern "C"
