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
#define SIGK_V_BWD(P, D) {P, D, nullptr, nullptr, launch_ckpt_##P##_##D, launch_bwd_##P##_##D, occupancy_ckpt_##P##_##D, occupancy_bwd_##P##_##D},
const Variant kBwdTable[] = {SIGK_BWD_VARIANTS(SIGK_V_BWD)};
#undef SIGK_V_BWD

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

const Variant* find_fwd(int P, int D) {
    for (const Variant& v : kFwdTable)
        if (v.P == P && v.D == D) return &v;
    return nullptr;
}
const Variant* find_bwd(int P, int D) {
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
enum { kKernelFwd = 0, kKernelBwd = 1, kKernelCkpt = 2 };

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
    if (kind == kKernelFwd) {
        const Variant* v = find_fwd(P, D);
        occ = v ? v->occ_fwd() : 0;
    } else {
        const Variant* v = find_bwd(P, D);
        occ = v ? (kind == kKernelBwd ? v->occ_bwd() : v->occ_ckpt()) : 0;
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
    a.tail_tol = o.tail_tol > 0 ? o.tail_tol : std::ldexp(1.0, -50);
    a.d = (int)d;
    a.watchdog_ticks = 2000000000LL;  // 20 s of the 100 MHz counter
    (void)P;
}

__global__ void reset_kernel(WsHeader* h, int* prog, int64_t nprog, double* out, int64_t nout,
                             unsigned order) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i0 == 0) {
        h->status = 0;
        h->ticket = 0;
        h->ticket2 = 0;
        h->cells = 0;
        h->flops = 0;
        h->order = order;
    }
    for (int64_t i = i0; i < nprog; i += stride) prog[i] = 0;
    // pairs without cells keep k = 1 (K = 1 on the axes)
    for (int64_t i = i0; i < nout; i += stride) out[i] = 1.0;
}

hipError_t launch_reset(WsHeader* h, int* prog, int64_t nprog, double* out, int64_t nout,
                        unsigned order, hipStream_t s) {
    int64_t n = std::max<int64_t>(std::max(nprog, nout), 1);
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, h, prog, nprog, out, nout,
                       order);
    return hipGetLastError();
}

thread_local char g_errbuf[256];

// ---------------------------------------------------------------- gram layout
struct GramLayout {
    size_t hdr = 0, prog = 0, front = 0, total = 0;
    int64_t strips = 0, npairs = 0, nprog = 0;
};

GramLayout gram_layout(int64_t nx, int64_t ny, int64_t lx, int64_t ly, int symmetric, int P) {
    GramLayout L;
    L.npairs = symmetric ? nx * (nx + 1) / 2 : nx * ny;
    const int64_t m = std::max<int64_t>(lx - 1, 0), n = std::max<int64_t>(ly - 1, 0);
    L.strips = (n + kWave - 1) / kWave;
    L.nprog = L.npairs * L.strips;
    L.hdr = 0;
    L.prog = align256(sizeof(WsHeader));
    L.front = align256(L.prog + sizeof(int) * (size_t)std::max<int64_t>(L.nprog, 1));
    L.total = align256(L.front + sizeof(double) * (size_t)(L.npairs * m * P));
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
    size_t o_desc = 0, o_tk = 0, o_tkr = 0, o_prog = 0, o_front = 0, fwd_total = 0;
    size_t o_snap = 0, o_ckpt = 0, o_lfront = 0, o_lprog = 0, o_gdx = 0, o_scr = 0,
           bwd_total = 0;
};

namespace {

constexpr int kBwdMaxGrid = 2048;

void plan_layout(sigk_plan& p) {
    size_t o = align256(sizeof(WsHeader));
    p.o_desc = o;
    o = align256(o + sizeof(PairDesc) * std::max<size_t>(p.desc.size(), 1));
    p.o_tk = o;
    o = align256(o + sizeof(Ticket) * std::max<size_t>(p.tickets.size(), 1));
    p.o_tkr = o;
    o = align256(o + sizeof(Ticket) * std::max<size_t>(p.tickets_rev.size(), 1));
    p.o_prog = o;
    o = align256(o + sizeof(int) * (size_t)std::max<int64_t>(p.nprog, 1));
    p.o_front = o;
    o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(p.front_doubles, 1));
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
    p.bwd_grid = kBwdMaxGrid;
    o = align256(o + sizeof(double) * (size_t)p.bwd_grid * kCkptEvery * p.P * kWave);
    p.bwd_total = o;
}

bool valid_opts(const sigk_opts* o) { return o == nullptr || (std::isfinite(o->tol) && std::isfinite(o->tail_tol)); }

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
    o->tail_tol = std::ldexp(1.0, -50);
    o->order = 12;
}

int sigk_supported_order(int order) { return round_order(order); }

int sigk_device_grid(int order, int64_t d, int backward) {
    const int P = round_order(order);
    const int D = round_dim(d);
    if (!P || !D) return 0;
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
    if (!P || !round_dim(d)) return SIGK_EUNSUPPORTED;
    *bytes = gram_layout(nx, ny, lx, ly, symmetric, P).total;
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
    const int D = round_dim(d);
    if (!P || !D) return SIGK_EUNSUPPORTED;
    const GramLayout L = gram_layout(nx, ny, lx, ly, symmetric, P);
    if (L.nprog > INT32_MAX) return SIGK_EINVAL;  // progress slots are indexed in 32 bits
    if (ws_bytes < L.total) return SIGK_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    WsHeader* hdr = (WsHeader*)(base + L.hdr);
    int* prog = (int*)(base + L.prog);
    hipError_t e = launch_reset(hdr, prog, L.nprog, G, nx * ny, (unsigned)P, s);
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
    const Variant* v = find_fwd(P, D);
    if (!v) return SIGK_EUNSUPPORTED;
    int grid = op.grid > 0 ? op.grid : device_wgs(P, D, kKernelFwd);
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    e = v->fwd(a, std::max(grid, 1), s);
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
    if (!P || !D) return SIGK_EUNSUPPORTED;
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
    const int64_t lag_fwd = fwd_chunk_cols(P, D) + kWave - 1, lag_adj = chunk_cols(P) + kWave - 1;
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
    plan_layout(*pl);
    *plan = pl;
    return SIGK_OK;
}

namespace {

// Adjoint ticket counter (the adjoint may run long after the checkpoint pass
// that reset the header).
__global__ void zero_tickets_kernel(WsHeader* h) { h->ticket2 = 0; }

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
    char* base = (char*)ws;
    WsHeader* hdr = (WsHeader*)base;
    int* prog = (int*)(base + plan->o_prog);
    hipError_t e = launch_reset(hdr, prog, plan->nprog, out, plan->npairs, (unsigned)plan->P, s);
    if (e != hipSuccess) return device_error(e);
    if (plan->tickets.empty()) return SIGK_OK;
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, plan->opts, plan->P, plan->d, plan->max_cells);
    a.mode = kModeTable;
    a.X = pool;
    a.Y = pool;
    a.npairs = plan->npairs;
    a.ntickets = (int64_t)plan->tickets.size();
    a.desc = (const PairDesc*)(base + plan->o_desc);
    a.tickets = (const Ticket*)(base + plan->o_tk);
    a.out = out;
    a.frontier = (double*)(base + plan->o_front);
    a.progress = prog;
    a.hdr = hdr;
    const Variant* v = find_fwd(plan->P, plan->D);
    if (!v) return SIGK_EUNSUPPORTED;
    int grid = plan->opts.grid > 0 ? plan->opts.grid : device_wgs(plan->P, plan->D, kKernelFwd);
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    e = v->fwd(a, std::max(grid, 1), s);
    if (e != hipSuccess) return device_error(e);
    return SIGK_OK;
}

int sigk_gram_ragged_workspace_size(const int64_t* offsets, int64_t npaths, int64_t d,
                                    const int32_t* pairs, int64_t npairs, const sigk_opts* o,
                                    size_t* bytes) {
    if (!bytes) return SIGK_EINVAL;
    sigk_plan* pl = nullptr;
    int rc = sigk_plan_ragged(offsets, npaths, d, pairs, npairs, o, &pl);
    if (rc) return rc;
    *bytes = pl->fwd_total;
    sigk_plan_destroy(pl);
    return SIGK_OK;
}

int sigk_gram_ragged(const double* pool, const int64_t* offsets, int64_t npaths, int64_t d,
                     const int32_t* pairs, int64_t npairs, const sigk_opts* o, double* out,
                     void* ws, size_t ws_bytes, void* stream) {
    sigk_plan* pl = nullptr;
    int rc = sigk_plan_ragged(offsets, npaths, d, pairs, npairs, o, &pl);
    if (rc) return rc;
    if (ws_bytes < pl->fwd_total) {
        sigk_plan_destroy(pl);
        return SIGK_EWORKSPACE;
    }
    rc = sigk_plan_upload(pl, ws, ws_bytes, stream);
    if (!rc) rc = sigk_plan_run(pl, pool, out, ws, ws_bytes, stream);
    // the table copies come from pageable plan memory: wait before freeing it
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (!rc && e != hipSuccess) rc = device_error(e);
    sigk_plan_destroy(pl);
    return rc;
}

int sigk_backward_workspace_size(const int64_t* offsets, int64_t npaths, int64_t d,
                                 const int32_t* pairs, int64_t npairs, const sigk_opts* o,
                                 size_t* bytes) {
    if (!bytes) return SIGK_EINVAL;
    sigk_plan* pl = nullptr;
    int rc = sigk_plan_ragged(offsets, npaths, d, pairs, npairs, o, &pl);
    if (rc) return rc;
    *bytes = pl->bwd_total;
    sigk_plan_destroy(pl);
    return SIGK_OK;
}

int sigk_backward(const double* pool, const int64_t* offsets, int64_t npaths, int64_t d,
                  const int32_t* pairs, int64_t npairs, const double* grad_out, const sigk_opts* o,
                  double* grad_pool, void* ws, size_t ws_bytes, void* stream) {
    sigk_plan* pl = nullptr;
    int rc = sigk_plan_ragged(offsets, npaths, d, pairs, npairs, o, &pl);
    if (rc) return rc;
    if (ws_bytes < pl->bwd_total) {
        sigk_plan_destroy(pl);
        return SIGK_EWORKSPACE;
    }
    rc = sigk_plan_upload(pl, ws, ws_bytes, stream);
    if (!rc) rc = sigk_plan_backward(pl, pool, grad_out, grad_pool, ws, ws_bytes, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (!rc && e != hipSuccess) rc = device_error(e);
    sigk_plan_destroy(pl);
    return rc;
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
                    char* base, hipStream_t s) {
    WsHeader* hdr = (WsHeader*)base;
    int* prog = (int*)(base + plan->o_prog);
    hipError_t e = launch_reset(hdr, prog, plan->nprog, out, out ? plan->npairs : 0,
                                (unsigned)plan->P, s);
    if (e != hipSuccess) return device_error(e);
    FwdArgs a;
    std::memset(&a, 0, sizeof a);
    fill_common(a, plan->opts, plan->P, plan->d, plan->max_cells);
    a.mode = kModeTable;
    a.X = pool;
    a.Y = pool;
    a.npairs = plan->npairs;
    a.ntickets = (int64_t)plan->tickets.size();
    a.desc = (const PairDesc*)(base + plan->o_desc);
    a.tickets = (const Ticket*)(base + plan->o_tk);
    a.out = out;
    a.frontier = (double*)(base + plan->o_snap);
    a.progress = prog;
    a.hdr = hdr;
    a.ckpt = (double*)(base + plan->o_ckpt);
    int grid = plan->opts.grid > 0 ? plan->opts.grid : device_wgs(plan->P, plan->D, kKernelCkpt);
    grid = (int)std::min<int64_t>(grid, a.ntickets);
    e = v->ckpt(a, std::max(grid, 1), s);
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
    b.ntickets = (int64_t)plan->tickets_rev.size();
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
    if (plan->tickets.empty()) {
        hipError_t e = launch_reset((WsHeader*)ws, (int*)((char*)ws + plan->o_prog), plan->nprog,
                                    out, plan->npairs, (unsigned)plan->P, s);
        return e == hipSuccess ? SIGK_OK : device_error(e);
    }
    const Variant* v = find_bwd(plan->P, plan->D);
    if (!v) return SIGK_EUNSUPPORTED;
    return checkpoint_pass(plan, v, pool, out, (char*)ws, s);
}

int sigk_plan_backward_checkpointed(const sigk_plan* plan, const double* pool,
                                    const double* grad_out, double* grad_pool, void* ws,
                                    size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !grad_out || !grad_pool)))
        return SIGK_EINVAL;
    if (ws_bytes < plan->bwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0 || plan->tickets.empty()) return SIGK_OK;
    const Variant* v = find_bwd(plan->P, plan->D);
    if (!v) return SIGK_EUNSUPPORTED;
    return adjoint_pass(plan, v, pool, grad_out, grad_pool, (char*)ws, (hipStream_t)stream);
}

int sigk_plan_backward(const sigk_plan* plan, const double* pool, const double* grad_out,
                       double* grad_pool, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !ws || (plan->npairs > 0 && (!pool || !grad_out || !grad_pool)))
        return SIGK_EINVAL;
    if (ws_bytes < plan->bwd_total) return SIGK_EWORKSPACE;
    if (plan->npairs == 0 || plan->tickets.empty()) return SIGK_OK;
    const Variant* v = find_bwd(plan->P, plan->D);
    if (!v) return SIGK_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    int rc = checkpoint_pass(plan, v, pool, nullptr, (char*)ws, s);
    if (rc) return rc;
    return adjoint_pass(plan, v, pool, grad_out, grad_pool, (char*)ws, s);
}

}  // extern "C"
