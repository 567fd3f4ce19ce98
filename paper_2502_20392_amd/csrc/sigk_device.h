// sigk_device.h -- device helpers for the gfx950 kernels of libsigk.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sigk.h"
#include "sigk_internal.h"

namespace sigk {

// ---------------------------------------------------------------- lanes
__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }

__device__ __forceinline__ uint64_t ballot(bool p) {
    return (uint64_t)__builtin_amdgcn_ballot_w64(p);
}

// Lane i receives v from lane i-1; lane 0 receives `lane0` (DPP wave_shr:1).
__device__ __forceinline__ double shift_up(double v, double lane0) {
    const long long b = __double_as_longlong(v);
    const long long o = __double_as_longlong(lane0);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), 0x138, 0xf, 0xf,
                                               false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane i receives v from lane i+1; lane 63 receives `lane63` (DPP wave_shl:1).
__device__ __forceinline__ double shift_down(double v, double lane63) {
    const long long b = __double_as_longlong(v);
    const long long o = __double_as_longlong(lane63);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), 0x130, 0xf, 0xf,
                                               false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------- sync
__device__ __forceinline__ unsigned load_status(WsHeader* h) {
    return __hip_atomic_load(&h->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_status(WsHeader* h, unsigned bits) {
    if (bits && lane_id() == 0)
        __hip_atomic_fetch_or(&h->status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent accesses for data exchanged between workgroups without
// cache maintenance: the producer writes with device-scope stores (written
// through to the level shared by all XCDs), waits for them to complete and
// then raises a flag; the consumer polls the flag and reads the data with
// device-scope loads (CoherentSpan).  No L2 write-back or invalidation is
// needed.
__device__ __forceinline__ void store_coherent(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// n doubles at p read with device-coherent plain loads (buffer loads with the
// coherence bit that device-scope atomic loads use, but free for the compiler
// to batch).  Indices outside [0, n) read 0 (hardware range check).
struct CoherentSpan {
    __amdgpu_buffer_rsrc_t r;
    // p and n must be uniform over the wave (made explicit for the compiler,
    // which needs the descriptor in scalar registers)
    __device__ CoherentSpan(const double* p, int n) {
        const uint64_t a = (uint64_t)p;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
        void* u = (void*)(((uint64_t)hi << 32) | lo);
        r = __builtin_amdgcn_make_buffer_rsrc(u, (short)0, __builtin_amdgcn_readfirstlane(n * 8),
                                              0x00020000);
    }
    __device__ __forceinline__ double load(int i) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0,
                                                                               kCoherentLoad));
    }
    static constexpr int kCoherentLoad = 16;  // cache-policy operand: sc1
};

// Wait until *flag >= need, for data then read back with device-coherent
// loads (no cache invalidation, only ordering of the following loads after
// the flag).  Returns false (and raises the watchdog bit for everyone) if the
// wait exceeds `ticks` of the 100 MHz real-time counter, or if another wave
// already raised it.
__device__ bool wait_flag(const int* flag, int need, WsHeader* h, long long ticks) {
    int v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (uniform(v) < need) {
        const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
        for (;;) {
            __builtin_amdgcn_s_sleep(2);
            v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (uniform(v) >= need) break;
            if (uniform((int)(load_status(h) & SIGK_ERR_WATCHDOG))) return false;
            const long long now = (long long)__builtin_amdgcn_s_memrealtime();
            if (now - t0 > ticks) {
                raise_status(h, SIGK_ERR_WATCHDOG);
                return false;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return true;
}

// Raise a flag after store_coherent writes: wait until they have completed
// (gfx9 counts stores in vmcnt), then store the flag.
__device__ __forceinline__ void publish_coherent(int* flag, int value) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    if (lane_id() == 0) __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- geometry
struct Geo {
    const double* x;  // path along the columns (u direction)
    const double* y;  // path along the rows (v direction)
    int m, n;         // cells: columns, rows
    int64_t front;    // frontier offset (doubles)
    int64_t ckpt;     // checkpoint offset (doubles)
    int64_t delta;    // cell-coefficient field offset (doubles; channel bucket 0)
    int prog;         // progress offset
    int o1, o2;       // output slots
};

// Row i and column j of entry p of the upper triangle (i <= j) of an N x N
// matrix enumerated row by row.
__device__ __forceinline__ void tri_decode(int64_t p, int64_t N, int64_t& i, int64_t& j) {
    const double b = 2.0 * (double)N + 1.0;
    int64_t r = (int64_t)((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
    if (r < 0) r = 0;
    if (r >= N) r = N - 1;
    auto start = [N](int64_t q) { return q * N - q * (q - 1) / 2; };
    while (r > 0 && start(r) > p) --r;
    while (r + 1 < N && start(r + 1) <= p) ++r;
    i = r;
    j = r + (p - start(r));
}

__device__ Geo resolve(const FwdArgs& a, int pair, int P, int64_t ckpt_per_pair) {
    Geo g;
    if (a.mode == kModeGram) {
        int64_t i, j;
        if (a.symmetric) {
            tri_decode(pair, a.nx, i, j);
        } else {
            i = pair / a.ny;
            j = pair % a.ny;
        }
        g.x = a.X + i * a.lx * a.d;
        g.y = a.Y + j * a.ly * a.d;
        g.m = (int)a.lx - 1;
        g.n = (int)a.ly - 1;
        g.front = (int64_t)pair * (int64_t)g.m * P * (a.ckpt ? a.strips : 1);
        g.ckpt = (int64_t)pair * ckpt_per_pair;
        g.delta = (int64_t)pair * a.delta_pair;
        g.prog = pair * a.strips;
        g.o1 = (int)(i * a.ny + j);
        g.o2 = (a.symmetric && i != j) ? (int)(j * a.ny + i) : -1;
    } else {
        const PairDesc& p = a.desc[pair];
        g.x = a.X + p.x_off;
        g.y = a.Y + p.y_off;
        g.m = p.lx - 1;
        g.n = p.ly - 1;
        g.front = p.front_off;
        g.ckpt = p.ckpt_off;
        g.delta = 0;
        g.prog = p.prog_off;
        g.o1 = p.out_idx;
        g.o2 = p.out_idx2;
    }
    return g;
}

// kModeLines: the whole pair (X = x, Y = y), one output.
__device__ __forceinline__ Geo resolve_lines(const FwdArgs& a) {
    Geo g;
    g.x = a.X;
    g.y = a.Y;
    g.m = (int)a.blk.m;
    g.n = (int)a.blk.n;
    g.front = 0;
    g.ckpt = 0;
    g.delta = 0;
    g.prog = 0;
    g.o1 = 0;
    g.o2 = -1;
    return g;
}

// Boundary data of a block in kModeBlock (null where the block touches the
// axes, i.e. its bottom or left edge is the constant 1).
struct BlockRef {
    int I, J;           // block row and column
    const double* bot;  // primal bottom edges of its columns ([cb][P])
    const double* left; // primal left edges of its rows ([rb][P])
    bool above, right;  // a block above / to the right exists
};

// Block of slot `slot` on the launch's anti-diagonal: a sub-pair of the paths
// with its own strips, snapshots, checkpoints and progress counters.
__device__ __forceinline__ Geo resolve_block(const FwdArgs& a, int slot, int P, BlockRef& r) {
    const BlockGeo& k = a.blk;
    const int J = k.j_lo + slot, I = k.diag - J;
    Geo g;
    g.x = a.X + (int64_t)J * k.cb * a.d;
    g.y = a.Y + (int64_t)I * k.rb * a.d;
    g.m = (int)(k.m - (int64_t)J * k.cb < k.cb ? k.m - (int64_t)J * k.cb : k.cb);
    g.n = (int)(k.n - (int64_t)I * k.rb < k.rb ? k.n - (int64_t)I * k.rb : k.rb);
    g.front = (int64_t)slot * k.slot_snap;
    g.ckpt = (int64_t)slot * k.slot_ckpt;
    g.delta = 0;
    g.prog = slot * k.slot_prog + 1;
    g.o1 = -1;
    g.o2 = -1;
    r.I = I;
    r.J = J;
    r.bot = I > 0 ? k.hline + ((int64_t)(I - 1) * k.m + (int64_t)J * k.cb) * P : nullptr;
    r.left = J > 0 ? k.vline + ((int64_t)(J - 1) * k.n + (int64_t)I * k.rb) * P : nullptr;
    r.above = I + 1 < k.ni;
    r.right = J + 1 < k.nj;
    return g;
}

}  // namespace sigk
