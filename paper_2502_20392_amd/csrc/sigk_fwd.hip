// sigk_fwd.hip -- persistent forward kernel: k(x, y) for many pairs.
//
// Work unit ("ticket") = one 64-row strip of one pair.  Workgroups (one
// wavefront each) claim tickets from a global counter in an order in which
// every strip's producer (the strip below it) has a smaller ticket, so a
// waiting wave always waits on a wave that is already running (no deadlock
// for any grid size).  Gram mode interleaves pairs strip-major (all pairs'
// strip 0, then strip 1, ...); table mode takes the host-built order.
//
// Compiled once per (P, D) variant: -DSIGK_P=<order> -DSIGK_D=<channel bucket>;
// -DSIGK_SQ=1 builds the square-truncation variant (the paper's fixed-order
// tile matrix, selected by SIGK_FLAG_SQUARE) under the launcher names
// launch_fwdsq_P_D / occupancy_fwdsq_P_D; -DSIGK_ALT=1 the variant with the
// other frontier chunk width (alt_chunk_cols) as launch_fwdt_P_D /
// occupancy_fwdt_P_D.
#include "sigk_strip.h"

#ifndef SIGK_P
#define SIGK_P 8
#endif
#ifndef SIGK_D
#define SIGK_D 8
#endif
#ifndef SIGK_SQ
#define SIGK_SQ 0
#endif
#ifndef SIGK_ALT
#define SIGK_ALT 0
#endif

namespace sigk {

template <int P, int D, bool SQ, int CH>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(P <= 6 && D <= 8 ? 3 : 1))) fwd_kernel(FwdArgs a) {
    constexpr int RB = CH == 64 ? 128 : ring_cols(P);
    __shared__ LdsStrip<P, D, CH, RB> L;
    Acc acc;
    const int lane = lane_id();
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(&a.hdr->ticket, 1u);
        t = (unsigned)uniform((int)t);
        if ((int64_t)t >= a.ntickets) break;
        if (uniform((int)(load_status(a.hdr) & SIGK_ERR_WATCHDOG))) break;
        int pair, strip;
        if (a.mode == kModeGram) {
            pair = (int)((int64_t)t % a.npairs);
            strip = (int)((int64_t)t / a.npairs);
        } else {
            pair = a.tickets[t].pair;
            strip = a.tickets[t].strip;
            if (pair < 0) break;  // unused slots close a table built on the device
        }
        Geo g = resolve(a, pair, P, 0);
        StripCtx<P, D, CH, RB, SQ> S(a, g, L, acc, strip);
        S.pair = pair;
        S.Fout = a.frontier + g.front;
        S.Fin = S.Fout;
        S.prog = a.progress + g.prog;
        S.ck = nullptr;
        S.ckq = nullptr;
        S.ck_every = 1;
        if (!S.sweep()) break;
    }
    if (lane == 0) {
        atomicAdd(&a.hdr->cells, acc.cells);
        atomicAdd(&a.hdr->flops, acc.flops);
        if (acc.status) atomicOr(&a.hdr->status, acc.status);
    }
}

#define SIGK_CAT3(a, b, c) a##b##_##c
#define SIGK_NAME(pre, P, D) SIGK_CAT3(pre, P, D)

#if SIGK_SQ
#define SIGK_LAUNCH launch_fwdsq_
#define SIGK_OCC occupancy_fwdsq_
#elif SIGK_ALT
#define SIGK_LAUNCH launch_fwdt_
#define SIGK_OCC occupancy_fwdt_
#else
#define SIGK_LAUNCH launch_fwd_
#define SIGK_OCC occupancy_fwd_
#endif
constexpr int kChunk = SIGK_ALT ? alt_chunk_cols(SIGK_P, SIGK_D) : fwd_chunk_cols(SIGK_P, SIGK_D);

hipError_t SIGK_NAME(SIGK_LAUNCH, SIGK_P, SIGK_D)(const FwdArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((fwd_kernel<SIGK_P, SIGK_D, SIGK_SQ != 0, kChunk>), dim3(grid),
                       dim3(kWave), 0, s, a);
    return hipGetLastError();
}

int SIGK_NAME(SIGK_OCC, SIGK_P, SIGK_D)() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fwd_kernel<SIGK_P, SIGK_D, SIGK_SQ != 0, kChunk>, kWave, 0) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace sigk
