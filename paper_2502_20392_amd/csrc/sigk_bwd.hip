// sigk_bwd.hip -- gradient of kernel values with respect to the paths.
//
// Two persistent kernels per (P, D) variant:
//   ckpt_kernel: the forward sweep of every strip, keeping (a) the frontier row
//                each strip reads (one snapshot per strip instead of the single
//                in-place row), (b) the wave state (left edges and in-flight top
//                edges of all 64 lanes) every kCkptEvery steps and (c) the
//                Neumann depth of every chunk.
//   bwd_kernel:  the adjoint sweep, strips in reverse topological order (top
//                strip of each pair first).  Per segment of kCkptEvery steps,
//                taken last to first: restore the wave state, recompute the
//                segment forward while storing each step's bottom-edge inputs
//                in a per-workgroup scratch, then run the adjoint cell map over
//                the segment in reverse step order, recovering each cell's left
//                edge from its right edge (the left-edge update is
//                triangular).  dL/dc of every cell is chained into
//                dL/d(increment) of both paths: the x side through an LDS ring
//                indexed by column (each column is complete once lane 0 has
//                passed it), the y side in registers of the row's lane.
// Both also run the blocks of a long pair (block checkpointing, see BlockGeo):
// a block is a small pair whose bottom and left edges come from lines kept by
// a first sweep and whose top and right edge cotangents come from the blocks
// processed before it.
#include "sigk_adjoint.h"

#ifndef SIGK_P
#define SIGK_P 8
#endif
#ifndef SIGK_D
#define SIGK_D 8
#endif

namespace sigk {

// Frontier chunk of the checkpointing forward sweep (which also sets the
// granularity of the Neumann depths the adjoint reads back): 64 columns where
// the kernel runs one wave per SIMD anyway (orders 10-20, D <= 16), as in the
// plain forward sweep; 32 elsewhere.
template <int P, int D>
constexpr int ckpt_chunk = (P >= 10 && P <= 20 && D <= 16) ? 64 : 32;

// Modes: kModeTable, the checkpointing sweep of a batch (snap: per-strip
// frontier rows); kModeBlock, the checkpointing sweep of the blocks of one
// anti-diagonal (snap: per-slot frontier rows; strip 0 reads its bottom line,
// column 0 its left line).
// (three waves per SIMD at orders 4-5 with d <= 8: 168 registers, 7% faster
// at order 5; at order 6 that limit would spill)
template <int P, int D>
__global__ void __launch_bounds__(kWave)
    __attribute__((amdgpu_waves_per_eu(P <= 5 && D <= 8 ? 3 : 1))) ckpt_kernel(FwdArgs a,
                                                                              double* snap) {
    constexpr int CH = ckpt_chunk<P, D>, RB = CH == 64 ? 128 : ring_cols(P);
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
        Geo g;
        BlockRef r;
        r.bot = nullptr;
        r.left = nullptr;
        if (a.mode == kModeTable) {
            pair = a.tickets[t].pair;
            strip = a.tickets[t].strip;
            if (pair < 0) break;  // unused slots close a table built on the device
            g = resolve(a, pair, P, 0);
            g.front = a.desc[pair].snap_off;
        } else {
            pair = (int)(t % (unsigned)a.blk.nb);
            strip = (int)(t / (unsigned)a.blk.nb);
            g = resolve_block(a, pair, P, r);
            if (strip * kWave >= g.n) continue;  // the top block row has fewer strips
        }
        StripCtx<P, D, CH, RB, false, true> S(a, g, L, acc, strip);
        S.pair = pair;
        S.prog = a.progress + g.prog;
        const int64_t row = (int64_t)g.m * P;
        S.Fin = (strip == 0 && r.bot) ? r.bot : snap + g.front + (int64_t)strip * row;
        S.Fout = snap + g.front + (int64_t)(strip + 1) * row;
        double* ck = a.ckpt + g.ckpt + (int64_t)strip * ckpt_strip_doubles(g.m, P);
        S.ck = ck;
        S.ckq = ck + ckpt_states(g.m) * 2 * P * kWave;
        S.ck_every = kCkptEvery;
        S.left = r.left;
        S.below_line = r.bot != nullptr;
        if (!S.sweep()) break;
    }
    if (lane == 0) {
        atomicAdd(&a.hdr->cells, acc.cells);
        atomicAdd(&a.hdr->flops, acc.flops);
        if (acc.status) atomicOr(&a.hdr->status, acc.status);
    }
}

// The first sweep of a long pair's gradient (kModeLines): the plain forward
// sweep of the whole pair, with the plain forward kernel's chunks and
// occupancy, writing k(x, y) and keeping the block-boundary lines: a strip
// that ends a block row writes its top edges to that row's line instead of
// the in-place frontier row (the next strip reads them there), and every
// lane stores its right edge at the last column of each block column.
template <int P, int D>
__global__ void __launch_bounds__(kWave)
    __attribute__((amdgpu_waves_per_eu(P <= 6 && D <= 8 ? 3 : 1))) lines_kernel(FwdArgs a) {
    constexpr int CH = fwd_chunk_cols(P, D), RB = fwd_ring_cols(P, D);
    __shared__ LdsStrip<P, D, CH, RB> L;
    Acc acc;
    const int lane = lane_id();
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(&a.hdr->ticket, 1u);
        t = (unsigned)uniform((int)t);
        if ((int64_t)t >= a.ntickets) break;
        if (uniform((int)(load_status(a.hdr) & SIGK_ERR_WATCHDOG))) break;
        const int strip = (int)t;
        Geo g = resolve_lines(a);
        StripCtx<P, D, CH, RB, false, true> S(a, g, L, acc, strip);
        S.pair = 0;
        S.prog = a.progress;
        const int64_t row = (int64_t)g.m * P;
        const int kb = a.blk.kb;
        S.Fin = (strip > 0 && strip % kb == 0) ? a.blk.hline + (int64_t)(strip / kb - 1) * row
                                               : a.frontier;
        S.Fout = ((strip + 1) % kb == 0 && (int64_t)(strip + 1) * kWave < g.n)
                     ? a.blk.hline + (int64_t)((strip + 1) / kb - 1) * row
                     : a.frontier;
        S.ck = nullptr;
        S.ckq = nullptr;
        S.ck_every = 1;
        S.vl = a.blk.nj > 1 ? a.blk.vline : nullptr;
        if (!S.sweep()) break;
    }
    if (lane == 0) {
        atomicAdd(&a.hdr->cells, acc.cells);
        atomicAdd(&a.hdr->flops, acc.flops);
        if (acc.status) atomicOr(&a.hdr->status, acc.status);
    }
}

// A workgroup's segment scratch as a buffer resource: rows of 64 doubles,
// one per lane.  The lane's column goes in the vector offset and the row
// (step and coefficient) in the scalar offset, so stepping through the rows
// costs no vector instructions.  Every access is range-checked against the
// buffer's size by the hardware.
struct SegScratch {
    using u32x2 = unsigned int __attribute__((__vector_size__(8)));
    __amdgpu_buffer_rsrc_t r;
    __device__ void init(double* p, int rows) {
        const uint64_t a = (uint64_t)p;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
        r = __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0,
                                              rows * kWave * 8, 0x00020000);
    }
    __device__ __forceinline__ void store(int row, double v) const {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, lane_id() * 8,
                                              row * (kWave * 8), 0);
    }
    __device__ __forceinline__ double load(int row) const {
        return __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_id() * 8, row * (kWave * 8), 0));
    }
};

// Byte offset of a lane's slot in a ring of ARB columns, stepped one column
// at a time (two or three vector instructions instead of a division).
template <int ARB>
struct RingPos {
    unsigned b;
    __device__ __forceinline__ void set(int col) { b = (unsigned)ring_slot_of<ARB>(col) * 8u; }
    __device__ __forceinline__ void next() {
        if constexpr ((ARB & (ARB - 1)) == 0)
            b = (b + 8u) & (unsigned)((ARB - 1) * 8);
        else
            b = b + 8u == (unsigned)(ARB * 8) ? 0u : b + 8u;
    }
    __device__ __forceinline__ void prev() {
        if constexpr ((ARB & (ARB - 1)) == 0)
            b = (b - 8u) & (unsigned)((ARB - 1) * 8);
        else
            b = b == 0u ? (unsigned)((ARB - 1) * 8) : b - 8u;
    }
};

template <int P, int D>
struct LdsBwd {
    // Columns per cotangent-frontier chunk and of the increment rings.  At
    // orders 10-12 with D = 8 the adjoint exchanges 64-column chunks (a
    // 128-column ring; the buffers then fill LDS exactly at four waves per
    // CU, the register-bound occupancy): 2% faster on the MMD^2 workload.
    // Per-chunk Neumann depths are still read at the checkpointing sweep's
    // chunk width (depth_at).
    static constexpr int ACH = (P >= 10 && P <= 12 && D <= 8) ? 64 : 32;
    // (96 columns hold a 32-column chunk and the 63 before it; at orders 4-5
    // with d <= 8 the smaller rings let an eighth wave per CU fit its LDS:
    // 4.5% faster there than with 128)
    static constexpr int ARB = ACH == 64 ? 128 : 96;
    static_assert(ARB >= ACH + kWave - 1,
                  "the rings must hold a chunk and the 63 columns before it");
    // (the edge rows first: one address register with the instructions'
    // immediate offsets reaches a whole row)
    double bin[ACH * P];    // primal bottom edges (lane 0) of a chunk
    double lin[2 * ACH * P];  // top-edge cotangents (top lane), 2 chunks
    double lout[ACH * P];   // bottom-edge cotangents (lane 0), 1 chunk
    // increments of x and dL/d(dx) being accumulated, by ring slot,
    // interleaved per channel: [channel][dx, gx][slot].  A channel's rows lie
    // 2 ARB doubles apart, a multiple of 512 bytes, so one address register
    // and offsets in 512-byte units reach every channel's slot.
    double xg[D * 2 * ARB];
    static_assert((2 * ARB * 8) % 512 == 0 && (ACH * P * 4 * 8) % 512 == 0,
                  "channel rows on 512-byte boundaries");
    __device__ __forceinline__ double& dx(int ch, int slot) { return xg[2 * ch * ARB + slot]; }
    __device__ __forceinline__ double& gx(int ch, int slot) {
        return xg[(2 * ch + 1) * ARB + slot];
    }
    // the same by a RingPos byte offset
    __device__ __forceinline__ double& dx_at(int ch, const RingPos<ARB>& p) {
        return *(double*)((char*)&xg[2 * ch * ARB] + p.b);
    }
    __device__ __forceinline__ double& gx_at(int ch, const RingPos<ARB>& p) {
        return *(double*)((char*)&xg[(2 * ch + 1) * ARB] + p.b);
    }
};

template <int P, int D>
struct StripBwd {
    static constexpr int ACH = LdsBwd<P, D>::ACH;
    static constexpr int ARB = LdsBwd<P, D>::ARB;
    const BwdArgs& b;
    const FwdArgs& a;
    Geo& g;
    LdsBwd<P, D>& L;
    int s, nrows, m;
    bool lane_ok, has_below, has_above;
    double dy[D];
    double gy[D];
    Recip<P, false> R;  // scalar or rematerialised constants: registers are scarce here
    int dx_lo, lin_lo, bin_chunk;
    SegScratch scr;  // kCkptEvery x P recomputed bottom-edge rows, then as many left-edge rows
    unsigned long long* cells;  // per-workgroup tallies (cells, algorithmic flops)
    unsigned long long* flops;
    const double* ck;
    const double* ckq;
    const double* snap_in;   // primal frontier row read by lane 0 ([m][P])
    double* lam_row;         // adjoint frontier row of the pair ([m][P])
    int* lam_prog;           // adjoint progress of the pair's strips
    double seed_scale;       // grad_out of the pair (0: no seed in this grid)
    double* gxp;             // dL/d(dx) of the pair's columns ([m][d])
    double* gyp;             // dL/d(dy) of the pair's rows ([n][d])
    // block checkpointing (null / false for whole pairs): primal left edges at
    // column 0, a primal bottom line for strip 0 and a cotangent row from a
    // block above; the right-edge cotangents of the rows (read at the last
    // column when a block to the right exists, written at column 0 when one
    // to the left does)
    const double* left = nullptr;
    bool below_line = false;
    bool above_blk = false;
    double* lamv = nullptr;
    bool right_in = false;
    bool left_out = false;

    __device__ StripBwd(const BwdArgs& b_, Geo& g_, LdsBwd<P, D>& L_, int s_)
        : b(b_), a(b_.f), g(g_), L(L_), s(s_) {}

    // Increments of x in steps of kCkptEvery columns, descending, so that the
    // ring holds [t0-63, t0+kCkptEvery) for segment t0 (and never more than
    // 63 + chunk columns of pending dL/d(dx) share its slots).
    __device__ void load_dx_down_to(int lo_needed) {
        const int lane = lane_id();
        while (dx_lo > lo_needed && dx_lo > 0) {
            const int c0 = max(dx_lo - kCkptEvery, 0);
            const int col = c0 + lane;
            if (col < dx_lo && col < m) {
                const double* xp = g.x + (int64_t)col * a.d;
#pragma unroll
                for (int ch = 0; ch < D; ++ch)
                    L.dx(ch, ring_slot_of<ARB>(col)) = ch < a.d ? xp[a.d + ch] - xp[ch] : 0.0;
            }
            dx_lo = c0;
            __syncthreads();
        }
    }

    __device__ bool load_lin_down_to(int lo_needed) {
        const int CH = ACH;
        const int lane = lane_id();
        while (lin_lo > lo_needed && lin_lo > 0) {
            const int c0 = lin_lo - CH;
            const int nc = min(CH, m - c0);
            if (!wait_flag(&lam_prog[s + 1], m - c0, a.hdr, a.watchdog_ticks)) return false;
            double* dst = &L.lin[((c0 / CH) & 1) * CH * P];
            constexpr int NB = (ACH * P + kWave - 1) / kWave;
            const CoherentSpan src(lam_row + (int64_t)c0 * P, nc * P);
            double v[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) v[k] = src.load(lane + k * kWave);
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (lane + k * kWave < nc * P) dst[lane + k * kWave] = v[k];
            lin_lo = c0;
            __syncthreads();
        }
        return true;
    }

    __device__ void load_bin(int chunk) {
        const int CH = ACH;
        const int lane = lane_id();
        const int c0 = chunk * CH;
        const int nc = min(CH, m - c0);
        if (has_below) {
            const double* src = snap_in + (int64_t)c0 * P;
            for (int e = lane; e < nc * P; e += kWave) L.bin[e] = src[e];
        } else {
            for (int e = lane; e < CH * P; e += kWave) L.bin[e] = (e % P) == 0 ? 1.0 : 0.0;
        }
        bin_chunk = chunk;
        __syncthreads();
    }

    // columns [c0, c1) are final: publish the bottom-edge cotangents to the
    // strip below and add dL/d(dx) to the path's gradient scratch
    __device__ void flush_cols(int c0, int c1) {
        const int CH = ACH;
        const int lane = lane_id();
        __syncthreads();
        const int nc = c1 - c0;
        if (has_below) {
            double* dst = lam_row + (int64_t)c0 * P;
            for (int e = lane; e < nc * P; e += kWave) store_coherent(&dst[e], L.lout[e]);
            publish_coherent(&lam_prog[s], m - c0);
        }
        if (lane < nc) {
            const int col = c0 + lane;
            const int sl = ring_slot_of<ARB>(col);
            double* gp = gxp + (int64_t)col * a.d;
#pragma unroll
            for (int ch = 0; ch < D; ++ch) {
                if (ch < a.d) atomicAdd(&gp[ch], L.gx(ch, sl));
                L.gx(ch, sl) = 0.0;
            }
        }
        (void)CH;
        __syncthreads();
    }

    // depth record of the chunk of step t: depth + kRoughFlag if rough
    __device__ __forceinline__ int depth_at(int t) const {
        const int CKCH = ckpt_chunk<P, D>;
        const int k = min(t, m - 1) / CKCH;
        return uniform((int)ckq[k]);
    }

    double lAprev[P];  // bottom-edge cotangents of the previous (later) step
    double lBst[P];    // left-edge cotangent carried along the row
    int topl;          // lane whose top-edge cotangent comes from outside the wave

    // Depth dispatch: one specialised segment loop per Neumann depth.
    template <int Q>
    __device__ __forceinline__ void segment_at_depth(int q, bool rough, int t0, int t1) {
        if constexpr (Q < P - 1) {
            if (q > Q) {
                segment_at_depth<Q + 1>(q, rough, t0, t1);
                return;
            }
        }
        if (t0 >= kWave && t1 <= m - 1)
            segment<Q, true>(q, rough, t0, t1);
        else
            segment<Q, false>(q, rough, t0, t1);
    }

    // One segment [t0, t1) of kCkptEvery steps: recompute it forward from its
    // checkpoint, storing each step's bottom edges, then run the adjoint steps
    // last to first.  Q >= 0: depth fixed at compile time (== q); Q < 0: q.
    // rough: the left edges are stored too (second half of the scratch) and
    // read back instead of recovered from the right edges.  IN: every cell
    // of the segment is inside the strip's columns and none is in its first
    // or last column (t0 >= 64, t1 <= m - 1), so the per-lane tests for the
    // row ends, the corner seed and the block lines drop out.
    template <int Q, bool IN>
    __device__ void segment(int q, bool rough, int t0, int t1) {
        const int lane = lane_id();
        const int CH = ACH;
        const int W = kCkptEvery;
        double B[P], Ac[P];
        {
            const double* src = ck + (int64_t)(t0 / W) * (2 * P * kWave);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                B[i] = src[i * kWave + lane];
                Ac[i] = src[(P + i) * kWave + lane];
            }
        }
        RingPos<ARB> rp;
        rp.set(t0 - lane);
        for (int t = t0; t < t1; ++t) {
            const int col = t - lane;
            if (!IN && col == 0) {
                if (left != nullptr && lane_ok) {
                    const double* lp = left + ((int64_t)s * kWave + lane) * P;
#pragma unroll
                    for (int i = 0; i < P; ++i) B[i] = lp[i];
                } else {
#pragma unroll
                    for (int i = 0; i < P; ++i) B[i] = i == 0 ? 1.0 : 0.0;
                }
            }
            double c0 = 0.0, c1 = 0.0;
#pragma unroll
            for (int ch = 0; ch < D; ch += 2) {
                c0 = fma(dy[ch], L.dx_at(ch, rp), c0);
                c1 = fma(dy[ch + 1], L.dx_at(ch + 1, rp), c1);
            }
            rp.next();
            const double c = c0 + c1;
            const int row0 = (t - t0) * P;
            if (rough) {
#pragma unroll
                for (int i = 0; i < P; ++i) scr.store(kCkptEvery * P + row0 + i, B[i]);
            }
            double A[P], An[P], Bn[P];
            const double* bsrc = &L.bin[(t % CH) * P];
            if constexpr (Q >= 0 && P <= 12) {
                // the map in two halves, as in the forward sweep (the same
                // sums in the same order): the B-only half covers the latency
                // of the lane shift that delivers A
                SplitMap<P, Q, false> S;
                S.pre(B, c, Bn, R);
#pragma unroll
                for (int i = 0; i < P; ++i) A[i] = shift_up(Ac[i], bsrc[i]);
#pragma unroll
                for (int i = 0; i < P; ++i) scr.store(row0 + i, A[i]);
                S.post(A, An, Bn, R);
            } else {
#pragma unroll
                for (int i = 0; i < P; ++i) A[i] = shift_up(Ac[i], bsrc[i]);
#pragma unroll
                for (int i = 0; i < P; ++i) scr.store(row0 + i, A[i]);
                cell_map<P>(A, B, c, An, Bn, Q >= 0 ? Q : q, R);
            }
            // past the end of the row B keeps the row's last right edge
            const bool live = IN || col < m;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                B[i] = live ? Bn[i] : B[i];
                Ac[i] = An[i];
            }
        }
        // adjoint over the segment, last step first; B walks back from the
        // right edge after the segment to each cell's left edge
        const unsigned long long fl =
            (unsigned long long)(adjoint_flops(P, Q >= 0 ? Q : q, a.d) +
                                 cell_flops(P, Q >= 0 ? Q : q, a.d));
        rp.set(t1 - 1 - lane);
        for (int t = t1 - 1; t >= t0; --t) {
            const int col = t - lane;
            const bool act = lane_ok && (IN || (col >= 0 && col < m));
            {
                const unsigned cnt = (unsigned)__builtin_popcountll(ballot(act));
                *cells += cnt;
                *flops += cnt * fl;
            }
            const int row0 = (t - t0) * P;
            double A[P];
#pragma unroll
            for (int i = 0; i < P; ++i) A[i] = scr.load(row0 + i);
            if (rough) {
#pragma unroll
                for (int i = 0; i < P; ++i) B[i] = scr.load(kCkptEvery * P + row0 + i);
            }
            double dxv[D];
            double c0 = 0.0, c1 = 0.0;
#pragma unroll
            for (int ch = 0; ch < D; ch += 2) {
                dxv[ch] = L.dx_at(ch, rp);
                dxv[ch + 1] = L.dx_at(ch + 1, rp);
                c0 = fma(dy[ch], dxv[ch], c0);
                c1 = fma(dy[ch + 1], dxv[ch + 1], c1);
            }
            const double c = c0 + c1;
            // cotangent of the top edge: from the lane above, the strip above
            // (top lane of a full strip) or the seed of the corner cell
            const int tcol = t - topl;  // column of the top lane at this step
            double lAo[P];
            if (has_above) {
                const double* lsrc = &L.lin[(((tcol >= 0 ? tcol : 0) / CH) & 1) * CH * P +
                                            ((tcol >= 0 ? tcol : 0) % CH) * P];
#pragma unroll
                for (int i = 0; i < P; ++i) lAo[i] = shift_down(lAprev[i], lsrc[i]);
            } else {
                const bool corner = !IN && col == m - 1;
                double f = seed_scale;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const double topv = corner ? f : 0.0;
                    lAo[i] = shift_down(lAprev[i], topv);
                    if (nrows < kWave) lAo[i] = lane == topl ? topv : lAo[i];
                    f = f * R(i + 1);
                }
            }
            if (!IN && col == m - 1) {
                if (right_in && lane_ok) {
                    const double* lp = lamv + ((int64_t)s * kWave + lane) * P;
#pragma unroll
                    for (int i = 0; i < P; ++i) lBst[i] = lp[i];
                } else {
#pragma unroll
                    for (int i = 0; i < P; ++i) lBst[i] = 0.0;
                }
            }
            // column 0 on a left line: the left edge is recovered like any
            // other (it is the right edge of the block to the left)
            const bool axis = !IN && col == 0 && left == nullptr;
            const bool recover = !rough && (IN || col < m);  // rough: B is the stored left edge
            double lA[P], lB[P];
            double gc;
            if constexpr (Q >= 0)
                gc = cell_adjoint_fixed<P, Q>(A, B, c, axis, recover, lAo, lBst, lA, lB, R);
            else
                gc = cell_adjoint<P>(A, B, c, q, axis, recover, lAo, lBst, lA, lB, R);
            if (!act) gc = 0.0;
            if (!IN && left_out && act && col == 0) {
                double* lp = lamv + ((int64_t)s * kWave + lane) * P;
#pragma unroll
                for (int i = 0; i < P; ++i) lp[i] = lB[i];
            }
#pragma unroll
            for (int ch = 0; ch < D; ++ch) gy[ch] = fma(gc, dxv[ch], gy[ch]);
            if (act) {
#pragma unroll
                for (int ch = 0; ch < D; ++ch) {
                    double& gv = L.gx_at(ch, rp);
                    gv = fma(gc, dy[ch], gv);
                }
                if (has_below && lane == 0) {
                    // lane 0's column is t (a uniform address)
#pragma unroll
                    for (int i = 0; i < P; ++i) L.lout[((unsigned)t % (unsigned)CH) * P + i] = lA[i];
                }
            }
            rp.prev();
#pragma unroll
            for (int i = 0; i < P; ++i) {
                lBst[i] = lB[i];
                lAprev[i] = lA[i];
            }
        }
    }

    __device__ bool sweep() {
        const int lane = lane_id();
        const int CH = ACH;
        const int W = kCkptEvery;
        m = g.m;
        const int row0 = s * kWave;
        nrows = min(kWave, g.n - row0);
        lane_ok = lane < nrows;
        has_below = s > 0 || below_line;
        has_above = row0 + kWave < g.n || above_blk;
        R.init();
        const int l = row0 + lane;
#pragma unroll
        for (int ch = 0; ch < D; ++ch) {
            dy[ch] = (ch < a.d && lane_ok)
                         ? g.y[(int64_t)(l + 1) * a.d + ch] - g.y[(int64_t)l * a.d + ch]
                         : 0.0;
            gy[ch] = 0.0;
        }
        for (int e = lane; e < 2 * D * ARB; e += kWave) L.xg[e] = 0.0;
        const int top = CH * ((m + CH - 1) / CH);
        dx_lo = kCkptEvery * ((m + kCkptEvery - 1) / kCkptEvery);
        lin_lo = top;
        bin_chunk = -1;
        __syncthreads();

        const int T = m + nrows - 1;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            lAprev[i] = 0.0;
            lBst[i] = 0.0;
        }
        topl = has_above ? kWave - 1 : nrows - 1;
        for (int t0 = ((T - 1) / W) * W; t0 >= 0; t0 -= W) {
            const int t1 = min(t0 + W, T);
            const int rec = depth_at(t0);
            const int q = rec % kRoughFlag;
            const bool rough = rec >= kRoughFlag;
            load_dx_down_to(max(t0 - (kWave - 1), 0));
            if (has_above && !load_lin_down_to(max(t0 - (kWave - 1), 0))) return false;
            if (t0 < m && t0 / CH != bin_chunk) load_bin(t0 / CH);
            if constexpr (P <= 12)
                segment_at_depth<0>(q, rough, t0, t1);
            else
                segment<-1, false>(q, rough, t0, t1);
            if (t0 < m && (t0 % CH) == 0) flush_cols(t0, min(t0 + CH, m));
        }
        // dL/d(dy_l) of this lane's row
        if (lane_ok) {
            double* gp = gyp + (int64_t)l * a.d;
#pragma unroll
            for (int ch = 0; ch < D; ++ch)
                if (ch < a.d) atomicAdd(&gp[ch], gy[ch]);
        }
        __syncthreads();
        return true;
    }
};

template <int P, int D>
__global__ void __launch_bounds__(kWave) bwd_kernel(BwdArgs b) {
    __shared__ LdsBwd<P, D> L;
    const FwdArgs& a = b.f;
    const int lane = lane_id();
    double* scratch = b.scratch + (int64_t)blockIdx.x * (2 * kCkptEvery * P * kWave);
    unsigned long long cells = 0, flops = 0;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(&a.hdr->ticket2, 1u);
        t = (unsigned)uniform((int)t);
        if ((int64_t)t >= b.ntickets) break;
        if (uniform((int)(load_status(a.hdr) & SIGK_ERR_WATCHDOG))) break;
        int pair, strip;
        Geo g;
        BlockRef r;
        if (a.mode == kModeTable) {
            pair = b.tickets[t].pair;
            strip = b.tickets[t].strip;
            if (pair < 0) break;  // unused slots close a table built on the device
            g = resolve(a, pair, P, 0);
        } else {
            // kModeBlock: the blocks of one anti-diagonal, strips top-down
            pair = (int)(t % (unsigned)a.blk.nb);
            strip = a.blk.kb - 1 - (int)(t / (unsigned)a.blk.nb);
            g = resolve_block(a, pair, P, r);
            if (strip * kWave >= g.n) continue;  // the top block row has fewer strips
        }
        StripBwd<P, D> S(b, g, L, strip);
        S.scr.init(scratch, 2 * kCkptEvery * P);
        S.cells = &cells;
        S.flops = &flops;
        S.ck = b.ckpt + g.ckpt + (int64_t)strip * ckpt_strip_doubles(g.m, P);
        S.ckq = S.ck + ckpt_states(g.m) * 2 * P * kWave;
        if (a.mode == kModeTable) {
            const PairDesc& pd = a.desc[pair];
            S.snap_in = b.snap + pd.snap_off + (int64_t)strip * g.m * P;
            S.lam_row = b.lam_front + pd.front_off;
            S.lam_prog = b.lam_prog + pd.prog_off;
            S.seed_scale = b.grad_out[pair];
            S.gxp = b.gdx + pd.x_off;
            S.gyp = b.gdx + pd.y_off;
        } else {
            const BlockGeo& k = a.blk;
            S.snap_in = (strip == 0 && r.bot) ? r.bot
                                              : b.snap + g.front + (int64_t)strip * g.m * P;
            S.lam_row = b.lam_front + (int64_t)r.J * k.cb * P;
            S.lam_prog = b.lam_prog + g.prog;
            // the grid's corner cell belongs to the top-right block
            S.seed_scale = (!r.above && !r.right) ? b.grad_out[0] : 0.0;
            S.gxp = b.gdx + (int64_t)r.J * k.cb * a.d;
            S.gyp = b.gdx + k.y_gdx + (int64_t)r.I * k.rb * a.d;
            S.left = r.left;
            S.below_line = r.bot != nullptr;
            S.above_blk = r.above;
            S.lamv = b.lam_v + (int64_t)r.I * k.rb * P;
            S.right_in = r.right;
            S.left_out = r.J > 0;
        }
        if (!S.sweep()) break;
    }
    if (lane == 0) {
        atomicAdd(&a.hdr->bwd_cells, cells);
        atomicAdd(&a.hdr->bwd_flops, flops);
    }
}

#define SIGK_CAT3(a, b, c) a##b##_##c
#define SIGK_NAME(pre, P, D) SIGK_CAT3(pre, P, D)

hipError_t SIGK_NAME(launch_ckpt_, SIGK_P, SIGK_D)(const FwdArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((ckpt_kernel<SIGK_P, SIGK_D>), dim3(grid), dim3(kWave), 0, s, a,
                       a.frontier);
    return hipGetLastError();
}

hipError_t SIGK_NAME(launch_lines_, SIGK_P, SIGK_D)(const FwdArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((lines_kernel<SIGK_P, SIGK_D>), dim3(grid), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

int SIGK_NAME(occupancy_lines_, SIGK_P, SIGK_D)() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lines_kernel<SIGK_P, SIGK_D>, kWave,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t SIGK_NAME(launch_bwd_, SIGK_P, SIGK_D)(const BwdArgs& b, int grid, hipStream_t s) {
    hipLaunchKernelGGL((bwd_kernel<SIGK_P, SIGK_D>), dim3(grid), dim3(kWave), 0, s, b);
    return hipGetLastError();
}

int SIGK_NAME(occupancy_ckpt_, SIGK_P, SIGK_D)() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ckpt_kernel<SIGK_P, SIGK_D>, kWave, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

int SIGK_NAME(occupancy_bwd_, SIGK_P, SIGK_D)() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bwd_kernel<SIGK_P, SIGK_D>, kWave, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace sigk
