// sigk_strip.h -- the forward wavefront sweep of one 64-row strip.
//
// Mapping (MI355X, one wavefront per strip).  Lane j owns grid row
// l = 64*s + j of strip s and processes cell (k, l) at step t = k + j, so the
// 64 lanes work on one anti-diagonal of the strip at a time (the topological
// order of the tile DAG, Sec. 2.2 and the anti-diagonal schedule of App. C).
// The left-edge series of a lane's current cell stays in its registers; the
// top-edge series it produces moves to lane j+1 for the next step by a DPP
// wave shift.  Lane 0 takes its bottom edge from the frontier row written by
// the strip below; lane 63 writes its top edge to the frontier for the strip
// above.  Frontier columns are exchanged between strips in chunks (32 or 64
// columns, a template parameter chosen per variant and sweep):
// lane 63's edges are staged in LDS and written out with device-coherent
// stores, followed by a progress flag per strip; the strip above polls the
// flag and reads the chunk with device-coherent loads (no cache maintenance).
//
// Cell map (Prop. 2.8 in the derivative basis).  With A the bottom-edge and B
// the left-edge series in unit-cell coordinates, f(u) = sum_i A_i u^i / i!,
// g(v) = sum_j B_j v^j / j!, A_0 the corner value (B_0 := A_0) and c the cell
// coefficient, the entries of C = A o B o W give
//     A'_i = sum_{n=0}^{i} e_n A_{i-n} + e_i * sum_{r>=1} B_r i!/(i+r)!
//     B'_j = sum_{n=0}^{j} e_n B_{j-n} + e_j * sum_{r>=1} A_r j!/(j+r)!
// with e_n = c^n/n!; A' is the top edge, B' the right edge.  The Hankel sums
// are evaluated in nested (Horner) form, which needs only the constants 1/k.
//
// Neumann depth.  Term n (the entries of C with min(i, j) = n, the n-th term
// of the series of Prop. 2.5) is bounded by |c|^n/(n!)^2 relative to the edge
// data.  It is applied while |c| may exceed tau_n = (tol (n!)^2)^(1/n)
// anywhere in the cells a chunk of steps covers, using the exact bound
// |c| = |<dx_k, dy_l>| <= |dx_k| |dy_l| (Cauchy-Schwarz).  The depth is
// therefore uniform over the wave and known before each chunk, so the step
// loop carries no data-dependent branch.
//
// Truncation estimate.  Keeping P coefficients per edge drops, in every cell,
// the coefficients of degree >= P of both output edges.  The first of them is
// led by c times the last kept coefficient of the input edge (the n = 1
// Toeplitz term of the map: A'_P = c A_{P-1} + ...), so a cell's local error is
// estimated as |c| (|A_{P-1}| + |B_{P-1}|) / P! relative to the local value of
// K (the local series error of the error analysis of App. C, taken at its
// leading term).  Local errors propagate with O(1) weight relative to K, so
// they are summed over every cell of the pair: each lane keeps a running sum
// over its cells; per chunk the wave adds the lanes' sums, each divided by
// max(1, |K|) of its row where the chunk starts or ends (the smaller), and
// each strip adds its share to the pair's total, which the host-side launch
// compares with the pair's budget (SIGK_WARN_TRUNC above it).
#pragma once
#include "sigk_device.h"

namespace sigk {

// Slot of column col in a ring of RB columns (col >= -RB).
template <int RB>
__device__ __forceinline__ int ring_slot_of(int col) {
    if constexpr ((RB & (RB - 1)) == 0)
        return col & (RB - 1);
    else
        return (int)((unsigned)(col + RB) % (unsigned)RB);
}

// The same for the adjoint's rings (ring_cols(P) columns).
template <int P>
__device__ __forceinline__ int ring_slot(int col) {
    return ring_slot_of<ring_cols(P)>(col);
}

// D > 0: the channel bucket (d <= D, increments in LDS and registers);
// D = 0: the cell coefficients come from a field computed beforehand.
template <int P, int D, int CH, int RB>
struct LdsStrip {
    static_assert(RB >= CH + kWave - 1,
                  "the ring must hold the columns a chunk's steps touch");
    // D > 0: increments of x, [channel][ring slot]; D = 0: the chunk's cell
    // coefficients, [step][lane] (no LDS beyond what D > 0 needs: every byte
    // more costs the order-5 kernel a wave per CU)
    // (bin first: its rows are then addressed from one register with the
    // instructions' immediate offsets)
    double bin[CH * P];   // bottom edges of the current chunk (lane 0)
    double tout[CH * P];  // top edges of the top lane, current chunk
    double dx[D > 0 ? D * RB : CH * kWave];
    float nrm2[D > 0 ? RB : 1];     // |dx_k|^2 of the same columns, rounded up
};

struct Acc {
    unsigned long long cells = 0, flops = 0;
    unsigned status = 0;
};

// Reciprocals 1/k, k = 0..2P (entry 0 unused).  For mid-size P they are pinned
// in vector registers (the wave runs alone on its SIMD there anyway), so the
// hot loop neither rebuilds them nor spills them from scalar registers; for
// small P the registers buy more occupancy instead.
template <int P, bool kPinVector = (P >= 10 && P <= 12)>
struct Recip {
    double v[2 * P + 1];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int k = 0; k <= 2 * P; ++k) {
            v[k] = k == 0 ? 0.0 : 1.0 / (double)k;
            if (kPinVector) asm volatile("" : "+v"(v[k]));
            else if (P <= 8 && k > 2) asm volatile("" : "+s"(v[k]));
        }
    }
    __device__ __forceinline__ double operator()(int k) const { return v[k]; }
};

// Algorithmic flops of one cell at edge order P, Neumann depth q, d channels
// (FMA = 2 flops):
//   n = 0 : two Horner edge evaluations, 2(P-2) FMA + 2 add       -> 4P - 6
//   n >= 1: e_n = c^n/n! (1 mul, none for n = 1), Toeplitz 2(P-n) FMA,
//           Horner sums 2(P-2) FMA, e_n/(n+1) (1 mul), 2 FMA       -> 8P - 4n - 2
//                                                            (n = 1: 8P - 7)
//   Delta : d FMA                                                  -> 2d
__host__ __device__ constexpr long long cell_flops(int P, int q, int d) {
    return 4LL * P - 6 + (long long)q * (8LL * P - 2) - 2LL * q * (q + 1) - (q > 0 ? 1 : 0) +
           2LL * d;
}

// Last edge coefficient r in the Hankel sum of output coefficient n.  The
// map keeps every product of a kept edge coefficient (r <= P-1); the square
// truncation (SQ) is the paper's fixed-order tile of App. C and
// Proposition A.3, which keeps only the entries C_ij with i, j <= N = P-1 of
// the tile matrix, i.e. n + r <= P-1.
template <int P, bool SQ>
__host__ __device__ constexpr int hankel_top(int n) {
    return SQ ? P - 1 - n : P - 1;
}

// sum_{r=1}^{top} V_r n!/(n+r)! without the leading 1/(n+1):
// V_1 + (1/(n+2)) [V_2 + (1/(n+3)) [V_3 + ...]] (Horner form), 0 if top < 1.
template <int P, int top, class RC>
__device__ __forceinline__ double hankel_horner(const double (&V)[P], int n, const RC& R) {
    if constexpr (top < 1) {
        return 0.0;
    } else {
        double t = V[top];
#pragma unroll
        for (int r = top - 1; r >= 1; --r) t = fma(t, R(n + r + 1), V[r]);
        return t;
    }
}

// Neumann term N of the cell map (Toeplitz part and Horner-form Hankel part),
// then the following terms while N < q.  ep = c^(N-1)/N! from the previous
// term (1 for N = 1), so e_N = ep c and e_N/(N+1) = e_N (1/(N+1)).  Written
// as a compile-time recursion so that every coefficient index is a constant
// (registers, never scratch).
template <int P, int N, bool SQ = false, class RC>
__device__ __forceinline__ void neumann_terms(const double (&A)[P], const double (&B)[P],
                                              double c, double ep, double (&An)[P],
                                              double (&Bn)[P], int q, const RC& R) {
    if constexpr (N < P) {
        if (N > q) return;  // scalar, uniform (folds away for a constant q)
        const double e = N == 1 ? c : ep * c;
#pragma unroll
        for (int i = N; i < P; ++i) {
            An[i] = fma(e, A[i - N], An[i]);
            Bn[i] = fma(e, B[i - N], Bn[i]);
        }
        // sum_{r>=1} B_r N!/(N+r)! = (1/(N+1)) [B_1 + (1/(N+2)) [B_2 + ...]]
        constexpr int top = hankel_top<P, SQ>(N);
        const double tb = hankel_horner<P, top>(B, N, R);
        const double ta = hankel_horner<P, top>(A, N, R);
        const double en = e * R(N + 1);
        if constexpr (top >= 1) {
            An[N] = fma(en, tb, An[N]);
            Bn[N] = fma(en, ta, Bn[N]);
        }
        neumann_terms<P, N + 1, SQ>(A, B, c, en, An, Bn, q, R);
    }
}

// The truncated cell map with Neumann depth q (wave-uniform, q <= P-1).
template <int P, bool SQ = false, class RC>
__device__ __forceinline__ void cell_map(const double (&A)[P], double (&B)[P], double c,
                                         double (&An)[P], double (&Bn)[P], int q,
                                         const RC& R) {
    B[0] = A[0];
    // n = 0: corner values from the edges, sum_{r>=1} B_r/r! and sum A_r/r!
    {
        double tb = B[P - 1], ta = A[P - 1];
#pragma unroll
        for (int r = P - 2; r >= 1; --r) {
            tb = fma(tb, R(r + 1), B[r]);
            ta = fma(ta, R(r + 1), A[r]);
        }
        An[0] = A[0] + tb;
        Bn[0] = A[0] + ta;
    }
#pragma unroll
    for (int i = 1; i < P; ++i) {
        An[i] = A[i];
        Bn[i] = B[i];
    }
    neumann_terms<P, 1, SQ>(A, B, c, 1.0, An, Bn, q, R);
}

// The same map for a compile-time depth Q, in two phases: first everything
// that needs only the left edge B and c (powers of c, the Hankel sums over B,
// the Toeplitz terms of B' that do not involve B_0), then the parts that need
// the bottom edge A (B_0 := A_0).  The first phase covers the latency of the
// cross-lane move and LDS read that deliver A.  Every sum accumulates in the
// same order as in cell_map.
template <int P, int Q, bool SQ = false>
struct SplitMap {
    double e[Q + 1], en[Q + 1], tb[Q + 1];

    template <class RC>
    __device__ __forceinline__ void pre(const double (&B)[P], double c, double (&Bn)[P],
                                        const RC& R) {
#pragma unroll
        for (int n = 0; n <= Q; ++n) {
            if (n > 0) {
                e[n] = n == 1 ? c : en[n - 1] * c;
                en[n] = e[n] * R(n + 1);
            }
            const int top = hankel_top<P, SQ>(n);
            double t = top >= 1 ? B[top >= 1 ? top : 1] : 0.0;
#pragma unroll
            for (int r = top - 1; r >= 1; --r) t = fma(t, R(n + r + 1), B[r]);
            tb[n] = t;
        }
#pragma unroll
        for (int i = 1; i < P; ++i) Bn[i] = B[i];
#pragma unroll
        for (int n = 1; n <= Q; ++n)
#pragma unroll
            for (int i = n + 1; i < P; ++i) Bn[i] = fma(e[n], B[i - n], Bn[i]);
    }

    template <class RC>
    __device__ __forceinline__ void post(const double (&A)[P], double (&An)[P], double (&Bn)[P],
                                         const RC& R) {
#pragma unroll
        for (int i = 1; i < P; ++i) An[i] = A[i];
#pragma unroll
        for (int n = 1; n <= Q; ++n) {
#pragma unroll
            for (int i = n; i < P; ++i) An[i] = fma(e[n], A[i - n], An[i]);
            Bn[n] = fma(e[n], A[0], Bn[n]);
        }
        double t = A[P - 1];
#pragma unroll
        for (int r = P - 2; r >= 1; --r) t = fma(t, R(r + 1), A[r]);
        An[0] = A[0] + tb[0];
        Bn[0] = A[0] + t;
#pragma unroll
        for (int n = 1; n <= Q; ++n) {
            const int top = hankel_top<P, SQ>(n);
            if (top < 1) continue;
            double ta = A[top >= 1 ? top : 1];
#pragma unroll
            for (int r = top - 1; r >= 1; --r) ta = fma(ta, R(n + r + 1), A[r]);
            An[n] = fma(en[n], tb[n], An[n]);
            Bn[n] = fma(en[n], ta, Bn[n]);
        }
    }
};

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// A value equal in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/P!
template <int P>
__host__ __device__ constexpr double inv_factorial() {
    double f = 1.0;
    for (int i = 2; i <= P; ++i) f /= (double)i;
    return f;
}

// Copy of P doubles between registers and 16-byte aligned LDS rows, in
// 16-byte accesses where P is even.
template <int P>
__device__ __forceinline__ void lds_copy(double* dst, const double* src) {
    if constexpr (P % 2 == 0) {
#pragma unroll
        for (int i = 0; i < P; i += 2) {
            const double2 v = *(const double2*)(src + i);
            *(double2*)(dst + i) = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < P; ++i) dst[i] = src[i];
    }
}

// CH: columns per frontier chunk; RB: columns of the increment ring; SQ:
// square truncation of the tile matrix (the paper's fixed-order tile); BLK:
// the boundary hooks of block checkpointing (left edges from a line, a bottom
// line for strip 0, right-edge lines written during the sweep).
template <int P, int D, int CH, int RB, bool SQ = false, bool BLK = false>
struct StripCtx {
    const FwdArgs& a;
    Geo& g;
    LdsStrip<P, D, CH, RB>& L;
    Acc& acc;
    int s;              // strip index
    int nrows;          // valid rows in this strip (<= 64)
    bool lane_ok;
    bool has_below, has_above;
    const double* Fin;  // frontier row read by lane 0 ([m][P])
    double* Fout;       // frontier row written by lane 63
    int* prog;          // progress counters of the pair
    double B[P];        // left-edge series of the lane's current cell
    double Ac[P];       // top-edge series produced at the previous step
    double dy[D > 0 ? D : 1];
    double cn;          // cell coefficient of the next step
    double dymax2;      // max_l |dy_l|^2 over the strip
    int q;              // Neumann depth of the current chunk
    unsigned nvalid;
    Recip<P> R;
    int pair;           // pair index (truncation estimate slot)
    int tload;          // chunks are loaded for steps below this (m; D = 0: all steps)
    // truncation estimate: sum of |c| (|A_{P-1}| + |B_{P-1}|) over the lane's
    // cells of the current chunk, the wave's total of the chunks done, each
    // relative to the local size of K (wave-uniform), and the binary exponent
    // of |K| where the lane's current chunk started
    double tacc, etot;
    int kexp;
    // checkpointing (adjoint support)
    double* ck;         // wave-state checkpoints of this strip or null
    double* ckq;        // Neumann depth per chunk (with ck)
    int ck_every;
    // block checkpointing (BLK): left edges of the strip's rows at column 0
    // (null: the axis), whether strip 0 reads a bottom line through Fin, and
    // the right-edge lines of the block columns (null: none written)
    const double* left = nullptr;
    bool below_line = false;
    double* vl = nullptr;
    int vnext = 0;  // step at which lane 0 reaches the last column of its block column

    __device__ StripCtx(const FwdArgs& a_, Geo& g_, LdsStrip<P, D, CH, RB>& L_, Acc& acc_, int s_)
        : a(a_), g(g_), L(L_), acc(acc_), s(s_) {}

    // One cell's local truncation estimate from its input edges (one FMA per
    // edge, placed where that edge is available).
    __device__ __forceinline__ void tally(double c, const double (&E)[P]) {
        tacc = fma(fabs(c), fabs(E[P - 1]), tacc);
    }
    // Close the current chunk's sum, relative to the local size of K: per
    // row, the smaller |K| of where the chunk started and where it ends (K is
    // the left edge's constant term), taken as the power of two at or below
    // it, at least 1.
    __device__ __forceinline__ void fold() {
        const double k1 = fabs(B[0]);
        const int e1 = k1 >= 1.0 && k1 <= 1.7e308 ? ilogb(k1) : 0;  // 0 also for NaN
        etot = uniform_d(etot + wave_sum(ldexp(tacc, -min(kexp, e1))));
        kexp = e1;
        tacc = 0.0;
    }

    // Bottom edges of columns [c0, c0+nc) from the strip below, once it has
    // published them.
    __device__ bool load_frontier(int c0, int nc) {
        const int lane = lane_id();
        if (!wait_flag(&prog[s - 1], c0 + nc, a.hdr, a.watchdog_ticks)) return false;
        constexpr int NB = (CH * P + kWave - 1) / kWave;
        const CoherentSpan src(Fin + (int64_t)c0 * P, nc * P);
        double bv[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) bv[k] = src.load(lane + k * kWave);
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (lane + k * kWave < nc * P) L.bin[lane + k * kWave] = bv[k];
        return true;
    }

    // Depth of the chunk from the bound of |c|^2 over its cells.  With
    // checkpoints, the depth is stored for the adjoint together with a flag
    // (+kRoughFlag) where the bound allows |c| > 1/2: there the adjoint keeps
    // each cell's left edge instead of recovering it from the right edge (the
    // recovery inverts a triangular Toeplitz factor of norm up to e^|c| per
    // step and loses precision over a segment for |c| of order 1 and above).
    __device__ __forceinline__ void set_depth(int c0, double cmax2) {
        int qq = 0;
#pragma unroll
        for (int n = 1; n < P; ++n) qq = cmax2 > a.tau2[n] ? n : qq;
        q = uniform(qq);
        if (ckq && lane_id() == 0)
            ckq[c0 / CH] = (double)(q + (cmax2 > kRoughC2 ? kRoughFlag : 0));
    }

    // D = 0: the coefficients of steps [c0, c0+CH) from the precomputed field
    // into LDS (lane j reads and later uses only its own row's cells: no
    // exchange between lanes), cells outside the grid as 0; the depth from
    // their exact maximum; the frontier as for D > 0.
    __device__ bool load_chunk_field(int c0) {
        const int lane = lane_id();
        const double* src =
            a.delta + g.delta + ((int64_t)s * delta_steps(g.m) + c0) * kWave + lane;
        double cm = 0.0;
        constexpr int NB = 16;
#pragma unroll
        for (int k0 = 0; k0 < CH; k0 += NB) {
            double v[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) v[k] = src[(int64_t)(k0 + k) * kWave];  // t < delta_steps
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int col = c0 + k0 + k - lane;
                const double c = (lane_ok && col >= 0 && col < g.m) ? v[k] : 0.0;
                L.dx[(k0 + k) * kWave + lane] = c;
                cm = fmax(cm, fabs(c));
            }
        }
        if (c0 < g.m && has_below && !load_frontier(c0, min(CH, g.m - c0))) return false;
        __syncthreads();
        const double cmax = wave_max(cm);
        set_depth(c0, cmax * cmax);
        return true;
    }

    // Load columns [c0, c0+CH) (increments, their norms, bottom edges) and set
    // the Neumann depth for steps [c0, c0+CH).
    __device__ bool load_chunk(int c0) {
        if constexpr (D == 0) return load_chunk_field(c0);
        const int lane = lane_id();
        const int nc = min(CH, g.m - c0);
        // Issue every load before the first wait: the path points of the
        // chunk's columns (lane j: column c0 + j, clamped to the chunk), then
        // the frontier columns once the strip below has published them.
        const int col = c0 + min(lane, nc - 1);
        const double* xp = g.x + (int64_t)col * a.d;
        double lo[D > 0 ? D : 1], hi[D > 0 ? D : 1];
#pragma unroll
        for (int ch = 0; ch < D; ++ch) {
            const int cc = ch < a.d ? ch : 0;
            lo[ch] = xp[cc];
            hi[ch] = xp[a.d + cc];
        }
        if (has_below && !load_frontier(c0, nc)) return false;
        if (lane < nc) {
            double n2 = 0.0;
#pragma unroll
            for (int ch = 0; ch < D; ++ch) {
                const double v = ch < a.d ? hi[ch] - lo[ch] : 0.0;
                L.dx[ch * RB + ring_slot_of<RB>(col)] = v;
                n2 = fma(v, v, n2);
            }
            // stored as a float no smaller than n2 (relative slack above the
            // float rounding, floor at the smallest normal float)
            L.nrm2[ring_slot_of<RB>(col)] =
                (float)fmax(n2 * (1.0 + 1e-6), n2 > 0.0 ? 1.2e-38 : 0.0);
        }
        __syncthreads();
        // columns touched by steps [c0, c0+CH): [c0-63, c0+nc)
        double w = 0.0;
        const int k1 = c0 - (kWave - 1) + lane, k2 = c0 + lane;
        if (k1 >= 0 && k1 < c0 + nc) w = (double)L.nrm2[ring_slot_of<RB>(k1)];
        if (lane < nc) w = fmax(w, (double)L.nrm2[ring_slot_of<RB>(k2)]);
        set_depth(c0, wave_max(w) * dymax2);
        return true;
    }

    // The top lane has produced columns [c0, c1) (staged in LDS): write them
    // to the frontier with coalesced device-coherent stores and publish.
    __device__ void flush(int c0, int c1) {
        double* dst = Fout + (int64_t)c0 * P;
        const int base = (c0 % CH) * P;
        for (int e = lane_id(); e < (c1 - c0) * P; e += kWave) store_coherent(&dst[e], L.tout[base + e]);
        publish_coherent(&prog[s], c1);
    }

    __device__ void save_state(int t) {
        // wave state before step t: (B, Ac) of every lane, layout [2P][64]
        double* dst = ck + (int64_t)(t / ck_every) * (2 * P * kWave);
        const int lane = lane_id();
#pragma unroll
        for (int i = 0; i < P; ++i) {
            dst[i * kWave + lane] = B[i];
            dst[(P + i) * kWave + lane] = Ac[i];
        }
    }

    // After the cell of column col (BLK, with vl): at the last column of a
    // block column (except the grid's last) keep the cell's right edge.
    __device__ __forceinline__ void vline_hook(int t, int col, bool act) {
        if (vl == nullptr) return;
        const int cb = a.blk.cb;
        bool mine;
        if (cb >= kWave) {
            // at most one lane per step, in the 64 steps after lane 0 reaches
            // the last column of a block column: a uniform test per step
            const int w = t - vnext;
            if ((unsigned)w >= (unsigned)kWave) return;
            if (w == kWave - 1) vnext += cb;
            mine = lane_id() == w;
        } else {
            mine = (col + 1) % cb == 0;
        }
        if (mine && act && col + 1 < g.m) {
            const int J = (col + 1) / cb;
            double* dst =
                vl + ((int64_t)(J - 1) * a.blk.n + (int64_t)s * kWave + lane_id()) * P;
#pragma unroll
            for (int i = 0; i < P; ++i) dst[i] = B[i];
        }
    }

    // Cell coefficient c = <dx_col, dy_row> of step t into cn.  For small
    // orders it is computed one step ahead so that the LDS latency of the
    // increments overlaps the cell map (several waves share a SIMD there and
    // registers allow it).  Every ring slot read is inside the LDS array for
    // any t; where step t starts a new chunk the value read ahead is stale and
    // is recomputed after load_chunk().
    static constexpr bool kAhead = P <= 8;
    __device__ __forceinline__ void prefetch(int t) {
        if constexpr (D == 0) {
            cn = L.dx[((unsigned)t % (unsigned)CH) * kWave + lane_id()];
            return;
        }
        const int ri = ring_slot_of<RB>(t - lane_id());
        double c0 = 0.0, c1 = 0.0;
#pragma unroll
        for (int ch = 0; ch < D; ch += 2) {
            c0 = fma(dy[ch], L.dx[ch * RB + ri], c0);
            c1 = fma(dy[ch + 1], L.dx[(ch + 1) * RB + ri], c1);
        }
        cn = c0 + c1;
    }

    // One step: every lane advances one cell along its row.  QC >= 0 fixes the
    // Neumann depth at compile time (QC == q), QC < 0 reads q.
    template <bool EDGE, int QC>
    __device__ __forceinline__ void step(int t, bool act) {
        const int lane = lane_id();
        const int col = t - lane;
        double A[P];
        const double* bsrc = &L.bin[((unsigned)t % (unsigned)CH) * P];  // t >= 0
        if constexpr (!EDGE && QC >= 0 && P <= 12) {
            // steady state, depth known at compile time: B-only work first
            double bv[P];
            lds_copy<P>(bv, bsrc);
            double c;
            double dxv[kAhead && D > 0 ? D : 1];
            if constexpr (kAhead && D == 0) {
                // the next step's coefficient (stale past the chunk's end: it
                // is read again after the next chunk is loaded)
                c = cn;
                cn = L.dx[((unsigned)(t + 1) % (unsigned)CH) * kWave + lane];
            } else if constexpr (kAhead) {
                // increments of the next step's column, consumed after the map
                c = cn;
                if constexpr ((RB & (RB - 1)) == 0) {
                    // byte offset of the slot: a uniform step part minus a
                    // lane part, masked (two vector instructions)
                    const unsigned off = ((unsigned)(t + 1) * 8u - (unsigned)lane * 8u) &
                                         (unsigned)((RB - 1) * 8);
                    const char* base = (const char*)L.dx + off;
#pragma unroll
                    for (int ch = 0; ch < D; ++ch)
                        dxv[ch] = *(const double*)(base + (size_t)ch * RB * 8);
                } else {
                    const int ri = ring_slot_of<RB>(t + 1 - lane);
#pragma unroll
                    for (int ch = 0; ch < D; ++ch) dxv[ch] = L.dx[ch * RB + ri];
                }
            } else {
                prefetch(t);
                c = cn;
            }
            double An[P], Bn[P];
            SplitMap<P, QC, SQ> S;
            S.pre(B, c, Bn, R);
            tally(c, B);  // every lane: rows past the grid have c = 0
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < P; ++i) A[i] = shift_up(Ac[i], bv[i]);
            S.post(A, An, Bn, R);
            tally(c, A);
            if constexpr (kAhead && D > 0) {
                __builtin_amdgcn_sched_barrier(0);
                double c0 = 0.0, c1 = 0.0;
#pragma unroll
                for (int ch = 0; ch < D; ch += 2) {
                    c0 = fma(dy[ch], dxv[ch], c0);
                    c1 = fma(dy[ch + 1], dxv[ch + 1], c1);
                }
                cn = c0 + c1;
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
                B[i] = Bn[i];
                Ac[i] = An[i];
            }
            if constexpr (BLK) vline_hook(t, col, act);
            if (has_above && lane == kWave - 1 && act) {
                // the top lane's column t - 63, a uniform address
                const unsigned tc = (unsigned)(t - (kWave - 1));
                double* dst = &L.tout[(tc % (unsigned)CH) * P];
                lds_copy<P>(dst, An);
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) A[i] = shift_up(Ac[i], bsrc[i]);
        if (EDGE && col == 0) {
            bool axis = true;
            if constexpr (BLK) {
                if (left != nullptr && lane_ok) {
                    const double* lp = left + ((int64_t)s * kWave + lane) * P;
#pragma unroll
                    for (int i = 0; i < P; ++i) B[i] = lp[i];
                    axis = false;
                }
            }
            if (axis) {
#pragma unroll
                for (int i = 0; i < P; ++i) B[i] = i == 0 ? 1.0 : 0.0;
            }
        }
        // small orders: coefficient computed one step ahead; large orders
        // (one wave per SIMD, registers scarce): computed here
        double c;
        if constexpr (kAhead) {
            c = cn;
            prefetch(t + 1);
        } else {
            prefetch(t);
            c = cn;
        }
        // at the ramps, lanes outside the grid hold stale values: skip them
        if (!EDGE || act) {
            tally(c, A);
            tally(c, B);
        }
        double An[P], Bn[P];
        cell_map<P, SQ>(A, B, c, An, Bn, QC >= 0 ? QC : q, R);
#pragma unroll
        for (int i = 0; i < P; ++i) {
            B[i] = Bn[i];
            Ac[i] = An[i];
        }
        if constexpr (BLK) vline_hook(t, col, act);
        if (has_above && lane == kWave - 1 && act) {
            double* dst = &L.tout[((unsigned)col % (unsigned)CH) * P];
#pragma unroll
            for (int i = 0; i < P; ++i) dst[i] = An[i];
        }
    }

    // Steady-state steps [t, te) at the chunk's depth q.  For small orders the
    // depth is dispatched to a loop specialised for it (no branch per term).
    template <int QD>
    __device__ __forceinline__ void run_depth(int& t, int te) {
        if constexpr (QD < P - 1) {
            if (q > QD) {
                run_depth<QD + 1>(t, te);
                return;
            }
        }
        constexpr int QC = QD;
        for (; t < te; ++t) {
            if (ck && ((unsigned)t % (unsigned)ck_every) == 0) save_state(t);
            step<false, QC>(t, lane_ok);
        }
    }

    template <bool EDGE>
    __device__ bool run(int t0, int t1) {
        const int lane = lane_id();
        const int m = g.m;
        int t = t0;
        while (t < t1) {
            if ((t % CH) == 0 && t < tload) {
                fold();
                if (!load_chunk(t)) return false;
                if (kAhead) prefetch(t);
            }
            // steps up to the next chunk boundary, flush point or range end
            int te = min(t1, t - (t % CH) + CH);
            if (has_above) {
                // the top lane finishes column tc at step tc + 63
                const int tc = t - (kWave - 1);
                const int nxt = tc < 0 ? CH - 1 : tc - (tc % CH) + CH - 1;
                te = min(te, min(nxt, m - 1) + kWave);
            }
            if (ck) te = min(te, t - (t % ck_every) + ck_every);
            const long long fl = cell_flops(P, q, D > 0 ? a.d : 0);  // D = 0: counted by the field
            if (EDGE) {
                for (; t < te; ++t) {
                    if (ck && ((unsigned)t % (unsigned)ck_every) == 0) save_state(t);
                    const int col = t - lane;
                    const bool act = lane_ok && col >= 0 && col < m;
                    const unsigned cnt = (unsigned)__builtin_popcountll(ballot(act));
                    acc.cells += cnt;
                    acc.flops += (unsigned long long)cnt * (unsigned long long)fl;
                    step<true, -1>(t, act);
                }
            } else {
                const int n = te - t;
                acc.cells += (unsigned long long)n * nvalid;
                acc.flops += (unsigned long long)n * nvalid * (unsigned long long)fl;
                run_depth<0>(t, te);
            }
            if (has_above) {
                const int tc = t - 1 - (kWave - 1);
                if (tc >= 0 && tc < m && ((tc % CH) == CH - 1 || tc == m - 1))
                    flush(tc - tc % CH, tc + 1);
            }
        }
        return true;
    }

    // Sweep the whole strip.  Returns false if abandoned (watchdog).
    __device__ bool sweep() {
        const int lane = lane_id();
        const int m = g.m;
        const int row0 = s * kWave;
        nrows = min(kWave, g.n - row0);
        lane_ok = lane < nrows;
        has_below = s > 0 || (BLK && below_line);
        has_above = row0 + kWave < g.n;
        nvalid = (unsigned)nrows;
        if constexpr (BLK) {
            vnext = a.blk.cb - 1;
        }
        R.init();
        const int l = row0 + lane;
        double n2 = 0.0;
#pragma unroll
        for (int ch = 0; ch < D; ++ch) {
            dy[ch] = (ch < a.d && lane_ok)
                         ? g.y[(int64_t)(l + 1) * a.d + ch] - g.y[(int64_t)l * a.d + ch]
                         : 0.0;
            n2 = fma(dy[ch], dy[ch], n2);
        }
        dymax2 = wave_max(n2);
        tload = D == 0 ? m + nrows - 1 : m;
        q = P - 1;
        tacc = 0.0;
        etot = 0.0;
        kexp = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            B[i] = i == 0 ? 1.0 : 0.0;
            Ac[i] = B[i];
        }
        if (!has_below) {
            // bottom row of the grid: K = 1 on the axis t = 0
                for (int e = lane; e < CH * P; e += kWave) L.bin[e] = (e % P) == 0 ? 1.0 : 0.0;
            __syncthreads();
        }
        const int T = m + nrows - 1;
        const int tA = min(T, kWave);
        if (!run<true>(0, tA)) return false;
        if (m > kWave && !run<false>(kWave, m)) return false;
        if (!run<true>(max(tA, m), T)) return false;
        if (ck && (T % ck_every) == 0) save_state(T);
        // the strip's share of the pair's truncation estimate
        fold();
        const double est = etot * inv_factorial<P>();
        if (!isfinite(est)) acc.status |= SIGK_WARN_NONFINITE;
        if (lane == 0 && a.trunc_est) atomicAdd(&a.trunc_est[pair], est);
        if (!has_above) {
            // the last row's lane holds the top edge of the corner cell
            const bool mine = lane == nrows - 1;
            double k = 0.0, f = 1.0;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                k = fma(Ac[i], f, k);
                f = f / (double)(i + 1);
            }
            if (ballot(mine && !isfinite(k))) acc.status |= SIGK_WARN_NONFINITE;
            if (mine && a.out) {
                a.out[g.o1] = k;
                if (g.o2 >= 0) a.out[g.o2] = k;
            }
        }
        __syncthreads();
        return true;
    }
};

}  // namespace sigk
