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
// above.  Frontier columns are exchanged between strips in chunks through
// LDS with one release/acquire progress counter per strip.
//
// Cell map (Prop. 2.8 in the derivative basis).  With A the bottom-edge and B
// the left-edge series in unit-cell coordinates, f(u) = sum_i A_i u^i / i!,
// g(v) = sum_j B_j v^j / j!, A_0 the corner value (B_0 := A_0) and c the cell
// coefficient, the entries of C = A o B o W give
//     A'_i = sum_{n=0}^{i} e_n A_{i-n} + e_i * sum_{r>=1} B_r i!/(i+r)!
//     B'_j = sum_{n=0}^{j} e_n B_{j-n} + e_j * sum_{r>=1} A_r j!/(j+r)!
// with e_n = c^n/n!; A' is the top edge, B' the right edge.  Neumann term n
// (the entries of C with min(i, j) = n, i.e. the n-th term of the series of
// Prop. 2.5) is applied only while some lane of the wave has
// |c|^n/(n!)^2 > tol, the bound of that term relative to the edge data.
#pragma once
#include "sigk_device.h"

namespace sigk {

template <int P, int D>
struct LdsStrip {
    double dx[D * kRing];                // increments of x, [channel][column mod 128]
    double bin[chunk_cols(P) * P];       // bottom edges of the current chunk (lane 0)
    double tout[chunk_cols(P) * P];      // top edges of the top lane, current chunk
};

struct Acc {
    unsigned long long cells = 0, flops = 0;
    unsigned status = 0;
};

// The truncated cell map.  Returns the Neumann depth applied (wave-uniform).
// `live` is the mask of lanes whose cells are real (others carry garbage).
template <int P>
__device__ __forceinline__ int cell_map(const double (&A)[P], double (&B)[P], double c,
                                        double (&An)[P], double (&Bn)[P], double tol,
                                        uint64_t live) {
    B[0] = A[0];
    An[0] = A[0];
    Bn[0] = A[0];
#pragma unroll
    for (int r = 1; r < P; ++r) {
        An[0] = fma(ifact(r), B[r], An[0]);
        Bn[0] = fma(ifact(r), A[r], Bn[0]);
    }
#pragma unroll
    for (int i = 1; i < P; ++i) {
        An[i] = A[i];
        Bn[i] = B[i];
    }
    double e = 1.0;
    int q = 0;
#pragma unroll
    for (int n = 1; n < P; ++n) {
        e = e * c * (1.0 / (double)n);
        // bound of Neumann term n relative to the edge data: |c|^n / (n!)^2
        const double bound = fabs(e) * ifact(n);
        if ((__builtin_amdgcn_fcmp(bound, tol, 2 /* ordered greater */) & live) == 0) break;
        q = n;
#pragma unroll
        for (int i = n; i < P; ++i) {
            An[i] = fma(e, A[i - n], An[i]);
            Bn[i] = fma(e, B[i - n], Bn[i]);
        }
        double hb = 0.0, ha = 0.0;
#pragma unroll
        for (int r = 1; r < P; ++r) {
            hb = fma(hank(n, r), B[r], hb);
            ha = fma(hank(n, r), A[r], ha);
        }
        An[n] = fma(e, hb, An[n]);
        Bn[n] = fma(e, ha, Bn[n]);
    }
    return q;
}

__host__ __device__ constexpr long long cell_flops_q(int P, int q, int d) {
    // closed form of cell_flops: 4(P-1) + sum_{n=1..q} (8P - 4n + 2) + 2d
    return 4LL * (P - 1) + (long long)q * (8LL * P + 2) - 2LL * q * (q + 1) + 2LL * d;
}
static_assert(cell_flops_q(8, 5, 3) == cell_flops(8, 5, 3), "flop formula");

// Edge-series tail check: last coefficient's weight against the edge norm.
template <int P>
__device__ __forceinline__ void tail_check(const double* v, double tail_tol, bool act,
                                           unsigned& status) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) s = fma(fabs(v[i]), ifact(i), s);
    const double tail = fabs(v[P - 1]) * ifact(P - 1);
    const bool bad_t = act && (tail > tail_tol * s);
    const bool bad_n = act && !isfinite(s);
    if (ballot(bad_t)) status |= SIGK_WARN_TRUNC;
    if (ballot(bad_n)) status |= SIGK_WARN_NONFINITE;
}

template <int P, int D>
struct StripCtx {
    const FwdArgs& a;
    Geo& g;
    LdsStrip<P, D>& L;
    Acc& acc;
    int s;            // strip index
    int nrows;        // valid rows in this strip (<= 64)
    bool lane_ok;
    bool has_below, has_above;
    const double* Fin;  // frontier row read by lane 0 ([m][P])
    double* Fout;       // frontier row written by lane 63
    int* prog;          // progress counters of the pair
    double B[P];        // left-edge series of the lane's current cell
    double Ac[P];       // top-edge series produced at the previous step
    double dy[D];
    unsigned nvalid;
    uint64_t okmask;   // lanes holding a grid row
    // checkpointing (adjoint support)
    double* ck;         // wave-state checkpoints of this strip or null
    int ck_every;

    __device__ StripCtx(const FwdArgs& a_, Geo& g_, LdsStrip<P, D>& L_, Acc& acc_, int s_)
        : a(a_), g(g_), L(L_), acc(acc_), s(s_) {}

    __device__ bool load_chunk(int c0) {
        const int lane = lane_id();
        const int CH = chunk_cols(P);
        const int nc = min(CH, g.m - c0);
        if (has_below) {
            if (!wait_at_least(&prog[s - 1], c0 + nc, a.hdr, a.watchdog_ticks)) return false;
            const double* src = Fin + (int64_t)c0 * P;
            for (int e = lane; e < nc * P; e += kWave) L.bin[e] = src[e];
        }
        if (lane < nc) {
            const int col = c0 + lane;
            const double* xp = g.x + (int64_t)col * a.d;
#pragma unroll
            for (int ch = 0; ch < D; ++ch)
                L.dx[ch * kRing + (col & (kRing - 1))] =
                    ch < a.d ? xp[a.d + ch] - xp[ch] : 0.0;
        }
        __syncthreads();
        return true;
    }

    __device__ void flush(int c0, int c1) {
        const int lane = lane_id();
        __syncthreads();
        const int nc = c1 - c0;
        double* dst = Fout + (int64_t)c0 * P;
        for (int e = lane; e < nc * P; e += kWave) dst[e] = L.tout[e];
        tail_check<P>(&L.tout[(lane < nc ? lane : 0) * P], a.tail_tol, lane < nc, acc.status);
        publish(&prog[s], c1);
        __syncthreads();
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

    template <bool EDGE>
    __device__ bool run(int t0, int t1) {
        const int lane = lane_id();
        const int CH = chunk_cols(P);
        const int m = g.m;
        for (int t = t0; t < t1; ++t) {
            if ((t % CH) == 0 && t < m) {
                if (!load_chunk(t)) return false;
                if (t > 0) tail_check<P>(B, a.tail_tol, lane_ok && t - lane > 0 && t - lane <= m,
                                         acc.status);
            }
            if (ck && (t % ck_every) == 0) save_state(t);
            const int col = t - lane;
            const bool act = EDGE ? (lane_ok && col >= 0 && col < m) : lane_ok;
            const uint64_t live = EDGE ? ballot(act) : okmask;
            double A[P];
            const double* bsrc = &L.bin[(t % CH) * P];
#pragma unroll
            for (int i = 0; i < P; ++i) A[i] = shift_up(Ac[i], bsrc[i]);
            if (EDGE && col == 0) {
#pragma unroll
                for (int i = 0; i < P; ++i) B[i] = i == 0 ? 1.0 : 0.0;
            }
            const int ri = col & (kRing - 1);
            double c = 0.0;
#pragma unroll
            for (int ch = 0; ch < D; ++ch) c = fma(dy[ch], L.dx[ch * kRing + ri], c);
            double An[P], Bn[P];
            const int q = cell_map<P>(A, B, c, An, Bn, a.tol, live);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                B[i] = Bn[i];
                Ac[i] = An[i];
            }
            const unsigned cnt = EDGE ? (unsigned)__builtin_popcountll(live) : nvalid;
            acc.cells += cnt;
            acc.flops += (unsigned long long)cnt * (unsigned long long)cell_flops_q(P, q, a.d);
            if (has_above) {
                if (lane == kWave - 1 && act) {
#pragma unroll
                    for (int i = 0; i < P; ++i) L.tout[(col % CH) * P + i] = An[i];
                }
                const int tc = t - (kWave - 1);
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
        has_below = s > 0;
        has_above = row0 + kWave < g.n;
        nvalid = (unsigned)nrows;
        okmask = ballot(lane_ok);
        const int l = row0 + lane;
#pragma unroll
        for (int ch = 0; ch < D; ++ch)
            dy[ch] = (ch < a.d && lane_ok)
                         ? g.y[(int64_t)(l + 1) * a.d + ch] - g.y[(int64_t)l * a.d + ch]
                         : 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            B[i] = i == 0 ? 1.0 : 0.0;
            Ac[i] = B[i];
        }
        if (!has_below) {
            // bottom row of the grid: K = 1 on the axis t = 0
            const int CH = chunk_cols(P);
            for (int e = lane; e < CH * P; e += kWave) L.bin[e] = (e % P) == 0 ? 1.0 : 0.0;
            __syncthreads();
        }
        const int T = m + nrows - 1;
        const int tA = min(T, kWave);
        if (!run<true>(0, tA)) return false;
        if (m > kWave && !run<false>(kWave, m)) return false;
        if (!run<true>(max(tA, m), T)) return false;
        if (ck && (T % ck_every) == 0) save_state(T);
        if (!has_above) {
            // the last row's lane holds the top edge of the corner cell
            const bool mine = lane == nrows - 1;
            tail_check<P>(Ac, a.tail_tol, mine, acc.status);
            if (mine) {
                double k = 0.0;
#pragma unroll
                for (int i = P - 1; i >= 0; --i) k = fma(Ac[i], ifact(i), k);
                a.out[g.o1] = k;
                if (g.o2 >= 0) a.out[g.o2] = k;
            }
        }
        __syncthreads();
        return true;
    }
};

}  // namespace sigk
