// sigk_adjoint.h -- reverse (adjoint) wavefront sweep of one 64-row strip.
//
// The forward cell map is linear in the edge data:
//     A'_i = sum_{n<=min(i,q)} e_n A_{i-n} + [i<=q] e_i hB_i,
//     B'_j = sum_{n<=min(j,q)} e_n B_{j-n} + [j<=q] e_j hA_j,
// with B_0 := A_0, e_n = c^n/n! and hB_n = sum_{r>=1} B_r n!/(n+r)!.  Its
// adjoint maps the cotangents (lA', lB') of the top and right edges to those
// of the bottom and left edges, and to dL/dc:
//     lA_r = sum_n e_n lA'_{r+n} + [r>=1] sum_{n<=q} e_n n!/(n+r)! lB'_n
//            (+ sum_n e_n lB'_n   for r = 0, through B_0 := A_0)
//     lB_r = sum_n e_n lB'_{r+n} + sum_{n<=q} e_n n!/(n+r)! lA'_n      (r >= 1)
//     dL/dc = sum_{n=1}^{q} e_{n-1} [ sum_{i>=n} (lA'_i A_{i-n} + lB'_i B_{i-n})
//                                     + lA'_n hB_n + lB'_n hA_n ].
// This is the exact gradient of the truncated forward map (the depth q is a
// piecewise-constant choice and carries no derivative).  In the limit of full
// depth it is the Riemann-function form of the derivative of the Volterra
// equation of Sec. 2.1.
//
// Cotangents flow in reverse topological order: the top-edge cotangent of
// cell (k, l) is the bottom-edge cotangent of cell (k, l+1), the right-edge
// cotangent is the left-edge cotangent of cell (k+1, l).  In the strip's
// step coordinates the adjoint of step t runs after that of step t+1, so lane
// j receives lA' from lane j+1 by a DPP shift, and lB' stays in the lane.
#pragma once
#include "sigk_strip.h"

namespace sigk {

// Algorithmic flops of one cell's adjoint at edge order P, Neumann depth q,
// d channels (FMA = 2 flops), counted on cell_adjoint_fixed:
//   powers c^n and e_n                      3q - 1 mul
//   Hankel sums of both edges               2q(P-2) FMA + 2q mul
//   left edge from the right edge           q(q+1)/2 + (P-1-q)q + q FMA
//   n = 0 rows                              2(P-1) FMA + (P-1) mul
//   terms n = 1..q (Toeplitz transposes
//     and dL/dc)                            sum_n (4(P-n) + 2) FMA + q mul
//   Hankel transposes (nested)              2q(P-1) FMA + 2q + (P-1) mul
//   B_0 := A_0, c = <dx, dy>, dL/dc chained
//     into both increments                  1 add, 3d FMA
__host__ __device__ constexpr long long adjoint_flops(int P, int q, int d) {
    const long long fma_n = 2LL * q * (P - 2) + (long long)q * (q + 1) / 2 +
                            (long long)(P - 1 - q) * q + q + 2LL * (P - 1) +
                            4LL * q * P - 2LL * q * (q + 1) + 2LL * q + 2LL * q * (P - 1) +
                            3LL * d;
    const long long mul_n = q > 0 ? (3LL * q - 1) + 2LL * q + q + 2LL * q + 2LL * (P - 1)
                                  : (long long)(P - 1);
    return 2 * fma_n + mul_n + 1;
}

// Powers e_n = c^n/n!, n = N..q (e[0] = 1).
template <int P, int N, class RC>
__device__ __forceinline__ void powers(double c, int q, double (&e)[P], const RC& R) {
    if constexpr (N < P) {
        if (N > q) return;
        e[N] = e[N - 1] * c * R(N);
        powers<P, N + 1>(c, q, e, R);
    }
}

// Hankel sums of one edge, h_n = sum_{r>=1} V_r n!/(n+r)!, n = N..q (Horner
// form, as in the forward map).
template <int P, int N, class RC>
__device__ __forceinline__ void hankel_sum(const double (&V)[P], int q, double (&h)[P],
                                           const RC& R) {
    if constexpr (N < P) {
        if (N > q) return;
        double t = V[P - 1];
#pragma unroll
        for (int r = P - 2; r >= 1; --r) t = fma(t, R(N + r + 1), V[r]);
        h[N] = t * R(N + 1);
        hankel_sum<P, N + 1>(V, q, h, R);
    }
}

// Left edge of a cell from its right edge.  The map B -> B' is unit lower
// triangular Toeplitz plus terms in A only:
//     B'_j = B_j + sum_{n=1}^{min(j,q)} e_n B_{j-n} + [j<=q] e_j hA_j,  B_0 := A_0,
// so B_j (j >= 1) follows by forward substitution.  On entry B holds B',
// on exit the cell's left edge with B_0 = A_0.
template <int P, int J>
__device__ __forceinline__ void unmap_left(const double (&A)[P], double (&B)[P],
                                           const double (&e)[P], const double (&hA)[P], int q) {
    if constexpr (J < P) {
        double t = B[J];
        if (J <= q) t = fma(-e[J], hA[J], t);
#pragma unroll
        for (int n = 1; n <= J; ++n)
            if (n <= q) t = fma(-e[n], B[J - n], t);
        B[J] = t;
        unmap_left<P, J + 1>(A, B, e, hA, q);
    }
}

// Term N >= 1 of the adjoint: Toeplitz transposes, Hankel transposes and the
// dL/dc contribution.  e = e_{N-1} on entry.
template <int P, int N, class RC>
__device__ __forceinline__ void adjoint_terms(const double (&A)[P], const double (&B)[P],
                                              double c, double e, int q, const double (&hA)[P],
                                              const double (&hB)[P], const double (&lAo)[P],
                                              const double (&lBo)[P], double (&lA)[P],
                                              double (&lB)[P], double& g, const RC& R) {
    if constexpr (N < P) {
        if (N > q) return;
        const double ep = e;             // e_{N-1} = d e_N / dc
        const double en = e * c * R(N);  // e_N
        double corr = fma(lAo[N], hB[N], lBo[N] * hA[N]);
#pragma unroll
        for (int r = 0; r + N < P; ++r) {
            lA[r] = fma(en, lAo[r + N], lA[r]);
            lB[r] = fma(en, lBo[r + N], lB[r]);  // r = 0 entry: cotangent of B_0 := A_0
            corr = fma(lAo[r + N], A[r], corr);
            corr = fma(lBo[r + N], B[r], corr);
        }
        g = fma(ep, corr, g);
        // Hankel transposes: weights e_N N!/(N+r)! as a running product
        double wa = en * lAo[N] * R(N + 1);
        double wb = en * lBo[N] * R(N + 1);
#pragma unroll
        for (int r = 1; r < P; ++r) {
            lB[r] += wa;
            lA[r] += wb;
            wa *= R(N + r + 1);
            wb *= R(N + r + 1);
        }
        adjoint_terms<P, N + 1>(A, B, c, en, q, hA, hB, lAo, lBo, lA, lB, g, R);
    }
}

// Adjoint of cell_map, run backwards in time.  A: the cell's bottom edge
// (stored by the recompute); B: on entry the cell's right edge (the left edge
// of the next cell of the row), on exit the cell's left edge (recovered by
// unmap_left, or the boundary series at the path's start when `boundary`).
// Where `live` is false (steps past the end of the row) B is left unchanged:
// the recompute holds the row's last right edge there, so the walk back starts
// from it exactly.  lAo, lBo: cotangents of the outputs.  Writes the input
// cotangents lA, lB and returns dL/dc.  The recovered left edge differs from
// the forward one by rounding only; it enters dL/dc, never the cotangents
// (those depend on c alone).
template <int P, class RC>
__device__ __forceinline__ double cell_adjoint(const double (&A)[P], double (&B)[P], double c,
                                               int q, bool boundary, bool live,
                                               const double (&lAo)[P],
                                               const double (&lBo)[P], double (&lA)[P],
                                               double (&lB)[P], const RC& R) {
    double e[P], hA[P], hB[P];
    e[0] = 1.0;
    powers<P, 1>(c, q, e, R);
    hankel_sum<P, 1>(A, q, hA, R);
    if (boundary) {
#pragma unroll
        for (int r = 1; r < P; ++r) B[r] = 0.0;
    } else if (live) {
        B[0] = A[0];
        unmap_left<P, 1>(A, B, e, hA, q);
    }
    B[0] = A[0];
    hankel_sum<P, 1>(B, q, hB, R);
    // n = 0 terms: identity parts and the constant-term Hankel rows
#pragma unroll
    for (int r = 0; r < P; ++r) {
        lA[r] = lAo[r];
        lB[r] = lBo[r];
    }
    {
        double wa = lAo[0], wb = lBo[0];
#pragma unroll
        for (int r = 1; r < P; ++r) {
            wa *= R(r);
            wb *= R(r);
            lB[r] += wa;  // d A'_0 / d B_r = 1/r!
            lA[r] += wb;  // d B'_0 / d A_r = 1/r!
        }
    }
    double g = 0.0;
    adjoint_terms<P, 1>(A, B, c, 1.0, q, hA, hB, lAo, lBo, lA, lB, g, R);
    // B_0 := A_0: its cotangent goes to A_0
    lA[0] += lB[0];
    lB[0] = 0.0;
    return g;
}

// The same adjoint for a depth Q fixed at compile time (no per-term branches).
// The Hankel transposes are summed over n first, in nested form: for r >= 1,
//     sum_{n=1}^{Q} e_n lA'_n n!/(n+r)!
//         = (1/(r+1)!) [u_1 + (1/(r+2)) [u_2 + ... + (1/(Q+r)) u_Q]],
// with u_n = c^n lA'_n: one FMA per (n, r) instead of a multiply and an add.
template <int P, int Q, class RC>
__device__ __forceinline__ double cell_adjoint_fixed(const double (&A)[P], double (&B)[P],
                                                     double c, bool boundary, bool live,
                                                     const double (&lAo)[P],
                                                     const double (&lBo)[P], double (&lA)[P],
                                                     double (&lB)[P], const RC& R) {
    double e[Q + 1], cp[Q + 1], hA[Q + 1], hB[Q + 1];
    e[0] = 1.0;
    cp[0] = 1.0;
#pragma unroll
    for (int n = 1; n <= Q; ++n) {
        cp[n] = n == 1 ? c : cp[n - 1] * c;
        e[n] = e[n - 1] * R(n) * c;
    }
#pragma unroll
    for (int n = 1; n <= Q; ++n) {
        double t = A[P - 1];
#pragma unroll
        for (int r = P - 2; r >= 1; --r) t = fma(t, R(n + r + 1), A[r]);
        hA[n] = t * R(n + 1);
    }
    if (boundary) {
#pragma unroll
        for (int r = 1; r < P; ++r) B[r] = 0.0;
    } else if (live) {
        // left edge from right edge: forward substitution (see unmap_left)
        B[0] = A[0];
#pragma unroll
        for (int j = 1; j < P; ++j) {
            double t = B[j];
            if (j <= Q) t = fma(-e[j <= Q ? j : 0], hA[j <= Q ? j : 0], t);
#pragma unroll
            for (int n = 1; n <= Q && n <= j; ++n) t = fma(-e[n], B[j - n], t);
            B[j] = t;
        }
    }
    B[0] = A[0];
#pragma unroll
    for (int n = 1; n <= Q; ++n) {
        double t = B[P - 1];
#pragma unroll
        for (int r = P - 2; r >= 1; --r) t = fma(t, R(n + r + 1), B[r]);
        hB[n] = t * R(n + 1);
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
        lA[r] = lAo[r];
        lB[r] = lBo[r];
    }
    {
        // n = 0 rows: d A'_0 / d B_r = d B'_0 / d A_r = 1/r!
        double f = 1.0;
#pragma unroll
        for (int r = 1; r < P; ++r) {
            f *= R(r);
            lB[r] = fma(lAo[0], f, lB[r]);
            lA[r] = fma(lBo[0], f, lA[r]);
        }
    }
    double g = 0.0;
#pragma unroll
    for (int n = 1; n <= Q; ++n) {
        double corr = fma(lAo[n], hB[n], lBo[n] * hA[n]);
#pragma unroll
        for (int r = 0; r + n < P; ++r) {
            lA[r] = fma(e[n], lAo[r + n], lA[r]);
            lB[r] = fma(e[n], lBo[r + n], lB[r]);  // r = 0 entry: cotangent of B_0 := A_0
            corr = fma(lAo[r + n], A[r], corr);
            corr = fma(lBo[r + n], B[r], corr);
        }
        g = fma(e[n - 1], corr, g);
    }
    if constexpr (Q >= 1) {
        double ua[Q + 1], ub[Q + 1];
#pragma unroll
        for (int n = 1; n <= Q; ++n) {
            ua[n] = cp[n] * lAo[n];
            ub[n] = cp[n] * lBo[n];
        }
        double f = 1.0;  // 1/(r+1)!
#pragma unroll
        for (int r = 1; r < P; ++r) {
            f *= R(r + 1);
            double sa = ua[Q], sb = ub[Q];
#pragma unroll
            for (int n = Q - 1; n >= 1; --n) {
                sa = fma(sa, R(n + r + 1), ua[n]);
                sb = fma(sb, R(n + r + 1), ub[n]);
            }
            lB[r] = fma(sa, f, lB[r]);
            lA[r] = fma(sb, f, lA[r]);
        }
    }
    // B_0 := A_0: its cotangent goes to A_0
    lA[0] += lB[0];
    lB[0] = 0.0;
    return g;
}

}  // namespace sigk
