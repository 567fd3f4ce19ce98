// sigk_delta.hip -- the cell-coefficient field for many channels.
//
// For d > 32 the coefficients c_kl = <dx_k, dy_l> are no longer cheap next to
// the cell map (2d flops against about 6P^2), and they form a dense matrix
// product of the two increment sequences, dY dX^T.  This kernel computes it on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64) for every pair of a Gram call
// and stores it in the order the strip sweep reads it: per 64-row strip s,
// step t and lane j, the coefficient of cell (t - j, 64 s + j), so that each
// step of the sweep reads 64 consecutive doubles.  Entries of cells outside
// the grid are never written (the sweep masks them).
//
// Block: 64 rows (one strip) x 64 columns of one pair, four waves of
// 32 x 32, each a 2 x 2 set of 16 x 16 MFMA tiles; channels are staged in LDS
// 16 at a time, the increments formed on the way in.  The result tile goes
// through LDS so that each step's run of lanes is written contiguously.
#include "sigk_device.h"

namespace sigk {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kKT = 16;  // channels per LDS stage

// Lane layout of v_mfma_f64_16x16x4f64 (checked on the device): A[i][k] in
// lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4),
// element i / 4.
__global__ void __launch_bounds__(256) delta_gemm_kernel(FwdArgs a) {
    __shared__ double sy[64][kKT + 1];
    __shared__ double sx[64][kKT + 1];
    __shared__ double so[64][65];
    const int pair = (int)blockIdx.z;
    const Geo g = resolve(a, pair, 1, 0);
    const int m = g.m, n = g.n, d = a.d;
    const int s = (int)blockIdx.y;
    const int k0 = (int)blockIdx.x * 64, l0 = s * 64;
    if (k0 >= m || l0 >= n) return;  // uniform over the block
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < d; kc += kKT) {
        for (int e = tid; e < 64 * kKT; e += 256) {
            const int r = e / kKT, cc = e % kKT, ch = kc + cc;
            const int l = l0 + r, k = k0 + r;
            sy[r][cc] = (l < n && ch < d)
                            ? g.y[(int64_t)(l + 1) * d + ch] - g.y[(int64_t)l * d + ch]
                            : 0.0;
            sx[r][cc] = (k < m && ch < d)
                            ? g.x[(int64_t)(k + 1) * d + ch] - g.x[(int64_t)k * d + ch]
                            : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKT; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = sy[rb + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = sx[cb + 16 * j + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                so[rb + 16 * i + (lane >> 4) + 4 * r][cb + 16 * j + (lane & 15)] = acc[i][j][r];
    __syncthreads();
    // step t = k0 + u: lane j of the strip holds column t - j
    double* dst = a.delta + g.delta + (int64_t)s * delta_steps(m) * kWave;
    for (int u = w; u < 127; u += 4) {
        const int kt = u - lane;  // column within the tile
        if (kt >= 0 && kt < 64 && l0 + lane < n && k0 + kt < m)
            dst[(int64_t)(k0 + u) * kWave + lane] = so[lane][kt];
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0)
        atomicAdd(&a.hdr->flops, 2ull * (unsigned long long)d * (unsigned long long)m *
                                     (unsigned long long)n);
}

}  // namespace

hipError_t launch_delta_gemm(const FwdArgs& a, hipStream_t s) {
    const int64_t m = a.lx - 1, n = a.ly - 1;
    const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64), (unsigned)a.npairs);
    hipLaunchKernelGGL(delta_gemm_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sigk
