// sigk_estimate.hip -- a-priori truncation order of a pair (App. C, "Error
// Analysis and Limitations"): the order is chosen from statistics of the two
// paths before any sweep, by bounding the tile matrix at the largest cell
// coefficient of the grid.
//
// Reading of the estimate.  In unit-cell coordinates the tile matrix of
// Proposition 2.8 has entries C_ij = c^min(i,j) w_ij (alpha_{i-j} or
// beta_{j-i}), w_ij = (max-min)!/(max! min!), alpha and beta the monomial
// coefficients of the bottom and left edges.  Along an edge, K's r-th
// derivative in unit-cell units is at most about h^r |K| with
// h = max(max_k |dx_k| max_l |y_l - y_0|, max_l |dy_l| max_k |x_k - x_0|)
// (the global derivative scale of the paths times the cell width, which is
// the role of the factors Delta sigma^N, Delta tau^N in App. C), so the edge
// coefficients are bounded by alpha_r, beta_r <= h^r / r!.  The entries of
// the last row and column of the (N+1) x (N+1) tile matrix at c = max|c_kl|
// then sum to
//     E(N) = 2/N! sum_{j=0}^{N} cmax^j h^(N-j) / j!,
// the estimated local error of order N relative to K.  Local errors add up
// over the cells of the pair, so the estimate is cells * E(N), and the order
// is the least N (searched upwards) with cells * E(N) <= tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/sigk.h"
#include "sigk_internal.h"

namespace {

__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    // nonnegative doubles order like their bit patterns
    atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

__device__ double block_max(double v) {
    __shared__ double sm[256];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = sm[0];
    __syncthreads();
    return r;
}

// out[0] = max_k |z_{k+1} - z_k|^2, out[1] = max_k |z_k - z_0|^2.
__global__ void path_stats_kernel(const double* z, int64_t len, int64_t d, double* out) {
    double m0 = 0.0, m1 = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len;
         k += (int64_t)gridDim.x * blockDim.x) {
        double s0 = 0.0, s1 = 0.0;
        for (int64_t c = 0; c < d; ++c) {
            const double v = z[k * d + c];
            const double dz = k + 1 < len ? z[(k + 1) * d + c] - v : 0.0;
            const double e = v - z[c];
            s0 = fma(dz, dz, s0);
            s1 = fma(e, e, s1);
        }
        m0 = fmax(m0, s0);
        m1 = fmax(m1, s1);
    }
    m0 = block_max(m0);
    m1 = block_max(m1);
    if (threadIdx.x == 0) {
        atomic_max_nonneg(&out[0], m0);
        atomic_max_nonneg(&out[1], m1);
    }
}

constexpr int kColsPerBlock = 1024;

// out[0] = max_{k,l} |<dx_k, dy_l>| over the grid.  Block (bx, by): rows
// [64 by, 64 by + 64) and columns [kColsPerBlock bx, ...); lane j of each of
// the 4 waves holds row j, wave w takes every 4th column (the column's
// increment is the same for the whole wave: a broadcast read).
__global__ void cell_max_kernel(const double* x, int64_t m, const double* y, int64_t n,
                                int64_t d, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t l = (int64_t)blockIdx.y * 64 + lane;
    const int64_t k0 = (int64_t)blockIdx.x * kColsPerBlock;
    const int64_t k1 = std::min<int64_t>(k0 + kColsPerBlock, m);
    double mx = 0.0;
    if (l < n && d <= 32) {
        // the row's increment in registers (zero beyond d)
        double dy[32];
#pragma unroll
        for (int ch = 0; ch < 32; ++ch)
            dy[ch] = ch < d ? y[(l + 1) * d + ch] - y[l * d + ch] : 0.0;
        for (int64_t k = k0 + wave; k < k1; k += 4) {
            double c = 0.0;
#pragma unroll
            for (int ch = 0; ch < 32; ++ch)
                if (ch < d) c = fma(dy[ch], x[(k + 1) * d + ch] - x[k * d + ch], c);
            mx = fmax(mx, fabs(c));
        }
    } else if (l < n) {
        for (int64_t k = k0 + wave; k < k1; k += 4) {
            double c = 0.0;
            for (int64_t ch = 0; ch < d; ++ch)
                c = fma(y[(l + 1) * d + ch] - y[l * d + ch], x[(k + 1) * d + ch] - x[k * d + ch], c);
            mx = fmax(mx, fabs(c));
        }
    }
    mx = block_max(mx);
    if (threadIdx.x == 0) atomic_max_nonneg(&out[0], mx);
}

__global__ void zero_kernel(double* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

}  // namespace

extern "C" {

int sigk_order_bound(double cmax, double h, double cells, double tol, int* N_out,
                     double* bound_out) {
    if (!N_out || !(cmax >= 0.0) || !(h >= 0.0) || !(cells >= 0.0) || !(tol > 0.0) ||
        !std::isfinite(cmax) || !std::isfinite(h) || !std::isfinite(cells))
        return SIGK_EINVAL;
    constexpr int kNmin = 1, kNmax = 64;
    double bound = 0.0;
    for (int N = kNmin; N <= kNmax; ++N) {
        // E(N) = 2/N! sum_j cmax^j h^(N-j)/j!, summed in log space
        const double lfN = std::lgamma((double)N + 1.0);
        double e = 0.0;
        for (int j = 0; j <= N; ++j) {
            if ((cmax == 0.0 && j > 0) || (h == 0.0 && j < N)) continue;
            const double lt = (j > 0 ? j * std::log(cmax) : 0.0) +
                              (j < N ? (N - j) * std::log(h) : 0.0) - lfN -
                              std::lgamma((double)j + 1.0);
            e += std::exp(lt);
        }
        bound = cells * 2.0 * e;
        if (bound <= tol) {
            *N_out = N;
            if (bound_out) *bound_out = bound;
            return SIGK_OK;
        }
    }
    *N_out = kNmax;
    if (bound_out) *bound_out = bound;
    return SIGK_EUNSUPPORTED;
}

int sigk_estimate_order(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                        double tol, int* order_out, double* bound_out, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!order_out || lx < 0 || ly < 0 || d < 1 || !(tol > 0.0)) return SIGK_EINVAL;
    if (lx < 2 || ly < 2) {  // no cells: nothing is truncated
        *order_out = sigk_supported_order(1);
        if (bound_out) *bound_out = 0.0;
        return SIGK_OK;
    }
    if (!x || !y || !ws) return SIGK_EINVAL;
    if (ws_bytes < 5 * sizeof(double)) return SIGK_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double* st = (double*)ws;  // [0] max|c|, [1..2] stats of x, [3..4] stats of y
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, st, 5);
    hipError_t e = hipGetLastError();
    const int pb_x = (int)std::min<int64_t>((lx + 255) / 256, 1024);
    const int pb_y = (int)std::min<int64_t>((ly + 255) / 256, 1024);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(path_stats_kernel, dim3(pb_x), dim3(256), 0, s, x, lx, d, st + 1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(path_stats_kernel, dim3(pb_y), dim3(256), 0, s, y, ly, d, st + 3);
        e = hipGetLastError();
    }
    const int64_t m = lx - 1, n = ly - 1;
    const int64_t gx = (m + kColsPerBlock - 1) / kColsPerBlock, gy = (n + 63) / 64;
    if (gy > 65535 || gx > INT32_MAX) return SIGK_EUNSUPPORTED;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(cell_max_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, x,
                           m, y, n, d, st);
        e = hipGetLastError();
    }
    double h_st[5] = {0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h_st, st, sizeof h_st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return sigk::device_error(e);
    const double cmax = h_st[0];
    const double h = std::max(std::sqrt(h_st[1]) * std::sqrt(h_st[4]),
                              std::sqrt(h_st[3]) * std::sqrt(h_st[2]));
    int N = 0;
    const int rc = sigk_order_bound(cmax, h, (double)m * (double)n, tol, &N, bound_out);
    const int P = sigk_supported_order(N + 1);
    *order_out = P;
    if (rc) return rc;
    return P ? SIGK_OK : SIGK_EUNSUPPORTED;
}

}  // extern "C"
