// sigk_static.hip -- sigk_gram_static: the Gram matrix (and, as its 1 x 1
// case, one pair) for callers that cannot allocate device memory.
//
// The workspace of sigk_gram (header, progress flags, frontier rows) lives
// here in a file-scope device array of kStaticBytes.  Host code never passes
// the array's name to a kernel: in host code that name is a host-side stand-in,
// not a device address.  The device address is looked up once per device with
// hipGetSymbolAddress (each GPU holds its own copy of the array) and kept;
// every launch receives that pointer, exactly like a caller-owned workspace.
//
// All calls on one device share the array, so calls that overlap on a device
// (different streams, or host threads without ordering) race on it.  The
// reset kernel that starts every sigk_gram launch clears what must start at
// zero (status, tickets, counters, progress flags); the frontier rows are
// written before they are read.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sigk.h"
#include "sigk_internal.h"

namespace {

constexpr size_t kStaticBytes = (size_t)SIGK_STATIC_WS_BYTES;

__device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (looked up on first use
// with the device current).
int static_workspace(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sigk::device_error(e);
    if (dev < 0 || dev >= kMaxDevices) return SIGK_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return sigk::device_error(e);
        if (!p) return SIGK_EDEVICE;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SIGK_OK;
}

__global__ void copy_status_kernel(const sigk::WsHeader* h, uint32_t* status) {
    *status = h->status;
}

}  // namespace

extern "C" int sigk_gram_static(const double* X, int64_t nx, const double* Y, int64_t ny,
                                int64_t lx, int64_t ly, int64_t d, int symmetric,
                                const sigk_opts* o, double* G, uint32_t* status, void* stream) {
    size_t need = 0;
    int rc = sigk_gram_workspace_size(nx, ny, lx, ly, d, symmetric, o, &need);
    if (rc) return rc;
    if (need > kStaticBytes) return SIGK_EWORKSPACE;
    if (nx * ny == 0) return SIGK_OK;
    void* ws = nullptr;
    rc = static_workspace(&ws);
    if (rc) return rc;
    rc = sigk_gram(X, nx, Y, ny, lx, ly, d, symmetric, o, G, ws, kStaticBytes, stream);
    if (rc || !status) return rc;
    hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream,
                       (const sigk::WsHeader*)ws, status);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIGK_OK : sigk::device_error(e);
}
