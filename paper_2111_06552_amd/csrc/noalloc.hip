// Block inner product for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  It runs the kernels of gcge_gram; the per-chunk partial tiles
// that gcge_gram keeps in the library's grow-only workspace live here in a
// file-scope device array of fixed size instead, and the result is written to
// the caller's device buffer (no host staging, no synchronization).
#include <mutex>

#include "gcge.h"
#include "internal.h"

namespace gcge {

// Partial tiles of the Gram kernels.  Each device the library runs on holds
// its own copy until the process ends.  In host code `scratch` is only a
// handle for hipGetSymbolAddress; kernels receive the device address.
static __device__ __align__(256) double scratch[GCGE_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_scratch[MAX_DEVICES];   // device address of `scratch` per device, looked up once

// Address of this device's `scratch` (the current device), looked up on the
// first call on that device with the device current.
hipError_t scratch_address(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// C = 0 (m x k, row-major with row length k): the product over zero rows.  A
// kernel rather than a memset, so that the call can be captured in a graph.
__global__ __launch_bounds__(256) void k_zero(int64_t count, double *C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) C[i] = 0.0;
}

int fail(int code, const std::string &msg) {
    set_thread_error(msg);
    return code;
}

}  // namespace
}  // namespace gcge

using namespace gcge;

extern "C" int gcge_gram_noalloc(int64_t n, const double *X, int64_t ldx, int m, const double *Y, int64_t ldy, int k,
                                 const double *d, double *C, void *stream) {
    if (n < 0 || m < 0 || k < 0 || (m > 0 && (ldx < m || (n > 0 && !X))) || (k > 0 && (ldy < k || (n > 0 && !Y))) ||
        ((int64_t)m * k > 0 && !C))
        return fail(GCGE_ERR_INVALID_ARG, "gcge_gram_noalloc: invalid argument");
    if (m == 0 || k == 0) return GCGE_OK;
    if (m > 48 * 64) return fail(GCGE_ERR_INVALID_ARG, "gcge_gram_noalloc: m above 3072 is not supported");
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        const int64_t count = (int64_t)m * k;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, C);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? GCGE_OK : fail(GCGE_ERR_HIP, std::string("gcge_gram_noalloc: ") + hipGetErrorString(e));
    }
    Segs XS;
    XS.add(X, ldx, m);
    // the largest product: one chunk of partial tiles must fit the scratch array
    size_t need = 0;
    hipError_t e = gram_into(n, XS, Y, ldy, k, d, C, k, nullptr, GCGE_NOALLOC_SCRATCH_BYTES, &need, st);
    if (e == hipErrorInvalidValue)
        return fail(GCGE_ERR_INVALID_ARG, "gcge_gram_noalloc: m x k needs more partial tiles than the " +
                                              std::to_string(GCGE_NOALLOC_SCRATCH_BYTES >> 20) +
                                              " MiB scratch array holds");
    if (e != hipSuccess) return fail(GCGE_ERR_HIP, std::string("gcge_gram_noalloc: ") + hipGetErrorString(e));
    double *part = nullptr;
    e = scratch_address(&part);
    if (e != hipSuccess)
        return fail(GCGE_ERR_HIP, std::string("gcge_gram_noalloc: scratch address: ") + hipGetErrorString(e));
    e = gram_into(n, XS, Y, ldy, k, d, C, k, part, GCGE_NOALLOC_SCRATCH_BYTES, nullptr, st);
    if (e != hipSuccess) return fail(GCGE_ERR_HIP, std::string("gcge_gram_noalloc: ") + hipGetErrorString(e));
    return GCGE_OK;
}
