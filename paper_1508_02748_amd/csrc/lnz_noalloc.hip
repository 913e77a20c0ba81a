// lnz_noalloc.hip -- the tensor-product reweighting forward for callers that
// cannot allocate device memory: the column sums A(beta_i, M) live in a fixed
// array of device memory that the library holds, instead of a caller-given
// workspace.  Same kernels and results as rewl_lnz_grid_forward.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rewl.h"
#include "rewl_internal.h"

namespace {

// The array, one copy per GPU, held until the process ends.  In host code its
// name stands for nothing usable: only the address hipGetSymbolAddress returns
// (per device) may be handed to kernels or copies.
constexpr size_t NOALLOC_BYTES = static_cast<size_t>(REWL_NOALLOC_SCRATCH_BYTES);
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" rewl_status rewl_lnz_grid_forward_noalloc(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0,
                                                     int32_t nM, const double* beta, int64_t nB, const double* h,
                                                     int64_t nH, double* lnz, void* hip_stream) {
    rewl_status s = rewl::lnz_grid_check(lng, N, e0, nE, m0, nM, beta, nB, h, nH);
    if (s != REWL_OK) return s;
    if (!lnz) return rewl::set_error(REWL_EINVAL, "null pointer");
    if (static_cast<unsigned long long>(nB) * static_cast<unsigned long long>(nM) * sizeof(double) > NOALLOC_BYTES)
        return rewl::set_error(REWL_EINVAL, "nB * nM * 8 bytes exceed REWL_NOALLOC_SCRATCH_BYTES");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return rewl::set_error(REWL_EDEVICE, "no usable current device");
    void* ws = nullptr;
    hipError_t e = scratch_address(dev, &ws);
    if (e != hipSuccess) return rewl::set_error(REWL_EDEVICE, "scratch address lookup failed");
    // every entry of A(i, M) that the row pass reads is written by the column pass
    // first, so the array needs no clearing between calls
    e = rewl::launch_lnz_grid_forward(lng, N, e0, nE, m0, nM, beta, nB, h, nH, static_cast<double*>(ws), lnz,
                                      static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return rewl::set_error(REWL_EDEVICE, "lnz grid forward (no-allocation) launch failed");
    return REWL_OK;
}
