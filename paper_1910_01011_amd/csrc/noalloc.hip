// Scratch of the allocation-free apply (bem_apply_noalloc): one file-scope
// device array, held by every GPU the library runs on until the process ends.
//
// In host code the array's name stands for a host-side shadow, not for device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (that device current) and only that address is handed to
// kernels and launchers.
#include <mutex>

#include "bem_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[bem::NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};   // device address of `scratch` per device ordinal

__global__ void k_zero_f64(double *p, int64_t n)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

namespace bem {

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) throw Error{BEM_ERR_INVALID_ARG, "device ordinal out of range"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        BEM_HIP(hipGetDevice(&cur));
        if (cur != device) throw Error{BEM_ERR_DEVICE, "scratch lookup: the problem's device is not current"};
        void *ptr = nullptr;
        BEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error{BEM_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array"};
        g_scratch[device] = ptr;
    }
    return g_scratch[device];
}

void launch_zero_f64(hipStream_t s, double *p, int64_t n)
{
    if (n <= 0) return;
    const int B = 256;
    k_zero_f64<<<dim3(blocks_1d(n, B, true)), dim3(B), 0, s>>>(p, n);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
