// Library-owned device scratch for the entry point that allocates nothing
// (pw_small_eigh_noalloc): one fixed array per GPU, resolved to its device
// address once per device when the first context on that device is created.
//
// In host code the array's name is only a host-side stand-in; kernels get the
// device address returned by hipGetSymbolAddress, kept per device below.
#include <mutex>

#include "pw_internal.h"

// Size: the Rayleigh-Ritz eigenproblems of the iteration (n = 3m <= 192) need
// ~0.3 MB; 4 MiB holds every (n, k) with heev_scratch_bytes(n, k) + 256 <= 4 MiB
// (k = n up to n ~ 700, k = 64 up to n = 1024).
static constexpr size_t kStaticScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace pw {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};   // device address of `scratch` on each device

__global__ void k_clear_ints(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
    return hipSuccess;
}

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

// Fill kernel rather than hipMemsetAsync, so a caller may record the call into a graph.
void launch_clear_ints(int *p, int count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_clear_ints, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    PW_HIP(hipGetLastError());
}

}  // namespace pw
