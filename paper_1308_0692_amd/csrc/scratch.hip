// The library's own device workspace, for callers that cannot allocate device memory
// (fdlb_step_static).  One fixed-size array per GPU, held from the moment the library's code
// object is loaded on that GPU until the process ends.
//
// On the host the array's name is only a stand-in: its device address differs per GPU and is
// looked up once per device with hipGetSymbolAddress (with that device current), then cached.
// Host code passes only that address to kernels and copies.
#include <mutex>

#include "fdlb_internal.h"

namespace fdlb {

namespace {

static __device__ __align__(256) char scratch[FDLB_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

// Reset of a control block: step 0, nothing recorded, no tolerance, no freeze request.
__global__ void __launch_bounds__(64) ctrl_reset_kernel(double* __restrict__ ctrl) {
    const int i = threadIdx.x;
    if (i >= 8) return;
    double v = 0.0;
    if (i == CTRL_FIRST_BELOW || i == CTRL_DIVERGED) v = -1.0;
    ctrl[i] = v;
}

}  // namespace

char* static_scratch() {
    static std::mutex mu;
    static char* addr[MAX_DEVICES] = {};
    int dev = -1;
    FDLB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) throw Error(FDLB_EINVAL, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        FDLB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) throw Error(FDLB_EHIP, "static scratch has no usable device address");
        addr[dev] = (char*)p;
    }
    return addr[dev];
}

void launch_ctrl_reset(double* ctrl, hipStream_t stream) {
    hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(64), 0, stream, ctrl);
    FDLB_HIP(hipGetLastError());
}

}  // namespace fdlb
