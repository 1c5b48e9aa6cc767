// Fixed device scratch for strassen_gemm_formed_noalloc: the formed one-level
// schedule's operand-sum workspace without any allocation at call time, for
// callers that cannot allocate (graph capture, tight serving loops).  The
// array lives in this file's code object, so every GPU the library runs on
// holds one copy of kNoAllocScratchBytes from module load until the process
// ends.  Its host-side name is only a stand-in: kernels are given the device
// address hipGetSymbolAddress returns, looked up once per device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "launch.hpp"

namespace strassen {
namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

}  // namespace

hipError_t noalloc_scratch(hipStream_t stream, void **ptr) {
    int dev = 0;
    hipError_t err = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev] == nullptr) {
        int cur = 0;
        if ((err = hipGetDevice(&cur)) != hipSuccess) return err;
        if (cur != dev && (err = hipSetDevice(dev)) != hipSuccess) return err;
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t back = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (err != hipSuccess) return err;
        if (back != hipSuccess) return back;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace strassen
