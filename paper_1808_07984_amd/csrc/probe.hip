// Measurement support: the matrix cores' attainable rate on this part, the
// ceiling the 16-bit kernels are compared with.  Every wave issues a long run
// of independent MFMAs on operands held in registers -- no memory traffic,
// no LDS, no barriers -- so the rate measured is the matrix cores' under the
// power and clock conditions the operand values bring about: constant
// operands (little switching) or random ones (the hardware's clock falls under
// sustained 16-bit MFMA work on random data).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "launch.hpp"

namespace strassen {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// A value in [-0.5, 0.5) from a 32-bit hash of (lane, set, element); a
// constant 0.25 when `random` is 0.
__device__ __forceinline__ float operand_value(uint32_t seed, int set, int e, int random) {
    if (!random) return 0.25f;
    uint32_t h = seed * 0x9E3779B1u ^ (uint32_t)(set * 131 + e) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (float)(h & 0xFFFFu) * (1.0f / 65536.0f) - 0.5f;
}

constexpr int kSets = 4;  // independent accumulators per wave (covers the MFMA latency)

// op 0: 32x32x16 bf16, op 1: 32x32x16 fp16, op 2: 32x32x2 fp32.  Each wave
// runs `iters` rounds of kSets MFMAs, cycling through kSets operand pairs,
// and every lane writes the sum of its accumulators to out (so no MFMA is
// dead code).
template <int OP>
__global__ __launch_bounds__(256) void mfma_probe_kernel(int64_t iters, int random, float *out) {
    const uint32_t seed = blockIdx.x * 256u + threadIdx.x + 1u;
    f32x16 acc[kSets];
#pragma unroll
    for (int s = 0; s < kSets; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[s][e] = 0.f;
    if constexpr (OP == 0 || OP == 1) {
        using V = typename std::conditional<OP == 0, bf16x8, f16x8>::type;
        using E = typename std::conditional<OP == 0, __bf16, _Float16>::type;
        V a[kSets], b[kSets];
#pragma unroll
        for (int s = 0; s < kSets; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[s][e] = (E)operand_value(seed, s, e, random);
                b[s][e] = (E)operand_value(seed ^ 0x5555u, s, e, random);
            }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int s = 0; s < kSets; ++s) {
                if constexpr (OP == 0)
                    acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], b[(s + 1) % kSets], acc[s], 0, 0, 0);
                else
                    acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[s], b[(s + 1) % kSets], acc[s], 0, 0, 0);
            }
        }
    } else {
        float a[kSets], b[kSets];
#pragma unroll
        for (int s = 0; s < kSets; ++s) {
            a[s] = operand_value(seed, s, 0, random);
            b[s] = operand_value(seed ^ 0x5555u, s, 1, random);
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int s = 0; s < kSets; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[(s + 1) % kSets], acc[s], 0, 0, 0);
        }
    }
    float sum = 0.f;
#pragma unroll
    for (int s = 0; s < kSets; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e) sum += acc[s][e];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = sum;
}

}  // namespace

hipError_t launch_mfma_probe(int op, int random, int64_t iters, int32_t workgroups, float *out, hipStream_t s) {
    if (op < 0 || op > 2 || iters < 0 || workgroups < 1 || out == nullptr) return hipErrorInvalidValue;
    switch (op) {
        case 0: hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(workgroups), dim3(256), 0, s, iters, random, out); break;
        case 1: hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(workgroups), dim3(256), 0, s, iters, random, out); break;
        default: hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3(workgroups), dim3(256), 0, s, iters, random, out); break;
    }
    return hipGetLastError();
}

}  // namespace strassen
