// C := beta * C, used when the product term vanishes (k == 0 or alpha == 0).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace strassen {
namespace {

// One workgroup row-strip: threads stride along n; grid.x walks rows.
__global__ __launch_bounds__(256) void scale_kernel(float *C, int64_t ldc, int64_t m, int64_t n,
                                                    float beta) {
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        float *row = C + i * ldc;
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
            row[j] = (beta == 0.f) ? 0.f : beta * row[j];
    }
}

}  // namespace

hipError_t launch_scale(float *C, int64_t ldc, int64_t m, int64_t n, float beta, hipStream_t s) {
    if (m <= 0 || n <= 0 || beta == 1.f) return hipSuccess;
    const int64_t rows = m < 65536 ? m : 65536;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)rows), dim3(256), 0, s, C, ldc, m, n, beta);
    return hipGetLastError();
}

}  // namespace strassen
