// Top level of the hybrid two-level scheme (Two-Level Strassen's Algorithm
// section, "Hybrid 2-level"): the signed quadrant sum of one product,
//     out := sum_t s_t X_t       (X_t a quadrant of A or B, zero outside it),
// written densely into caller-provided workspace.  Memory bound: each term is
// read once and the sum written once, in 16-byte vectors where aligned.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace strassen {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct FormArgs {
    float *out;
    int64_t ld_out;
    int32_t rows, cols;  // extent of out (multiple of 4 in cols)
    int32_t nterms;
    int64_t ld_src;
    FormTerm t[2];
};

// One thread per 4 consecutive columns of one row.
template <bool VEC>
__global__ __launch_bounds__(256) void form_kernel(const FormArgs a) {
    const int64_t quads = a.cols / 4;
    const int64_t total = (int64_t)a.rows * quads;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(idx / quads);
        const int c = (int)(idx % quads) * 4;
        f32x4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t >= a.nterms) break;
            const FormTerm x = a.t[t];
            if (r >= x.rows) continue;
            const float *p = x.src + (int64_t)r * a.ld_src + c;
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (VEC && c + 3 < x.cols) {
                v = *reinterpret_cast<const f32x4 *>(p);
            } else {
                if (c + 0 < x.cols) v.x = p[0];
                if (c + 1 < x.cols) v.y = p[1];
                if (c + 2 < x.cols) v.z = p[2];
                if (c + 3 < x.cols) v.w = p[3];
            }
            s += x.sign * v;
        }
        *reinterpret_cast<f32x4 *>(a.out + (int64_t)r * a.ld_out + c) = s;
    }
}

}  // namespace

hipError_t launch_form(float *out, int64_t ld_out, int64_t rows, int64_t cols, int64_t ld_src,
                       const FormTerm *terms, int nterms, bool vec, hipStream_t s) {
    if (nterms < 1 || nterms > 2 || cols % 4 != 0 || ld_out % 4 != 0) return hipErrorInvalidValue;
    FormArgs a;
    a.out = out;
    a.ld_out = ld_out;
    a.rows = (int32_t)rows;
    a.cols = (int32_t)cols;
    a.nterms = nterms;
    a.ld_src = ld_src;
    for (int t = 0; t < nterms; ++t) a.t[t] = terms[t];
    const int64_t total = rows * (cols / 4);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    if (vec)
        hipLaunchKernelGGL(form_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(form_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace strassen
