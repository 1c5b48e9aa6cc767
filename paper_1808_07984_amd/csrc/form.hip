// Top level of the hybrid two-level scheme (Two-Level Strassen's Algorithm
// section, "Hybrid 2-level"): the signed quadrant sum of one product,
//     out := sum_t s_t X_t       (X_t a quadrant of A or B, zero outside it),
// written densely into caller-provided workspace.  Memory bound: each term is
// read once and the sum written once, in 16-byte vectors where aligned.
#include <hip/hip_runtime.h>

#include <cstring>

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

// Operand sums of the one-level "formed" schedule: every signed sum of two
// quadrants that a product needs is written once into workspace by one
// streaming pass per operand, which reads each quadrant once:
//     out_o[r][c] = x_{t0}[r][c] + s1_o * x_{t1}[r][c]      (t1 < 0: x_{t0})
// summed in fp32 from the stored values and, for 16-bit data, rounded once to
// nearest even, exactly as the fused kernels stage the same sum (eq.
// straprim1 with the first term's sign factored out).  A source element
// outside its quadrant's extent is a virtual zero ("Handling the Fringes").
// One row of the output block per workgroup step; each thread handles one
// 16-byte unit per source and output.
struct SumsArgs {
    FormSource src[kFormMaxSources];
    FormOut out[kFormMaxOutputs];
    int32_t nsrc, nout;
    int64_t ld_src, ld_out;
    int64_t rows, cols;  // output block extent, cols a multiple of the unit
};

template <FormElem E>
struct Elem;
template <>
struct Elem<FormElem::kF32> {
    static constexpr int NV = 4;
    using In = float;
    __device__ static float get(float x) { return x; }
    __device__ static float put(float x) { return x; }
};
template <>
struct Elem<FormElem::kBf16> {
    static constexpr int NV = 8;
    using In = unsigned short;
    __device__ static float get(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
    __device__ static unsigned short put(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
};
template <>
struct Elem<FormElem::kF16> {
    static constexpr int NV = 8;
    using In = unsigned short;
    __device__ static float get(unsigned short h) { return (float)__builtin_bit_cast(_Float16, h); }
    __device__ static unsigned short put(float x) { return __builtin_bit_cast(unsigned short, (_Float16)x); }
};

// fp32 sources, outputs pre-split for the compensated mode (written by
// store_split, not put).
template <>
struct Elem<FormElem::kX3Split> {
    static constexpr int NV = 4;
    using In = float;
    __device__ static float get(float x) { return x; }
};

// Four sums, pre-split: hi_e = bf16(s_e) and lo_e = bf16(s_e - hi_e), both
// rounded to nearest even (the compensated kernels' split of a staged value),
// stored as the words (hi_0 | hi_1 << 16, hi_2 | hi_3 << 16, lo_0 | lo_1 << 16,
// lo_2 | lo_3 << 16).
__device__ __forceinline__ void store_split(float *dst, const float (&s)[4]) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const unsigned h01 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{s[0], s[1]}, bf16x2));
    const unsigned h23 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{s[2], s[3]}, bf16x2));
    const float r0 = s[0] - __uint_as_float(h01 << 16), r1 = s[1] - __uint_as_float(h01 & 0xffff0000u);
    const float r2 = s[2] - __uint_as_float(h23 << 16), r3 = s[3] - __uint_as_float(h23 & 0xffff0000u);
    const unsigned l01 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{r0, r1}, bf16x2));
    const unsigned l23 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{r2, r3}, bf16x2));
    *reinterpret_cast<u32x4 *>(dst) = u32x4{h01, h23, l01, l23};
}

template <FormElem E, bool VEC>
__global__ __launch_bounds__(256) void form_sums_kernel(const SumsArgs a) {
    using T = Elem<E>;
    using In = typename T::In;
    constexpr int NV = T::NV;
    typedef In Vec __attribute__((ext_vector_type(NV)));
    const int64_t units = a.cols / NV;
    for (int64_t r = blockIdx.x; r < a.rows; r += gridDim.x) {
        for (int64_t u = threadIdx.x; u < units; u += blockDim.x) {
            const int64_t c = u * NV;
            float x[kFormMaxSources][NV];
#pragma unroll
            for (int q = 0; q < kFormMaxSources; ++q) {
#pragma unroll
                for (int e = 0; e < NV; ++e) x[q][e] = 0.f;
                if (q >= a.nsrc) continue;
                const FormSource sq = a.src[q];
                if (r >= sq.rows) continue;
                const In *p = static_cast<const In *>(sq.ptr) + r * a.ld_src + c;
                if (VEC && c + NV <= sq.cols) {
                    const Vec v = *reinterpret_cast<const Vec *>(p);
#pragma unroll
                    for (int e = 0; e < NV; ++e) x[q][e] = T::get(v[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < NV; ++e)
                        if (c + e < sq.cols) x[q][e] = T::get(p[e]);
                }
            }
#pragma unroll
            for (int o = 0; o < kFormMaxOutputs; ++o) {
                if (o >= a.nout) break;
                const FormOut fo = a.out[o];
                float sv[NV];
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    float s = 0.f;
#pragma unroll
                    for (int q = 0; q < kFormMaxSources; ++q)
                        if (q == fo.t0) s = x[q][e];
                    if (fo.t1 >= 0) {
                        float y = 0.f;
#pragma unroll
                        for (int q = 0; q < kFormMaxSources; ++q)
                            if (q == fo.t1) y = x[q][e];
                        s = __builtin_fmaf(fo.s1, y, s);
                    }
                    sv[e] = s;
                }
                In *dst = static_cast<In *>(fo.ptr) + r * a.ld_out + c;
                if constexpr (E == FormElem::kX3Split) {
                    store_split(dst, sv);
                } else {
                    Vec v;
#pragma unroll
                    for (int e = 0; e < NV; ++e) v[e] = T::put(sv[e]);
                    *reinterpret_cast<Vec *>(dst) = v;
                }
            }
        }
    }
}

struct TermsArgs {
    FormTermsOut out[kFormTermsMaxOutputs];
    int32_t nout;
    int64_t ld_src, ld_out;
    int64_t rows, cols;  // output block extent, cols a multiple of the unit
};

// One 16-byte unit of stored elements at (r, c) of a term block, kept as
// stored (16-bit data stays packed, two elements per register, until it is
// added), zero outside the extent.
template <class T, bool VEC, int NV, class Vec>
__device__ __forceinline__ Vec load_raw(const FormSource &sq, int64_t r, int64_t c, int64_t ld) {
    using In = typename T::In;
    Vec x;
#pragma unroll
    for (int e = 0; e < NV; ++e) x[e] = 0;
    if (r >= sq.rows) return x;
    const In *p = static_cast<const In *>(sq.ptr) + r * ld + c;
    if (VEC && c + NV <= sq.cols) return *reinterpret_cast<const Vec *>(p);
#pragma unroll
    for (int e = 0; e < NV; ++e)
        if (c + e < sq.cols) x[e] = p[e];
    return x;
}

// The terms of one output at (r, c), in order.
template <class T, bool VEC, int NV, class Vec>
__device__ __forceinline__ void load_terms(const FormTermsOut &fo, int64_t r, int64_t c, int64_t ld,
                                           Vec (&x)[kFormTermsMax]) {
#pragma unroll
    for (int t = 0; t < kFormTermsMax; ++t)
        if (t < fo.n) x[t] = load_raw<T, VEC, NV, Vec>(fo.src[t], r, c, ld);
}

// Grid-stride over rows (workgroups) and 16-byte units (threads); per unit
// every output in turn, its terms added in order; a term block shared by
// several outputs of the launch is re-read from cache, not from memory.
// fp32: the next output's terms are loaded before the current output is
// stored (the compiler cannot move loads above a store that may alias
// them), so two outputs' loads are in flight: 0.228 ms for seven 4096^2
// sums from eight blocks, 4.4 TB/s (2.81 ms for all fourteen launches of a
// 16384^3 call, against 3.29 ms with one output in flight).  16-bit data
// keeps one output's loads in flight: with two, its fourteen launches took
// 2.65 ms instead of 1.58.  Outputs and terms are unrolled: the
// kernel-argument arrays are read at constant indices only (no private copy
// of the arguments).
template <FormElem E, bool VEC>
__global__ __launch_bounds__(256) void form_terms_kernel(const TermsArgs a) {
    using T = Elem<E>;
    using In = typename T::In;
    constexpr int NV = T::NV;
    typedef In Vec __attribute__((ext_vector_type(NV)));
    const int64_t units = a.cols / NV;
    for (int64_t r = blockIdx.x; r < a.rows; r += gridDim.x) {
        for (int64_t u = threadIdx.x; u < units; u += blockDim.x) {
            const int64_t c = u * NV;
            constexpr bool kAhead = E == FormElem::kF32 || E == FormElem::kX3Split;
            Vec cur[kFormTermsMax], nxt[kFormTermsMax];
            if constexpr (kAhead) load_terms<T, VEC, NV, Vec>(a.out[0], r, c, a.ld_src, cur);
#pragma unroll
            for (int o = 0; o < kFormTermsMaxOutputs; ++o) {
                if (o >= a.nout) break;
                const FormTermsOut &fo = a.out[o];
                if constexpr (kAhead) {
                    if (o + 1 < kFormTermsMaxOutputs && o + 1 < a.nout)
                        load_terms<T, VEC, NV, Vec>(a.out[o + 1 < kFormTermsMaxOutputs ? o + 1 : o], r, c,
                                                    a.ld_src, nxt);
                } else {
                    load_terms<T, VEC, NV, Vec>(fo, r, c, a.ld_src, cur);
                }
                float acc[NV];
#pragma unroll
                for (int e = 0; e < NV; ++e) acc[e] = T::get(cur[0][e]);
#pragma unroll
                for (int t = 1; t < kFormTermsMax; ++t) {
                    if (t >= fo.n) break;
                    const float st = fo.s[t];
#pragma unroll
                    for (int e = 0; e < NV; ++e) acc[e] = __builtin_fmaf(st, T::get(cur[t][e]), acc[e]);
                }
                In *dst = static_cast<In *>(fo.ptr) + r * a.ld_out + c;
                if constexpr (E == FormElem::kX3Split) {
                    store_split(dst, acc);
                } else {
                    Vec v;
#pragma unroll
                    for (int e = 0; e < NV; ++e) v[e] = T::put(acc[e]);
                    *reinterpret_cast<Vec *>(dst) = v;
                }
                if (kAhead && o + 1 < a.nout) {
#pragma unroll
                    for (int t = 0; t < kFormTermsMax; ++t) cur[t] = nxt[t];
                }
            }
        }
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

namespace strassen {

hipError_t launch_form_sums(FormElem elem, const FormSource *src, int nsrc, int64_t ld_src,
                            const FormOut *out, int nout, int64_t ld_out, int64_t rows, int64_t cols,
                            bool vec, hipStream_t s) {
    const int nv = (elem == FormElem::kF32 || elem == FormElem::kX3Split) ? 4 : 8;
    if (nsrc < 1 || nsrc > kFormMaxSources || nout < 1 || nout > kFormMaxOutputs || cols % nv != 0 ||
        ld_out % nv != 0 || rows < 0)
        return hipErrorInvalidValue;
    for (int o = 0; o < nout; ++o)
        if (out[o].t0 < 0 || out[o].t0 >= nsrc || out[o].t1 >= nsrc) return hipErrorInvalidValue;
    if (rows == 0 || cols == 0) return hipSuccess;
    SumsArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int q = 0; q < nsrc; ++q) a.src[q] = src[q];
    for (int o = 0; o < nout; ++o) a.out[o] = out[o];
    a.nsrc = nsrc;
    a.nout = nout;
    a.ld_src = ld_src;
    a.ld_out = ld_out;
    a.rows = rows;
    a.cols = cols;
    const unsigned blocks = (unsigned)(rows < 65536 ? rows : 65536);
    switch (elem) {
        case FormElem::kF32:
            if (vec) hipLaunchKernelGGL((form_sums_kernel<FormElem::kF32, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_sums_kernel<FormElem::kF32, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kBf16:
            if (vec) hipLaunchKernelGGL((form_sums_kernel<FormElem::kBf16, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_sums_kernel<FormElem::kBf16, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kF16:
            if (vec) hipLaunchKernelGGL((form_sums_kernel<FormElem::kF16, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_sums_kernel<FormElem::kF16, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kX3Split:
            if (vec) hipLaunchKernelGGL((form_sums_kernel<FormElem::kX3Split, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_sums_kernel<FormElem::kX3Split, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
    }
    return hipGetLastError();
}

}  // namespace strassen

namespace strassen {

hipError_t launch_form_terms(FormElem elem, const FormTermsOut *out, int nout, int64_t ld_src,
                             int64_t ld_out, int64_t rows, int64_t cols, bool vec, hipStream_t s) {
    const int nv = (elem == FormElem::kF32 || elem == FormElem::kX3Split) ? 4 : 8;
    if (nout < 1 || nout > kFormTermsMaxOutputs || cols % nv != 0 || ld_out % nv != 0 || rows < 0)
        return hipErrorInvalidValue;
    for (int o = 0; o < nout; ++o)
        if (out[o].n < 1 || out[o].n > kFormTermsMax || out[o].ptr == nullptr) return hipErrorInvalidValue;
    if (rows == 0 || cols == 0) return hipSuccess;
    TermsArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int o = 0; o < nout; ++o) a.out[o] = out[o];
    a.nout = nout;
    a.ld_src = ld_src;
    a.ld_out = ld_out;
    a.rows = rows;
    a.cols = cols;
    const unsigned blocks = (unsigned)(rows < 65536 ? rows : 65536);
    switch (elem) {
        case FormElem::kF32:
            if (vec) hipLaunchKernelGGL((form_terms_kernel<FormElem::kF32, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_terms_kernel<FormElem::kF32, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kBf16:
            if (vec) hipLaunchKernelGGL((form_terms_kernel<FormElem::kBf16, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_terms_kernel<FormElem::kBf16, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kF16:
            if (vec) hipLaunchKernelGGL((form_terms_kernel<FormElem::kF16, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_terms_kernel<FormElem::kF16, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
        case FormElem::kX3Split:
            if (vec) hipLaunchKernelGGL((form_terms_kernel<FormElem::kX3Split, true>), dim3(blocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((form_terms_kernel<FormElem::kX3Split, false>), dim3(blocks), dim3(256), 0, s, a);
            break;
    }
    return hipGetLastError();
}

}  // namespace strassen
