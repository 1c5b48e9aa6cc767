// Entry points of the device code, called by the C ABI (api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "kernel_args.hpp"

namespace strassen {

struct KernelShape {
    int mt, nt, kt;  // workgroup tile
    int vec;         // elements per vector load along k (A) and n (B)
};

// fp32 operands, fp32 MFMA.  Launches one batch of `batch` products of
// variant (wa, wb, wc); vec = 16-byte loads are aligned (see api.cpp);
// trans_x = operand stored transposed; large = 256x256 tile (else 128x128).
KernelShape f32_tile_shape(bool large, int wa = 1, int wb = 1, int wc = 1, bool untransposed = true);
hipError_t launch_f32(bool trans_a, bool trans_b, bool large, int wa, int wb, int wc,
                      const LaunchArgs &a, int batch, bool vec, hipStream_t s);
const char *f32_kernel_name(bool large);
#define STRASSEN_F32_DECL(name)                                                         \
    hipError_t name(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec, \
                    hipStream_t s);
STRASSEN_F32_DECL(launch_f32_nn_s)
STRASSEN_F32_DECL(launch_f32_nn_l)
STRASSEN_F32_DECL(launch_f32_nt_s)
STRASSEN_F32_DECL(launch_f32_nt_l)
STRASSEN_F32_DECL(launch_f32_tn_s)
STRASSEN_F32_DECL(launch_f32_tn_l)
STRASSEN_F32_DECL(launch_f32_tt_s)
STRASSEN_F32_DECL(launch_f32_tt_l)
#undef STRASSEN_F32_DECL
// Concurrent schedule (A and B as stored): a launch mixes products of any
// variant with at most wmax terms per operand/output; outputs are added with
// fp32 atomics (beta applied beforehand).
hipError_t launch_f32_conc_s(int wmax, const LaunchArgs &a, int batch, bool vec, hipStream_t s);
hipError_t launch_f32_conc_l(int wmax, const LaunchArgs &a, int batch, bool vec, hipStream_t s);

// 16-bit MFMA path: bf16 or fp16 operands, or fp32 operands split into
// bf16 hi/lo pairs (compensated product hi*hi + hi*lo + lo*hi).  Transposed
// operands exist for the compensated mode only.  large = 256x256 tile.
enum class Operand16 { kBf16, kF16, kBf16x3 };
KernelShape m16_tile_shape(bool x3, bool large, int wa = 1, int wb = 1, bool untransposed = true);
hipError_t launch_m16(Operand16 op, bool trans_a, bool trans_b, bool large, int wa, int wb, int wc,
                      const LaunchArgs &a, int batch, bool vec, hipStream_t s);
const char *m16_kernel_name(Operand16 op, bool large);
#define STRASSEN_M16_DECL(name)                                                              \
    hipError_t name(bool large, int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec, \
                    hipStream_t s);
STRASSEN_M16_DECL(launch_m16_bf16)
STRASSEN_M16_DECL(launch_m16_f16)
STRASSEN_M16_DECL(launch_m16_bf16x3_nn)
STRASSEN_M16_DECL(launch_m16_bf16x3_nt)
STRASSEN_M16_DECL(launch_m16_bf16x3_tn)
STRASSEN_M16_DECL(launch_m16_bf16x3_tt)
#undef STRASSEN_M16_DECL
// Chained launch of single-term products on 256x256 tiles, A and B as stored:
// nchains chains of two products (a.prod[2z] carries its output
// a.prod[2z].carry - 1 into a.prod[2z + 1], whose one output is the same C
// block), one workgroup grid per chain.
hipError_t launch_m16_chained(Operand16 op, const LaunchArgs &a, int nchains, bool vec, hipStream_t s);
hipError_t launch_m16_bf16_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s);
hipError_t launch_m16_f16_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s);
hipError_t launch_m16_bf16x3_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s);

// The compensated mode on pre-split operands (four elements per 16-byte unit:
// their bf16 hi parts, then their bf16 lo parts; written by launch_form_sums
// with FormElem::kX3Split), A and B as stored, single-term products (W_A =
// W_B = 1, W_C in {1, 2, 4}): A pre-split, B pre-split (pre_b) or fp32.
// Chained launches: both pre-split, 256x256 tiles.
hipError_t launch_m16_x3pre(bool pre_b, bool large, int wa, int wb, int wc, const LaunchArgs &a, int batch,
                            bool vec, hipStream_t s);
hipError_t launch_m16_x3pre_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s);
const char *m16_x3pre_kernel_name(bool pre_b, bool large);

// Hybrid top level: out[r][c] = sum_t sign_t * src_t[r * ld_src + c], zero
// where r >= rows_t or c >= cols_t; out is rows x cols (cols % 4 == 0) with
// leading dimension ld_out (% 4 == 0), 16-byte aligned.  1 or 2 terms.
struct FormTerm {
    const float *src;
    int32_t rows, cols;
    float sign;
};
hipError_t launch_form(float *out, int64_t ld_out, int64_t rows, int64_t cols, int64_t ld_src,
                       const FormTerm *terms, int nterms, bool vec, hipStream_t s);

// One-level "formed" schedule: out_o = x_{t0} + s1_o * x_{t1} (t1 < 0: the
// single term x_{t0}) over a rows x cols block, for up to five outputs from up
// to four source quadrants sharing ld_src; sums in fp32 from the stored
// element type, 16-bit outputs rounded once to nearest even; a source element
// outside its rows x cols extent is zero.  Outputs are dense (ld_out), cols
// and ld_out multiples of the 16-byte unit (4 fp32 or 8 16-bit elements),
// 16-byte aligned; vec = sources aligned for 16-byte loads.
// FormElem::kX3Split: fp32 sources, each output written pre-split for the
// compensated mode (per four elements x: bf16 hi = x rounded to nearest even,
// then bf16 lo = (x - hi) rounded to nearest even; see launch_m16_x3pre).
enum class FormElem { kF32, kBf16, kF16, kX3Split };
constexpr int kFormMaxSources = 4, kFormMaxOutputs = 7;
struct FormSource {
    const void *ptr;
    int32_t rows, cols;
};
struct FormOut {
    void *ptr;
    int32_t t0, t1;
    float s1;
};
hipError_t launch_form_sums(FormElem elem, const FormSource *src, int nsrc, int64_t ld_src,
                            const FormOut *out, int nout, int64_t ld_out, int64_t rows, int64_t cols,
                            bool vec, hipStream_t s);

// Two-level "formed" schedule: out_o = x_0 + sum_{t >= 1} s_t * x_t over up to
// four terms, each term a block of its own (pointer and rows x cols extent,
// zero outside it, all sharing ld_src), for up to eight outputs; the terms
// are added in order with one fused multiply-add each, in fp32 from the
// stored element type, 16-bit outputs rounded once to nearest even -- the
// arithmetic of the fused kernels' operand staging.  Layout rules as for
// launch_form_sums.
constexpr int kFormTermsMax = 4, kFormTermsMaxOutputs = 8;
struct FormTermsOut {
    void *ptr;
    int32_t n;                           // terms, 1..kFormTermsMax
    int32_t pad;
    FormSource src[kFormTermsMax];
    float s[kFormTermsMax];              // s[0] unused (the first term is added as is)
};
hipError_t launch_form_terms(FormElem elem, const FormTermsOut *out, int nout, int64_t ld_src,
                             int64_t ld_out, int64_t rows, int64_t cols, bool vec, hipStream_t s);

// strassen_probe_mfma: `workgroups` workgroups of four waves, each wave
// `iters` rounds of four independent MFMAs on register operands (op 0 bf16
// 32x32x16, 1 fp16 32x32x16, 2 fp32 32x32x2; random or constant values);
// out receives one float per thread (workgroups * 256).
hipError_t launch_mfma_probe(int op, int random, int64_t iters, int32_t workgroups, float *out, hipStream_t s);

// strassen_gemm_formed_noalloc: the device address of the library's fixed
// scratch array (kNoAllocScratchBytes, 256-byte aligned) on the device of
// `stream` (the current device for the null stream), looked up once per
// device.
constexpr int64_t kNoAllocScratchBytes = (int64_t)256 << 20;
hipError_t noalloc_scratch(hipStream_t stream, void **ptr);

// C := beta * C over an m x n matrix (beta == 0 writes zeros, C not read).
hipError_t launch_scale(float *C, int64_t ldc, int64_t m, int64_t n, float beta, hipStream_t s);

}  // namespace strassen
