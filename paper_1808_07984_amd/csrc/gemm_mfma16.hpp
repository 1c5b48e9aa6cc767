// Strassen primitive on the gfx950 16-bit matrix cores (template; each
// operand type is instantiated in its own translation unit)
// (v_mfma_f32_32x32x16_{bf16,f16}, fp32 accumulation).
//
// Three operand modes share one template:
//   * bf16 operands  -> signed sums in fp32, rounded once to bf16 (nearest
//                       even) on the way into LDS, bf16 MFMA;
//   * fp16 operands  -> the same with fp16;
//   * fp32 operands, compensated ("bf16x3") -> each fp32 operand sum x is split
//                       into hi = bf16(x) and lo = bf16(x - hi); LDS holds the
//                       hi and lo tiles and every product is accumulated as
//                       hi*hi + hi*lo + lo*hi.
// The structure follows the fp32 kernel (eq. straprim1: sums formed while the
// tiles are staged, signed scatter of the accumulator in the epilogue, zero
// padding at block edges), with the operand layouts the 16-bit MFMA needs:
// every lane supplies eight consecutive k of one row of A and eight
// consecutive k of one column of B, so the B tile is transposed while it is
// staged (B is stored k-major in HBM).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace strassen {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

struct M16Tile {
    static constexpr int MT = 128, NT = 128, KT = 32;
    static constexpr int WAVES_M = 2, WAVES_N = 2;
    static constexpr int THREADS = 256;
    static constexpr int WM = 64, WN = 64, BM = 2, BN = 2;
    // A tile: row-major, k contiguous, row stride 40 elements (80 bytes): the
    // eight rows read by one 16-byte LDS cycle land in eight distinct bank
    // groups.  B tile: transposed (column j holds its k values contiguously),
    // column stride 36 elements (18 words): 32 consecutive columns map to 32
    // distinct even banks, so the 8-byte fragment reads and the 4-byte staging
    // writes are conflict free.
    static constexpr int AS = KT + 8;
    static constexpr int BS = KT + 4;
    static constexpr int GROUP = 8;
};

// Element types.  In: storage type of A and B.  Mf: MFMA operand type.
struct Bf16Ops {
    using In = unsigned short;  // raw bf16 bits
    static constexpr bool kX3 = false;
    static constexpr int kInVec = 8;  // elements per 16-byte load
    __device__ static float to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
    __device__ static unsigned short from_f32(float f) {
        const __bf16 b = (__bf16)f;
        return __builtin_bit_cast(unsigned short, b);
    }
};

struct F16Ops {
    using In = unsigned short;  // raw fp16 bits
    static constexpr bool kX3 = false;
    static constexpr int kInVec = 8;
    __device__ static float to_f32(unsigned short h) {
        return (float)__builtin_bit_cast(_Float16, h);
    }
    __device__ static unsigned short from_f32(float f) {
        const _Float16 v = (_Float16)f;
        return __builtin_bit_cast(unsigned short, v);
    }
};

struct X3Ops {
    using In = float;
    static constexpr bool kX3 = true;
    static constexpr int kInVec = 4;
    __device__ static unsigned short from_f32(float f) {
        const __bf16 b = (__bf16)f;
        return __builtin_bit_cast(unsigned short, b);
    }
    __device__ static float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
};

// Raw register image of eight consecutive elements of one operand row.
template <class Ops> struct Raw8;
template <> struct Raw8<Bf16Ops> { u16x8 v; };
template <> struct Raw8<F16Ops> { u16x8 v; };
template <> struct Raw8<X3Ops> { f32x4 v0, v1; };

// Loads elements (r, c..c+7) of a block; zero outside rows x cols.  fast: the
// whole run is inside the block and 16-byte aligned (no predicates); lanes
// whose elements are outside never access memory.
template <class Ops>
__device__ __forceinline__ Raw8<Ops> load8(const typename Ops::In *__restrict__ base, int64_t ld,
                                           int r, int c, int rows, int cols, bool fast, bool vec) {
    Raw8<Ops> out;
    const typename Ops::In *p = base + (int64_t)r * ld + c;
    if constexpr (Ops::kX3) {
        out.v0 = f32x4{0.f, 0.f, 0.f, 0.f};
        out.v1 = out.v0;
        if (fast || (r < rows && vec && c + 7 < cols)) {
            out.v0 = *reinterpret_cast<const f32x4 *>(p);
            out.v1 = *reinterpret_cast<const f32x4 *>(p + 4);
        } else if (r < rows) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + e < cols) out.v0[e] = p[e];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + 4 + e < cols) out.v1[e] = p[4 + e];
        }
    } else {
        out.v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (fast || (r < rows && vec && c + 7 < cols)) {
            out.v = *reinterpret_cast<const u16x8 *>(p);
        } else if (r < rows) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (c + e < cols) out.v[e] = p[e];
        }
    }
    return out;
}

// Element e of a raw image as fp32.
template <class Ops>
__device__ __forceinline__ float elem(const Raw8<Ops> &x, int e) {
    if constexpr (Ops::kX3)
        return e < 4 ? x.v0[e] : x.v1[e - 4];
    else
        return Ops::to_f32(x.v[e]);
}

template <class Ops, int WA, int WB, int WC, bool VEC>
__global__ __launch_bounds__(M16Tile::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void strassen_m16_kernel(const LaunchArgs args) {
    using T = M16Tile;
    using In = typename Ops::In;
    constexpr int NPLANES = Ops::kX3 ? 2 : 1;  // hi (and lo) tiles
    __shared__ __attribute__((aligned(16))) unsigned short As[2][NPLANES][T::MT * T::AS];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NPLANES][T::NT * T::BS];

    const ProductArg &P = args.prod[blockIdx.z];
    const In *__restrict__ A = static_cast<const In *>(args.A);
    const In *__restrict__ B = static_cast<const In *>(args.B);
    const int64_t lda = args.lda, ldb = args.ldb;

    int tm, tn;
    tile_coords<T::GROUP>(args.tiles_m, args.tiles_n, tm, tn);
    const int row0 = tm * T::MT, col0 = tn * T::NT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % T::WAVES_M, wn = wave / T::WAVES_M;

    // A staging: thread owns rows ar and ar + 64, eight k from ac.
    const int ar = tid >> 2, ac = (tid & 3) * 8;
    // B staging: thread owns k rows 2*bk, 2*bk+1 and columns bc..bc+7.
    const int bk = tid & 15, bc = (tid >> 4) * 8;

    int a_rows, a_cols, b_rows, b_cols;
    min_extent(P.a, WA, a_rows, a_cols);
    min_extent(P.b, WB, b_rows, b_cols);
    const bool a_rows_full = row0 + T::MT <= a_rows;
    const bool b_cols_full = col0 + T::NT <= b_cols;

    Raw8<Ops> raw_a[WA][2], raw_b[WB][2];  // raw term loads of the next k-tile

    // Issue the global loads of every term of the k-tile starting at k0.
    auto stage_load = [&](int k0) {
        const bool fast = VEC && a_rows_full && b_cols_full && (k0 + T::KT <= a_cols) &&
                          (k0 + T::KT <= b_rows);
#pragma unroll
        for (int t = 0; t < WA; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                raw_a[t][p] = load8<Ops>(A + P.a[t].off, lda, row0 + ar + 64 * p, k0 + ac,
                                         P.a[t].rows, P.a[t].cols, fast, VEC);
#pragma unroll
        for (int t = 0; t < WB; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                raw_b[t][p] = load8<Ops>(B + P.b[t].off, ldb, k0 + 2 * bk + p, col0 + bc,
                                         P.b[t].rows, P.b[t].cols, fast, VEC);
    };

    // Signed sums in fp32, rounded to the MFMA type (and split into hi/lo for
    // the compensated mode), stored into LDS buffer `buf`.
    auto stage_store = [&](int buf) {
        float sa[2][8], sb[2][8];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float x = P.a[0].sign * elem<Ops>(raw_a[0][p], e);
#pragma unroll
                for (int t = 1; t < WA; ++t) x += P.a[t].sign * elem<Ops>(raw_a[t][p], e);
                sa[p][e] = x;
                float y = P.b[0].sign * elem<Ops>(raw_b[0][p], e);
#pragma unroll
                for (int t = 1; t < WB; ++t) y += P.b[t].sign * elem<Ops>(raw_b[t][p], e);
                sb[p][e] = y;
            }
        // A: one 16-byte store per row and plane.
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            u16x8 hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                hi[e] = Ops::from_f32(sa[p][e]);
                if constexpr (Ops::kX3) lo[e] = Ops::from_f32(sa[p][e] - Ops::bf16_to_f32(hi[e]));
            }
            const int off = (ar + 64 * p) * T::AS + ac;
            *reinterpret_cast<u16x8 *>(&As[buf][0][off]) = hi;
            if constexpr (Ops::kX3) *reinterpret_cast<u16x8 *>(&As[buf][NPLANES - 1][off]) = lo;
        }
        // B: transpose; one 4-byte store (two consecutive k) per column and plane.
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned short h0 = Ops::from_f32(sb[0][e]);
            const unsigned short h1 = Ops::from_f32(sb[1][e]);
            const int off = (bc + e) * T::BS + 2 * bk;
            *reinterpret_cast<unsigned *>(&Bs[buf][0][off]) = (unsigned)h0 | ((unsigned)h1 << 16);
            if constexpr (Ops::kX3) {
                const unsigned short l0 = Ops::from_f32(sb[0][e] - Ops::bf16_to_f32(h0));
                const unsigned short l1 = Ops::from_f32(sb[1][e] - Ops::bf16_to_f32(h1));
                *reinterpret_cast<unsigned *>(&Bs[buf][NPLANES - 1][off]) =
                    (unsigned)l0 | ((unsigned)l1 << 16);
            }
        }
    };

    f32x16 acc[T::BM][T::BN];
#pragma unroll
    for (int i = 0; i < T::BM; ++i)
#pragma unroll
        for (int j = 0; j < T::BN; ++j) acc[i][j] = f32x16{};

    // In MFMA step s of a k-tile, lanes 0-31 supply k = 16s + 0..7 and lanes
    // 32-63 supply k = 16s + 8..15, for A and B alike.
    const int h = lane >> 5, l32 = lane & 31;
    auto mfma = [&](const u32x4 &a, const u32x4 &b, f32x16 c) -> f32x16 {
        if constexpr (std::is_same<Ops, F16Ops>::value)
            return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                          __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                           __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int s = 0; s < T::KT / 16; ++s) {
            u32x4 af[NPLANES][T::BM], bf[NPLANES][T::BN];
#pragma unroll
            for (int q = 0; q < NPLANES; ++q) {
#pragma unroll
                for (int i = 0; i < T::BM; ++i)
                    af[q][i] = *reinterpret_cast<const u32x4 *>(
                        &As[buf][q][(wm * T::WM + i * 32 + l32) * T::AS + 16 * s + 8 * h]);
#pragma unroll
                for (int j = 0; j < T::BN; ++j) {
                    const unsigned short *pb =
                        &Bs[buf][q][(wn * T::WN + j * 32 + l32) * T::BS + 16 * s + 8 * h];
                    const u32x2 lo2 = *reinterpret_cast<const u32x2 *>(pb);
                    const u32x2 hi2 = *reinterpret_cast<const u32x2 *>(pb + 4);
                    bf[q][j] = u32x4{lo2.x, lo2.y, hi2.x, hi2.y};
                }
            }
#pragma unroll
            for (int i = 0; i < T::BM; ++i)
#pragma unroll
                for (int j = 0; j < T::BN; ++j) {
                    acc[i][j] = mfma(af[0][i], bf[0][j], acc[i][j]);
                    if constexpr (Ops::kX3) {
                        acc[i][j] = mfma(af[0][i], bf[NPLANES - 1][j], acc[i][j]);
                        acc[i][j] = mfma(af[NPLANES - 1][i], bf[0][j], acc[i][j]);
                    }
                }
        }
    };

    const int nk = (args.sk + T::KT - 1) / T::KT;
    stage_load(0);
    stage_store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) stage_load((kt + 1) * T::KT);
        compute(cur);
        if (more) stage_store(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: as in the fp32 kernel (same 32x32 accumulator layout); each
    // accumulator element is scattered to all outputs before the next one.
    float *__restrict__ C = args.C;
    const int64_t ldc = args.ldc;
    const float alpha = args.alpha, beta = args.beta;
    float g[WC];
    int64_t coff[WC];
    int crows[WC], ccols[WC], cfirst[WC];
#pragma unroll
    for (int o = 0; o < WC; ++o) {
        g[o] = P.c[o].sign * alpha;
        coff[o] = P.c[o].off;
        crows[o] = P.c[o].rows;
        ccols[o] = P.c[o].cols;
        cfirst[o] = P.c[o].first;
    }
#pragma unroll
    for (int i = 0; i < T::BM; ++i)
#pragma unroll
        for (int j = 0; j < T::BN; ++j) {
            const int cj = col0 + wn * T::WN + j * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ci = row0 + wm * T::WM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int64_t e = (int64_t)ci * ldc + cj;
                const float m = acc[i][j][r];
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    if (ci < crows[o] && cj < ccols[o]) {
                        float *pc = C + coff[o] + e;
                        const float v = g[o] * m;
                        if (cfirst[o])
                            *pc = (beta == 0.f) ? v : beta * *pc + v;
                        else
                            *pc += v;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
}

template <class Ops, int WA, int WB, int WC>
hipError_t launch_variant(const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    const dim3 grid(a.tiles_m * a.tiles_n, 1, batch);
    const dim3 block(M16Tile::THREADS);
    if (vec)
        hipLaunchKernelGGL((strassen_m16_kernel<Ops, WA, WB, WC, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((strassen_m16_kernel<Ops, WA, WB, WC, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class Ops>
hipError_t dispatch(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                    hipStream_t s) {
#define STRASSEN_CASE(X, Y, Z) \
    if (wa == X && wb == Y && wc == Z) return launch_variant<Ops, X, Y, Z>(a, batch, vec, s);
    STRASSEN_CASE(1, 1, 1)
    STRASSEN_CASE(2, 2, 2)
    STRASSEN_CASE(2, 2, 1)
    STRASSEN_CASE(1, 2, 2)
    STRASSEN_CASE(2, 1, 2)
    STRASSEN_CASE(4, 4, 4)
    STRASSEN_CASE(1, 4, 4)
    STRASSEN_CASE(2, 4, 4)
    STRASSEN_CASE(4, 1, 4)
    STRASSEN_CASE(4, 2, 4)
    STRASSEN_CASE(4, 4, 1)
    STRASSEN_CASE(4, 4, 2)
    STRASSEN_CASE(2, 2, 4)
    STRASSEN_CASE(2, 4, 2)
    STRASSEN_CASE(4, 2, 2)
#undef STRASSEN_CASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace strassen
