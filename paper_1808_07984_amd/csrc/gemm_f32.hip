// fp32 Strassen primitive on the gfx950 matrix cores.
//
// One workgroup computes a MT x NT tile of one product
//     M = (sum_t sa_t A_t)(sum_t sb_t B_t)
// of a batch (blockIdx.z) and adds it, with signs, into the W_C output blocks
// (eq. straprim1; Strassen's Algorithm on NVIDIA GPUs section):
//   * A-/B-operand sums are formed in registers between the global load of
//     every term and the store of the summed tile into LDS, so only the sum
//     occupies LDS and nothing extra goes to HBM;
//   * the tile product runs on v_mfma_f32_32x32x2_f32 from LDS fragments;
//   * the fp32 accumulator is scattered to every C block once, after the k
//     loop, so M never touches HBM;
//   * blocks extending past the matrix read zeros and store nothing
//     (Handling the Fringes section).
// W_A, W_B, W_C (Register Optimization section) are template parameters, so
// a variant with one term per operand carries no extra loads or adds.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace strassen {
namespace {

struct F32Tile {
    static constexpr int MT = 128, NT = 128, KT = 32;
    static constexpr int WAVES_M = 2, WAVES_N = 2;
    static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
    static constexpr int WM = MT / WAVES_M, WN = NT / WAVES_N;  // wave tile
    static constexpr int BM = WM / 32, BN = WN / 32;            // 32x32 blocks per wave
    // LDS strides (floats).  A is kept k-contiguous per row so a lane reads
    // four consecutive k with one 16-byte load; the 4-float pad puts eight
    // consecutive rows in eight distinct 4-bank groups.  B is kept
    // n-contiguous per k so 32 lanes read 32 consecutive floats.
    static constexpr int AS = KT + 4;
    static constexpr int BS = NT + 4;
    static constexpr int A_VECS = MT * KT / 4 / THREADS;  // float4 per thread per A term
    static constexpr int B_VECS = KT * NT / 4 / THREADS;
    static constexpr int A_QUADS = KT / 4;                // float4 per A tile row
    static constexpr int B_QUADS = NT / 4;                // float4 per B tile row
    static constexpr int GROUP = 8;
    static_assert(A_VECS * THREADS * 4 == MT * KT, "A tile split");
    static_assert(B_VECS * THREADS * 4 == KT * NT, "B tile split");
    static_assert(KT % 8 == 0, "k chunks of 8");
};

// Loads four consecutive elements (r, c..c+3) of a block, zero outside
// rows x cols.  Used for tiles that touch a block edge or when vector
// alignment is not guaranteed; lanes whose element is outside never access
// memory.
__device__ __forceinline__ f32x4 load4_guarded(const float *__restrict__ base, int64_t ld,
                                               int r, int c, int rows, int cols, bool vec) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r < rows) {
        const float *p = base + (int64_t)r * ld + c;
        if (vec && c + 3 < cols) {
            v = *reinterpret_cast<const f32x4 *>(p);
        } else {
            if (c + 0 < cols) v.x = p[0];
            if (c + 1 < cols) v.y = p[1];
            if (c + 2 < cols) v.z = p[2];
            if (c + 3 < cols) v.w = p[3];
        }
    }
    return v;
}

template <int WA, int WB, int WC, bool VEC>
__global__ __launch_bounds__(F32Tile::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void strassen_f32_kernel(const LaunchArgs args) {
    using T = F32Tile;
    __shared__ __attribute__((aligned(16))) float As[2][T::MT * T::AS];
    __shared__ __attribute__((aligned(16))) float Bs[2][T::KT * T::BS];

    const ProductArg &P = args.prod[blockIdx.z];
    const float *__restrict__ A = static_cast<const float *>(args.A);
    const float *__restrict__ B = static_cast<const float *>(args.B);
    const int64_t lda = args.lda, ldb = args.ldb;

    int tm, tn;
    tile_coords<T::GROUP>(args.tiles_m, args.tiles_n, tm, tn);
    const int row0 = tm * T::MT, col0 = tn * T::NT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % T::WAVES_M, wn = wave / T::WAVES_M;

    // Staging coordinates: A vector p covers tile row ar + p*(THREADS/A_QUADS),
    // k offset ac; B vector p covers tile k-row br + p*(THREADS/B_QUADS),
    // column offset bc.  Consecutive lanes read consecutive 16-byte chunks.
    const int ar = tid / T::A_QUADS, ac = (tid % T::A_QUADS) * 4;
    const int br = tid / T::B_QUADS, bc = (tid % T::B_QUADS) * 4;
    constexpr int A_ROW_STEP = T::THREADS / T::A_QUADS;
    constexpr int B_ROW_STEP = T::THREADS / T::B_QUADS;

    int a_rows, a_cols, b_rows, b_cols;
    min_extent(P.a, WA, a_rows, a_cols);
    min_extent(P.b, WB, b_rows, b_cols);
    const bool a_rows_full = row0 + T::MT <= a_rows;
    const bool b_cols_full = col0 + T::NT <= b_cols;

    f32x4 raw_a[WA][T::A_VECS];
    f32x4 raw_b[WB][T::B_VECS];

    // Issue the global loads of every term of the k-tile starting at k0.
    auto issue = [&](int k0) {
        const bool fast = VEC && a_rows_full && b_cols_full &&
                          (k0 + T::KT <= a_cols) && (k0 + T::KT <= b_rows);
        if (fast) {
#pragma unroll
            for (int t = 0; t < WA; ++t) {
                const float *base = A + P.a[t].off + (int64_t)(row0 + ar) * lda + (k0 + ac);
#pragma unroll
                for (int p = 0; p < T::A_VECS; ++p)
                    raw_a[t][p] = *reinterpret_cast<const f32x4 *>(base + (int64_t)(p * A_ROW_STEP) * lda);
            }
#pragma unroll
            for (int t = 0; t < WB; ++t) {
                const float *base = B + P.b[t].off + (int64_t)(k0 + br) * ldb + (col0 + bc);
#pragma unroll
                for (int p = 0; p < T::B_VECS; ++p)
                    raw_b[t][p] = *reinterpret_cast<const f32x4 *>(base + (int64_t)(p * B_ROW_STEP) * ldb);
            }
        } else {
#pragma unroll
            for (int t = 0; t < WA; ++t)
#pragma unroll
                for (int p = 0; p < T::A_VECS; ++p)
                    raw_a[t][p] = load4_guarded(A + P.a[t].off, lda, row0 + ar + p * A_ROW_STEP,
                                                k0 + ac, P.a[t].rows, P.a[t].cols, VEC);
#pragma unroll
            for (int t = 0; t < WB; ++t)
#pragma unroll
                for (int p = 0; p < T::B_VECS; ++p)
                    raw_b[t][p] = load4_guarded(B + P.b[t].off, ldb, k0 + br + p * B_ROW_STEP,
                                                col0 + bc, P.b[t].rows, P.b[t].cols, VEC);
        }
    };

    // Form the signed operand sums and store them into LDS buffer `buf`.
    auto sum_store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < T::A_VECS; ++p) {
            f32x4 s = raw_a[0][p] * P.a[0].sign;
#pragma unroll
            for (int t = 1; t < WA; ++t) s += raw_a[t][p] * P.a[t].sign;
            *reinterpret_cast<f32x4 *>(&As[buf][(ar + p * A_ROW_STEP) * T::AS + ac]) = s;
        }
#pragma unroll
        for (int p = 0; p < T::B_VECS; ++p) {
            f32x4 s = raw_b[0][p] * P.b[0].sign;
#pragma unroll
            for (int t = 1; t < WB; ++t) s += raw_b[t][p] * P.b[t].sign;
            *reinterpret_cast<f32x4 *>(&Bs[buf][(br + p * B_ROW_STEP) * T::BS + bc]) = s;
        }
    };

    f32x16 acc[T::BM][T::BN];
#pragma unroll
    for (int i = 0; i < T::BM; ++i)
#pragma unroll
        for (int j = 0; j < T::BN; ++j) acc[i][j] = f32x16{};

    // k ordering inside a chunk of 8: in MFMA step e, lanes 0-31 contribute
    // k = 4*0 + e and lanes 32-63 contribute k = 4*1 + e, for A and B alike,
    // so one 16-byte LDS read gives a lane its A values for four steps.
    const int h = lane >> 5, l32 = lane & 31;
    auto compute = [&](int buf) {
        const float *as = &As[buf][0];
        const float *bs = &Bs[buf][0];
#pragma unroll
        for (int kk = 0; kk < T::KT / 8; ++kk) {
            f32x4 af[T::BM];
#pragma unroll
            for (int i = 0; i < T::BM; ++i)
                af[i] = *reinterpret_cast<const f32x4 *>(
                    &as[(wm * T::WM + i * 32 + l32) * T::AS + kk * 8 + h * 4]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float bf[T::BN];
#pragma unroll
                for (int j = 0; j < T::BN; ++j)
                    bf[j] = bs[(kk * 8 + h * 4 + e) * T::BS + wn * T::WN + j * 32 + l32];
#pragma unroll
                for (int i = 0; i < T::BM; ++i)
#pragma unroll
                    for (int j = 0; j < T::BN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][e], bf[j], acc[i][j], 0, 0, 0);
            }
        }
    };

    const int nk = (args.sk + T::KT - 1) / T::KT;
    issue(0);
    sum_store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) issue((kt + 1) * T::KT);
        compute(cur);
        if (more) sum_store(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: C_o += sign_o * alpha * M for every output block; the first
    // update of a block in launch order applies beta instead of reading C
    // twice.  32x32 accumulator layout: lane l, register r holds row
    // 8*(r/4) + 4*(l/32) + r%4, column l%32.
    float *__restrict__ C = args.C;
    const int64_t ldc = args.ldc;
    const float alpha = args.alpha, beta = args.beta;
#pragma unroll
    for (int o = 0; o < WC; ++o) {
        const TermArg co = P.c[o];
        const float g = co.sign * alpha;
        float *cb = C + co.off;
#pragma unroll
        for (int i = 0; i < T::BM; ++i)
#pragma unroll
            for (int j = 0; j < T::BN; ++j) {
                const int cj = col0 + wn * T::WN + j * 32 + l32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ci = row0 + wm * T::WM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                    if (ci < co.rows && cj < co.cols) {
                        float *pc = cb + (int64_t)ci * ldc + cj;
                        const float v = g * acc[i][j][r];
                        if (co.first)
                            *pc = (beta == 0.f) ? v : beta * *pc + v;
                        else
                            *pc += v;
                    }
                }
            }
    }
}

template <int WA, int WB, int WC>
hipError_t launch_variant(const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    const dim3 grid(a.tiles_m * a.tiles_n, 1, batch);
    const dim3 block(F32Tile::THREADS);
    if (vec)
        hipLaunchKernelGGL((strassen_f32_kernel<WA, WB, WC, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((strassen_f32_kernel<WA, WB, WC, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

KernelShape f32_tile_shape() {
    return KernelShape{F32Tile::MT, F32Tile::NT, F32Tile::KT, 4};
}

hipError_t launch_f32(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                      hipStream_t s) {
#define STRASSEN_CASE(X, Y, Z) \
    if (wa == X && wb == Y && wc == Z) return launch_variant<X, Y, Z>(a, batch, vec, s);
    // plain GEMM and the one-level variants
    STRASSEN_CASE(1, 1, 1)
    STRASSEN_CASE(2, 2, 2)
    STRASSEN_CASE(2, 2, 1)
    STRASSEN_CASE(1, 2, 2)
    STRASSEN_CASE(2, 1, 2)
    // two-level variants
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

const char *f32_kernel_name() { return "strassen_f32_kernel"; }

}  // namespace strassen
