// fp32 Strassen primitive on the gfx950 matrix cores (template; instantiated
// per operand layout in gemm_f32_*.hip).
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
//
// Operand layouts.  Each operand is loaded in the direction it is contiguous
// in memory, so global loads are 16-byte vectors and LDS stores are 16-byte:
//   KC  (k contiguous: A as stored, or B stored transposed)  -> LDS [x][k]
//   XC  (m/n contiguous: B as stored, or A stored transposed) -> LDS [k][x],
//       or [x][k] through 4x4 register transposes (StageXT) in variants with
//       three or more operand terms
// where x is the operand's m (A) or n (B) index.  Element (x, k) of a block
// lives at off + x*ld + k (KC) or off + k*ld + x (XC).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace strassen {
namespace f32k {

// Tile shapes.  Small: 128x128x32, 4 waves of 64x64, two workgroups per CU.
// Large: 256x256x32, 8 waves of 128x64, one workgroup per CU; half the L2
// traffic per flop of Small.  LargeK16: the same with a 16-deep k-tile, for
// variants whose staging registers do not fit twice as deep.
struct Small {
    static constexpr int MT = 128, NT = 128, KT = 32;
    static constexpr int WAVES_M = 2, WAVES_N = 2;
    static constexpr int WAVES_PER_EU = 2;
    static constexpr int GROUP = 8;
};
struct Large {
    static constexpr int MT = 256, NT = 256, KT = 32;
    static constexpr int WAVES_M = 2, WAVES_N = 4;
    static constexpr int WAVES_PER_EU = 2;
    static constexpr int GROUP = 4;
};
// Large with a 16-deep k-tile: variants with more than four operand terms in
// total have no registers for 32-deep staging.
struct LargeK16 {
    static constexpr int MT = 256, NT = 256, KT = 16;
    static constexpr int WAVES_M = 2, WAVES_N = 4;
    static constexpr int WAVES_PER_EU = 2;
    static constexpr int GROUP = 4;
};

// Staging of an m/n-contiguous operand kept [x][k] in LDS instead ("XT"),
// so that its fragments are 16-byte reads like a k-contiguous operand's.
// Each thread loads 4 consecutive k rows of one 4-wide x quad (every load
// instruction still covers whole rows across the wave) and stores the
// transposed 4x4 block as four 16-byte rows.  Row stride KT + 8 and the
// 4-wide k group XOR swizzled by (x / 4) mod 8: measured on gfx950 with a
// microbenchmark of exactly these two access patterns, the stores (lanes
// writing rows 4 apart) are free of bank conflicts and the fragment reads
// (32 consecutive rows per half wave) take 4 conflict cycles per
// instruction; stride KT + 4 with a swizzle by x / 16 measured 8 and 4, and
// no swizzle 24 and 0.  (The stores behave like 32 banks served 8 lanes at a
// time, the 16-byte reads like 128 banks served 32 lanes at a time.)
template <int X, int KT, int THREADS>
struct StageXT {
    static constexpr int LDX = KT + 8;
    static constexpr int SIZE = X * LDX;
    static constexpr int VECS = X * KT / 4 / THREADS;  // float4 per thread per term
    static constexpr int QX = X / 4;                   // x quads per k row
    static constexpr int NG = KT / 4;                  // k groups
    static constexpr int GSTEP = THREADS / QX;         // k groups per 4 loads
    static_assert(VECS % 4 == 0 && THREADS % QX == 0, "whole 4x4 blocks");
    static_assert((NG & (NG - 1)) == 0, "power-of-two k groups");

    // Load p of thread tid: first x of the quad and its k row.
    __device__ static void coords(int tid, int p, int &x, int &k) {
        x = (tid % QX) * 4;
        k = 4 * (tid / QX + (p / 4) * GSTEP) + (p % 4);
    }
    // LDS offset of element (x, k), k a multiple of 4 (start of a group).
    __device__ static int lds(int x, int k) { return x * LDX + 4 * ((k / 4) ^ ((x / 4) % NG)); }
};

// Staging geometry of one operand tile of X x KT elements.
template <int X, int KT, int THREADS, bool KC>
struct Stage {
    static constexpr int LDX = KC ? KT + 4 : X + 4;  // LDS row stride (floats)
    static constexpr int SIZE = KC ? X * LDX : KT * LDX;
    static constexpr int VECS = X * KT / 4 / THREADS;  // float4 per thread per term
    static constexpr int QUADS = KC ? KT / 4 : X / 4;  // float4 per contiguous line
    static constexpr int LINE_STEP = THREADS / QUADS;  // lines advanced per vector
    static_assert(VECS * THREADS * 4 == X * KT, "tile split");
    static_assert(THREADS % QUADS == 0, "whole lines per pass");

    // Vector p of thread tid: element offset (x, k) of its first element.
    __device__ static void coords(int tid, int p, int &x, int &k) {
        const int line = tid / QUADS + p * LINE_STEP, q = (tid % QUADS) * 4;
        if (KC) {
            x = line;
            k = q;
        } else {
            x = q;
            k = line;
        }
    }
    // LDS offset of the first element of a stored vector.
    __device__ static int lds(int x, int k) { return KC ? x * LDX + k : k * LDX + x; }
};

// Loads the 4-vector of a block starting at (x, k) (consecutive along k for
// KC, along x for XC), zero outside xs x ks.  Lanes whose elements are
// outside never access memory.
template <bool KC>
__device__ __forceinline__ f32x4 load4_guarded(const float *__restrict__ base, int64_t ld, int x,
                                               int k, int xs, int ks, bool vec) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    // the line index (fixed for the 4 elements) and the run index (varies)
    const int line = KC ? x : k, run = KC ? k : x;
    const int lines = KC ? xs : ks, runs = KC ? ks : xs;
    if (line < lines) {
        const float *p = base + (int64_t)line * ld + run;
        if (vec && run + 3 < runs) {
            v = *reinterpret_cast<const f32x4 *>(p);
        } else {
            if (run + 0 < runs) v.x = p[0];
            if (run + 1 < runs) v.y = p[1];
            if (run + 2 < runs) v.z = p[2];
            if (run + 3 < runs) v.w = p[3];
        }
    }
    return v;
}

// CONC: concurrent schedule -- the launch mixes products of different
// variants (W_A, W_B, W_C are upper bounds, the product's own counts are
// read at run time) and outputs are added with fp32 atomics, beta having been
// applied beforehand; otherwise every term is used and the first update of a
// C block applies beta.
template <class Cfg, bool A_KC, bool B_KC, int WA, int WB, int WC, bool CONC>
__global__ __launch_bounds__(64 * Cfg::WAVES_M * Cfg::WAVES_N)
__attribute__((amdgpu_waves_per_eu(Cfg::WAVES_PER_EU, Cfg::WAVES_PER_EU)))
void strassen_f32_kernel(const LaunchArgs args, const int vec_flag) {
    const bool VEC = vec_flag != 0;
    constexpr int MT = Cfg::MT, NT = Cfg::NT, KT = Cfg::KT;
    constexpr int THREADS = 64 * Cfg::WAVES_M * Cfg::WAVES_N;
    constexpr int WM = MT / Cfg::WAVES_M, WN = NT / Cfg::WAVES_N;  // wave tile
    constexpr int BM = WM / 32, BN = WN / 32;  // 32x32 MFMA blocks per wave
    // m/n-contiguous operands are kept [x][k] (StageXT) in variants with at
    // least three operand terms, where the 16-byte fragment reads measured
    // faster (+4 % for (2,2,1)); with one term each the [k][x] layout is
    // slightly faster.
    constexpr bool XT_VARIANT = WA + WB >= 3;
    constexpr bool A_XT = !A_KC && XT_VARIANT && (MT * KT / 4 / THREADS) % 4 == 0;
    constexpr bool B_XT = !B_KC && XT_VARIANT && (NT * KT / 4 / THREADS) % 4 == 0;
    using SA = typename std::conditional<A_XT, StageXT<MT, KT, THREADS>, Stage<MT, KT, THREADS, A_KC>>::type;
    using SB = typename std::conditional<B_XT, StageXT<NT, KT, THREADS>, Stage<NT, KT, THREADS, B_KC>>::type;
    static_assert(KT % 8 == 0, "k chunks of 8");

    __shared__ __attribute__((aligned(16))) float As[2][SA::SIZE];
    __shared__ __attribute__((aligned(16))) float Bs[2][SB::SIZE];

    const ProductArg &P = args.prod[blockIdx.z];
    const float *__restrict__ A = static_cast<const float *>(args.A);
    const float *__restrict__ B = static_cast<const float *>(args.B);
    const int64_t lda = args.lda, ldb = args.ldb;

    int tm, tn;
    tile_coords<Cfg::GROUP>(args.tiles_m, args.tiles_n, tm, tn);
    const int row0 = tm * MT, col0 = tn * NT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;

    // Terms in use (all of them unless the schedule is concurrent).
    const int na = CONC ? P.na : WA, nb = CONC ? P.nb : WB, nc = CONC ? P.nc : WC;

    // Extents shared by every term: x (m for A, n for B) and k.
    int a_x, a_k, b_x, b_k;
    min_extent(P.a, na, a_x, a_k);  // A terms: rows = m extent, cols = k extent
    min_extent(P.b, nb, b_k, b_x);  // B terms: rows = k extent, cols = n extent
    const bool a_x_full = row0 + MT <= a_x;
    const bool b_x_full = col0 + NT <= b_x;

    f32x4 raw_a[WA][SA::VECS];
    f32x4 raw_b[WB][SB::VECS];

    // In-bounds k-tiles: loads of k-tiles [0, nfast) need no guard.  They
    // are buffer loads: each term's base (scalar registers, advanced one
    // k-tile per step) plus a per-thread 32-bit byte offset that does not
    // change along k.
    constexpr uint64_t kOffLimit = 1ull << 32;
    const bool a_off32 = (uint64_t)(A_KC ? MT : KT) * (uint64_t)lda * 4u < kOffLimit;
    const bool b_off32 = (uint64_t)(B_KC ? NT : KT) * (uint64_t)ldb * 4u < kOffLimit;
    const int nfast = (VEC && a_x_full && b_x_full && a_off32 && b_off32)
                          ? (a_k < b_k ? a_k : b_k) / KT : 0;
    uint32_t a_off[SA::VECS], b_off[SB::VECS];
#pragma unroll
    for (int p = 0; p < SA::VECS; ++p) {
        int x, k;
        SA::coords(tid, p, x, k);
        a_off[p] = 4u * (A_KC ? (uint32_t)x * (uint32_t)lda + k : (uint32_t)k * (uint32_t)lda + x);
    }
#pragma unroll
    for (int p = 0; p < SB::VECS; ++p) {
        int x, k;
        SB::coords(tid, p, x, k);
        b_off[p] = 4u * (B_KC ? (uint32_t)x * (uint32_t)ldb + k : (uint32_t)k * (uint32_t)ldb + x);
    }
    const int64_t a_step = 4 * (A_KC ? (int64_t)KT : (int64_t)KT * lda);
    const int64_t b_step = 4 * (B_KC ? (int64_t)KT : (int64_t)KT * ldb);
    const int64_t a_org = A_KC ? (int64_t)row0 * lda : row0;
    const int64_t b_org = B_KC ? (int64_t)col0 * ldb : col0;

    auto issue_fast_a = [&](int kt) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < WA; ++t) {
            if (t < na) {
                const auto r = raw_rsrc(reinterpret_cast<const char *>(A + P.a[t].off + a_org) +
                                        a_step * kt);
#pragma unroll
                for (int p = 0; p < SA::VECS; ++p) raw_a[t][p] = buffer_load16<f32x4>(r, a_off[p]);
            }
        }
    };
    auto issue_fast_b = [&](int kt) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < WB; ++t) {
            if (t < nb) {
                const auto r = raw_rsrc(reinterpret_cast<const char *>(B + P.b[t].off + b_org) +
                                        b_step * kt);
#pragma unroll
                for (int p = 0; p < SB::VECS; ++p) raw_b[t][p] = buffer_load16<f32x4>(r, b_off[p]);
            }
        }
    };
    // Loads of terms [t0, t1) only (the split staging below).
    auto issue_fast_a_terms = [&](int kt, int t0, int t1) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < WA; ++t) {
            if (t >= t0 && t < t1) {
                const auto r = raw_rsrc(reinterpret_cast<const char *>(A + P.a[t].off + a_org) +
                                        a_step * kt);
#pragma unroll
                for (int p = 0; p < SA::VECS; ++p) raw_a[t][p] = buffer_load16<f32x4>(r, a_off[p]);
            }
        }
    };
    auto issue_fast_b_terms = [&](int kt, int t0, int t1) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < WB; ++t) {
            if (t >= t0 && t < t1) {
                const auto r = raw_rsrc(reinterpret_cast<const char *>(B + P.b[t].off + b_org) +
                                        b_step * kt);
#pragma unroll
                for (int p = 0; p < SB::VECS; ++p) raw_b[t][p] = buffer_load16<f32x4>(r, b_off[p]);
            }
        }
    };
    auto issue_fast = [&](int kt) __attribute__((always_inline)) {
        issue_fast_a(kt);
        issue_fast_b(kt);
    };

    // Loads of any k-tile, each element guarded against its term's extents.
    auto issue_a = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int p = 0; p < SA::VECS; ++p) {
            int x, k;
            SA::coords(tid, p, x, k);
#pragma unroll
            for (int t = 0; t < WA; ++t)
                if (t < na) raw_a[t][p] = load4_guarded<A_KC>(A + P.a[t].off, lda, row0 + x, k0 + k,
                                                  P.a[t].rows, P.a[t].cols, VEC);
        }
    };
    auto issue_b = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int p = 0; p < SB::VECS; ++p) {
            int x, k;
            SB::coords(tid, p, x, k);
#pragma unroll
            for (int t = 0; t < WB; ++t)
                if (t < nb) raw_b[t][p] = load4_guarded<B_KC>(B + P.b[t].off, ldb, col0 + x, k0 + k,
                                                  P.b[t].cols, P.b[t].rows, VEC);
        }
    };
    auto issue = [&](int k0) __attribute__((always_inline)) {
        issue_a(k0);
        issue_b(k0);
    };

    // Form the signed operand sums and store them into LDS buffer `buf`.
    // The sign of each operand's first term is factored out of its sum and
    // applied in the epilogue (signs are +-1, so the staged values change by
    // that exact negation only): the stored sum is x_0 + sum_t (s_t s_0) x_t,
    // and a single-term operand is stored as loaded.
    auto store_operand = [&](auto stage, auto xt, float *tile, f32x4 (*raw)[decltype(stage)::VECS],
                             auto nterms, int n_use, const TermArg *terms) __attribute__((always_inline)) {
        using S = decltype(stage);
        constexpr int NT_ = decltype(nterms)::value;
        auto sum = [&](int p) __attribute__((always_inline)) {
            f32x4 v = raw[0][p];
#pragma unroll
            for (int t = 1; t < NT_; ++t)
                if (t < n_use) v += raw[t][p] * (terms[t].sign * terms[0].sign);
            return v;
        };
        if constexpr (decltype(xt)::value) {
#pragma unroll
            for (int p0 = 0; p0 < S::VECS; p0 += 4) {
                const f32x4 r0 = sum(p0), r1 = sum(p0 + 1), r2 = sum(p0 + 2), r3 = sum(p0 + 3);
                int x, k;
                S::coords(tid, p0, x, k);
                *reinterpret_cast<f32x4 *>(&tile[S::lds(x + 0, k)]) = f32x4{r0[0], r1[0], r2[0], r3[0]};
                *reinterpret_cast<f32x4 *>(&tile[S::lds(x + 1, k)]) = f32x4{r0[1], r1[1], r2[1], r3[1]};
                *reinterpret_cast<f32x4 *>(&tile[S::lds(x + 2, k)]) = f32x4{r0[2], r1[2], r2[2], r3[2]};
                *reinterpret_cast<f32x4 *>(&tile[S::lds(x + 3, k)]) = f32x4{r0[3], r1[3], r2[3], r3[3]};
            }
        } else {
#pragma unroll
            for (int p = 0; p < S::VECS; ++p) {
                const f32x4 v = sum(p);
                int x, k;
                S::coords(tid, p, x, k);
                *reinterpret_cast<f32x4 *>(&tile[S::lds(x, k)]) = v;
            }
        }
    };
    auto store_a = [&](int buf) __attribute__((always_inline)) {
        store_operand(SA{}, std::integral_constant<bool, A_XT>{}, &As[buf][0], raw_a,
                      std::integral_constant<int, WA>{}, na, P.a);
    };
    auto store_b = [&](int buf) __attribute__((always_inline)) {
        store_operand(SB{}, std::integral_constant<bool, B_XT>{}, &Bs[buf][0], raw_b,
                      std::integral_constant<int, WB>{}, nb, P.b);
    };
    auto sum_store = [&](int buf) __attribute__((always_inline)) {
        store_a(buf);
        store_b(buf);
    };

    f32x16 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = f32x16{};

    // k order inside a chunk of 8: in MFMA step e, lanes 0-31 contribute
    // k = 4*0 + e and lanes 32-63 contribute k = 4*1 + e, for A and B alike.
    // A KC operand gives a lane its values for four steps in one 16-byte read;
    // an XC operand is read one 4-byte value per step (32 consecutive x).
    const int h = lane >> 5, l32 = lane & 31;
    auto compute = [&](int buf, int c0, int c1) __attribute__((always_inline)) {
        const float *as = &As[buf][0];
        const float *bs = &Bs[buf][0];
#pragma unroll
        for (int c = c0; c < c1; ++c) {
            f32x4 af[BM], bf[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i) {
                const int x = wm * WM + i * 32 + l32;
                if (A_KC || A_XT)
                    af[i] = *reinterpret_cast<const f32x4 *>(&as[SA::lds(x, c * 8 + h * 4)]);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) af[i][e] = as[SA::lds(x, c * 8 + h * 4 + e)];
            }
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                const int x = wn * WN + j * 32 + l32;
                if (B_KC || B_XT)
                    bf[j] = *reinterpret_cast<const f32x4 *>(&bs[SB::lds(x, c * 8 + h * 4)]);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) bf[j][e] = bs[SB::lds(x, c * 8 + h * 4 + e)];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < BM; ++i)
#pragma unroll
                    for (int j = 0; j < BN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][e], bf[j][e],
                                                                         acc[i][j], 0, 0, 0);
        }
    };

    const int nk = (args.sk + KT - 1) / KT;
    // Scheduling-group sizes of the steady loop below: LDS fragment reads
    // per 8-deep chunk, 16-byte LDS stores per k-tile, MFMAs per store.
    constexpr int kFragReads = BM * ((A_KC || A_XT) ? 1 : 4) + BN * ((B_KC || B_XT) ? 1 : 4);
    constexpr int kStores = SA::VECS + SB::VECS;
    constexpr int kMfmaPerStore = (4 * BM * BN) / kStores > 0 ? (4 * BM * BN) / kStores : 1;
    static_assert(KT / 8 >= 2, "two chunks per k-tile");
    // Staggered staging (16-deep large tiles, i.e. variants with more than
    // four operand terms): A's terms are loaded and summed first, then B's,
    // so only one operand's raw terms occupy registers at a time (+3-6 %
    // measured for the (4,4,x) and (2,4,x) variants).
    constexpr bool kStagger = std::is_same<Cfg, LargeK16>::value;
    if constexpr (kStagger) {
        if (nfast > 0) {
            issue_fast_a(0);
            store_a(0);
            issue_fast_b(0);
            store_b(0);
        } else {
            issue_a(0);
            store_a(0);
            issue_b(0);
            store_b(0);
        }
    } else {
        if (nfast > 0)
            issue_fast(0);
        else
            issue(0);
        sum_store(0);
    }
    __syncthreads();
    int kt = 0;
    // Steady state: the next k-tile is in bounds, no guards, no branches.
    if constexpr (kStagger)
    for (; kt + 1 < nfast; ++kt) {
        // A's loads, the first half of the MFMAs, A's sums and stores, B's
        // loads, the second half, B's sums and stores.
        const int cur = kt & 1;
        issue_fast_a(kt + 1);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 0, KT / 16);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (WA != 2) {
            // B's loads first, then A's sums and stores woven between the
            // second half's MFMAs (+0.9-1.8 % for the seven such variants
            // with W_A = 1 or 4, bit-identical; W_A = 2 measured 0 and -1 %)
            issue_fast_b(kt + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute(cur, KT / 16, KT / 8);
            store_a(cur ^ 1);
            __builtin_amdgcn_sched_group_barrier(0x100, kFragReads, 0);
#pragma unroll
            for (int i = 0; i < SA::VECS; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, (4 * BM * BN) / SA::VECS, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 4 * (WA - 1) + 2, 0);
                __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
            }
        } else {
            store_a(cur ^ 1);
            issue_fast_b(kt + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute(cur, KT / 16, KT / 8);
        }
        __builtin_amdgcn_sched_barrier(0);
        store_b(cur ^ 1);
        __syncthreads();
    }
    // Split staging (32-deep large tiles with more than four operand terms,
    // the (4,1,4) and (4,2,2) variants): each operand's terms are loaded two
    // at a time and the second folded into the first term's registers
    // before the next two are loaded, so at most the partial sum and two raw
    // terms are live; the additions keep the order of the plain sum (results
    // bit-identical to the 16-deep kernels).  +4.3 % (4,1,4), +5.6 % (4,2,2)
    // against the 16-deep staggered loop; the other four-term variants
    // spill 130-660 more bytes this way and measured up to 21 % slower.
    constexpr bool kSplit = std::is_same<Cfg, Large>::value && WA + WB > 4 && !CONC;
    if constexpr (kSplit)
    for (; kt + 1 < nfast; ++kt) {
        const int cur = kt & 1;
        constexpr int HA = WA > 2 ? 2 : WA, HB = WB > 2 ? 2 : WB;
        issue_fast_a_terms(kt + 1, 0, HA);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 0, 1);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (WA > 2) {
#pragma unroll
            for (int p = 0; p < SA::VECS; ++p) raw_a[0][p] += raw_a[1][p] * (P.a[1].sign * P.a[0].sign);
#pragma unroll
            for (int p = 0; p < SA::VECS; ++p) raw_a[1][p] = f32x4{0.f, 0.f, 0.f, 0.f};
            issue_fast_a_terms(kt + 1, 2, WA);
        }
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 1, 2);
        __builtin_amdgcn_sched_barrier(0);
        store_a(cur ^ 1);
        issue_fast_b_terms(kt + 1, 0, HB);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 2, 3);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (WB > 2) {
#pragma unroll
            for (int p = 0; p < SB::VECS; ++p) raw_b[0][p] += raw_b[1][p] * (P.b[1].sign * P.b[0].sign);
#pragma unroll
            for (int p = 0; p < SB::VECS; ++p) raw_b[1][p] = f32x4{0.f, 0.f, 0.f, 0.f};
            issue_fast_b_terms(kt + 1, 2, WB);
        }
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 3, 4);
        __builtin_amdgcn_sched_barrier(0);
        store_b(cur ^ 1);
        __syncthreads();
    }
    if constexpr (!kStagger && !kSplit)
    for (; kt + 1 < nfast; ++kt) {
        const int cur = kt & 1;
        issue_fast(kt + 1);
        // Loads first, then the MFMAs of all but the last two chunks, then
        // the next-to-last chunk with the sums and LDS stores of the next
        // k-tile (its buffer is idle) woven between its MFMAs, then the last
        // chunk: the loads have half a k-tile or more to land, and the
        // stores, a burst of ~64 KB per CU when every wave issued them at
        // once, now trickle out between MFMAs (+1.4 % W = 1, +1.3-3.2 % for
        // the one-level variants, results bit-identical).  The scheduling
        // barriers keep that order (left to itself the scheduler moves the
        // sums next to the loads and exposes their latency).
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, 0, KT / 8 - 2);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, KT / 8 - 2, KT / 8 - 1);
        sum_store(cur ^ 1);
        // that chunk's fragment reads, then per 16-byte store: a share of
        // the chunk's MFMAs, up to four sums, the store
        __builtin_amdgcn_sched_group_barrier(0x100, kFragReads, 0);
#pragma unroll
        for (int i = 0; i < kStores; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, kMfmaPerStore, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * BM * BN, 0);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, KT / 8 - 1, KT / 8);
        __syncthreads();
    }
    // Remaining k-tiles (fringe workgroups, a ragged last k-tile).
    for (; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if constexpr (kStagger) {
            if (more) issue_a((kt + 1) * KT);
            compute(cur, 0, KT / 16);
            if (more) {
                store_a(cur ^ 1);
                issue_b((kt + 1) * KT);
            }
            compute(cur, KT / 16, KT / 8);
            if (more) store_b(cur ^ 1);
        } else {
            if (more) issue((kt + 1) * KT);
            compute(cur, 0, KT / 8);
            if (more) sum_store(cur ^ 1);
        }
        __syncthreads();
    }

    // Epilogue: C_o += sign_o * s_a0 * s_b0 * alpha * M' for every output
    // block (M' the product of the sign-folded operand sums); the first
    // update of a block in launch order applies beta instead of reading C
    // twice.  32x32 accumulator layout: lane l, register r holds row
    // 8*(r/4) + 4*(l/32) + r%4, column l%32.  Each accumulator element is
    // scattered to all outputs before the next one, so only one element
    // offset is live at a time.
    float *__restrict__ C = args.C;
    const int64_t ldc = args.ldc;
    const float alpha = args.alpha, beta = args.beta;
    float g[WC];
    int64_t coff[WC];
    int crows[WC], ccols[WC], cfirst[WC];
#pragma unroll
    for (int o = 0; o < WC; ++o) {
        g[o] = P.c[o].sign * (P.a[0].sign * P.b[0].sign) * alpha;
        coff[o] = P.c[o].off;
        crows[o] = P.c[o].rows;
        ccols[o] = P.c[o].cols;
        cfirst[o] = P.c[o].first;
    }
    // Interior tiles (every output block covers the whole tile): no
    // per-element guards, so each block's 16 reads of C per output are issued
    // together before its stores.
    bool c_full = !CONC;
#pragma unroll
    for (int o = 0; o < WC; ++o)
        c_full = c_full && row0 + MT <= crows[o] && col0 + NT <= ccols[o];
    if (c_full) {
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                const int cj = col0 + wn * WN + j * 32 + l32;
                const int ci0 = row0 + wm * WM + i * 32 + 4 * h;
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    float *pc = C + coff[o] + (int64_t)ci0 * ldc + cj;
                    const bool read = !(cfirst[o] && beta == 0.f);
                    const float cb = cfirst[o] ? beta : 1.f;
                    if (read) {
                        float cv[16];
#pragma unroll
                        for (int r = 0; r < 16; ++r) cv[r] = pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc];
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] = cb * cv[r] + g[o] * acc[i][j][r];
                    } else {
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] = g[o] * acc[i][j][r];
                    }
                    // one output's C values live at a time
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
            const int cj = col0 + wn * WN + j * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ci = row0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int64_t e = (int64_t)ci * ldc + cj;
                const float m = acc[i][j][r];
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    if (o < nc && ci < crows[o] && cj < ccols[o]) {
                        float *pc = C + coff[o] + e;
                        const float v = g[o] * m;
                        if (CONC)
                            atomicAdd(pc, v);
                        else if (cfirst[o])
                            *pc = (beta == 0.f) ? v : beta * *pc + v;
                        else
                            *pc += v;
                    }
                }
            }
            // keep the scheduler from hoisting the next block's C traffic
            // above this one (bounds the live registers of the epilogue)
            __builtin_amdgcn_sched_barrier(0);
        }
}

template <class Cfg, bool A_KC, bool B_KC, int WA, int WB, int WC, bool CONC = false>
hipError_t launch_variant(const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    const dim3 grid(a.tiles_m * a.tiles_n, 1, batch);
    const dim3 block(64 * Cfg::WAVES_M * Cfg::WAVES_N);
    hipLaunchKernelGGL((strassen_f32_kernel<Cfg, A_KC, B_KC, WA, WB, WC, CONC>), grid, block, 0, s,
                       a, vec ? 1 : 0);
    return hipGetLastError();
}

// Concurrent schedule: up to two (one level) or four (two levels) terms per
// operand and output, counts read per product.
// Large tiles take the 16-deep k-tile when the variant has more than four
// operand terms, except (4,1,4) and (4,2,2) with A and B as stored, which
// take the 32-deep k-tile with split staging.
template <int WA, int WB, int WC, bool A_KC, bool B_KC>
constexpr bool kSplitVariant = A_KC && !B_KC && WA == 4 && ((WB == 1 && WC == 4) || (WB == 2 && WC == 2));
template <class Cfg, int WA, int WB, int WC = 1, bool A_KC = true, bool B_KC = false>
using TileFor = typename std::conditional<
    std::is_same<Cfg, Large>::value && (WA + WB > 4) && !kSplitVariant<WA, WB, WC, A_KC, B_KC>, LargeK16,
    Cfg>::type;

template <class Cfg>
hipError_t dispatch_concurrent(int wmax, const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    if (wmax <= 2) return launch_variant<TileFor<Cfg, 2, 2>, true, false, 2, 2, 2, true>(a, batch, vec, s);
    return launch_variant<TileFor<Cfg, 4, 4>, true, false, 4, 4, 4, true>(a, batch, vec, s);
}

template <class Cfg, bool A_KC, bool B_KC>
hipError_t dispatch(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                    hipStream_t s) {
#define STRASSEN_CASE(X, Y, Z)        \
    if (wa == X && wb == Y && wc == Z) \
        return launch_variant<TileFor<Cfg, X, Y, Z, A_KC, B_KC>, A_KC, B_KC, X, Y, Z>(a, batch, vec, s);
    // plain GEMM and the one-level variants
    STRASSEN_CASE(1, 1, 1)
    STRASSEN_CASE(2, 2, 2)
    STRASSEN_CASE(2, 2, 1)
    STRASSEN_CASE(1, 2, 2)
    STRASSEN_CASE(2, 1, 2)
    // formed schedules (operands as stored): single-term products with two
    // outputs (one level) or four (two levels)
    if constexpr (A_KC && !B_KC) {
        STRASSEN_CASE(1, 1, 2)
        STRASSEN_CASE(1, 1, 4)
    }
    // hybrid two-level: one-level operands, up to four outputs
    STRASSEN_CASE(1, 2, 4)
    STRASSEN_CASE(2, 1, 4)
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

}  // namespace f32k
}  // namespace strassen
