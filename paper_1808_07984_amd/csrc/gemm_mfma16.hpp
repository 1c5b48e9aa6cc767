// Strassen primitive on the gfx950 16-bit matrix cores
// (v_mfma_f32_32x32x16_{bf16,f16}, fp32 accumulation).  Template; each
// operand type is instantiated in its own translation unit.
//
// Three operand modes share one template:
//   * bf16 operands  -> signed sums in fp32, rounded once to bf16 (nearest
//                       even) on the way into LDS, bf16 MFMA (a single-term
//                       operand is copied without arithmetic);
//   * fp16 operands  -> the same with fp16;
//   * fp32 operands, compensated ("bf16x3") -> each fp32 operand sum x is split
//                       into hi = bf16(x) and lo = bf16(x - hi); LDS holds the
//                       hi and lo tiles and every product is accumulated as
//                       hi*hi + hi*lo + lo*hi.
// The structure follows the fp32 kernel (eq. straprim1: sums formed while the
// tiles are staged, signed scatter of the accumulator in the epilogue, zero
// padding at block edges).  Every lane supplies eight consecutive k of one row
// of A and of one column of B, so both LDS tiles are kept [x][k] (x = m for A,
// n for B).  An operand that is k-contiguous in memory (A as stored, B stored
// transposed) is copied straight in with vector stores ("direct"); an operand
// that is m/n-contiguous (B as stored, A stored transposed) is transposed while
// staged: each thread loads two consecutive k rows and stores one 4-byte word
// (two k values) per column ("paired").
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace strassen {
namespace m16k {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Tile shapes.  LDS row strides are in 16-bit elements: direct tiles use
// KT + 8 (the eight rows of one 16-byte read cycle land in distinct bank
// groups), paired tiles KT + 4 (32 consecutive columns fall on 32 distinct
// even banks for the 8-byte reads, and the 4-byte staging stores of one wave
// on 64 distinct banks).  SQ_LDS_BANK_CONFLICT measures 0.7-0.9 conflict
// cycles per LDS instruction for these kernels (1.8 for the 32-deep
// compensated single-term one); LDS bandwidth is not what limits them.
template <int MT_, int NT_, int KT_, int WAVES_M_, int WAVES_N_, int GROUP_>
struct Cfg {
    static constexpr int MT = MT_, NT = NT_, KT = KT_;
    static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
    static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
    static constexpr int WM = MT / WAVES_M, WN = NT / WAVES_N;
    static constexpr int BM = WM / 32, BN = WN / 32;
    static constexpr int GROUP = GROUP_;
    static_assert(KT % 16 == 0, "k steps of 16");
};
using Small = Cfg<128, 128, 32, 2, 2, 8>;
using Large = Cfg<256, 256, 32, 2, 4, 4>;     // 16-bit operands
using LargeK64 = Cfg<256, 256, 64, 2, 4, 4>;  // 16-bit operands, at most four terms
using LargeX3 = Cfg<256, 256, 16, 2, 4, 4>;   // fp32 operands split hi/lo

// Operand types.
struct Bf16Ops {
    using In = unsigned short;  // raw bf16 bits
    using Vec = u16x8;          // one 16-byte load
    static constexpr int NV = 8;
    static constexpr bool kX3 = false;
    static constexpr bool kPreA = false, kPreB = false;
    __device__ static float to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
    __device__ static unsigned short from_f32(float f) {
        return __builtin_bit_cast(unsigned short, (__bf16)f);
    }
    // (lo, hi) rounded to nearest even and packed into one word
    __device__ static unsigned pack2(float lo, float hi) {
        return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
    }
};
struct F16Ops {
    using In = unsigned short;  // raw fp16 bits
    using Vec = u16x8;
    static constexpr int NV = 8;
    static constexpr bool kX3 = false;
    static constexpr bool kPreA = false, kPreB = false;
    __device__ static float to_f32(unsigned short h) {
        return (float)__builtin_bit_cast(_Float16, h);
    }
    __device__ static unsigned short from_f32(float f) {
        return __builtin_bit_cast(unsigned short, (_Float16)f);
    }
    __device__ static unsigned pack2(float lo, float hi) {
        return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, f16x2));
    }
};
struct X3Ops {
    using In = float;
    using Vec = f32x4;
    static constexpr int NV = 4;
    static constexpr bool kX3 = true;
    static constexpr bool kPreA = false, kPreB = false;
    __device__ static float to_f32(float x) { return x; }
    __device__ static unsigned short from_f32(float f) {
        return __builtin_bit_cast(unsigned short, (__bf16)f);
    }
    __device__ static float bf16_to_f32(unsigned short h) {
        return __uint_as_float((unsigned)h << 16);
    }
    __device__ static unsigned pack2(float lo, float hi) {
        return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
    }
};

// The compensated mode on operands already split ("pre-split", written by the
// formed schedule's sum pass): every 16-byte unit holds four consecutive
// elements as hi(e0..e3) in its first 8 bytes and lo(e0..e3) in its last 8
// (bf16 each, element e at 16-bit position e of its half), so an operand has
// the fp32 operand's size, strides and alignment, and staging it is moving
// the two halves into the two LDS planes -- the same LDS contents the split
// of the fp32 value gives.  kPreA / kPreB: which operand is pre-split (the
// other one is fp32 and split while staged).  Pre-split operands need
// 16-byte aligned units (cols and leading dimension multiples of 4).
template <bool PA, bool PB>
struct X3PreOps : X3Ops {
    static constexpr bool kPreA = PA, kPreB = PB;
};

// Staging geometry of one operand (X = MT or NT rows of the [x][k] tile).
// direct: units of one x row and NV consecutive k; paired: units of two
// consecutive k rows and NV consecutive x (X / NV / 8 and KT / 16 whole
// blocks of 8 x 8 units).
template <class C, class Ops, int X, bool DIRECT, bool ONE_TERM>
struct Stage {
    static constexpr int NV = Ops::NV;
    static constexpr int LDX = DIRECT ? C::KT + 8 : C::KT + 4;
    static constexpr int SIZE = X * LDX;
    static constexpr int UNITS = DIRECT ? X * C::KT / NV : (C::KT / 2) * (X / NV);
    static constexpr int VECS = UNITS / C::THREADS;  // units per thread per term
    static constexpr int LOADS = DIRECT ? 1 : 2;     // global vectors per unit
    static_assert(VECS * C::THREADS == UNITS, "tile split");
    static_assert(DIRECT || ((X / NV) % 8 == 0 && (C::KT / 2) % 8 == 0), "8 x 8 unit blocks");
    // Single-term paired 16-bit tiles 256 wide: consecutive lanes take
    // consecutive x units of one k row pair, so one load instruction covers
    // two rows (8 cache lines instead of 32; the 32-row spread filled the
    // texture-address queue of these buffer-load kernels for 13 % of their
    // cycles).  The staging stores of one wave then hit rows 8 apart; the
    // 4-element groups of each LDS row are XOR-swizzled with (x / 32) mod 8,
    // which spreads those stores and the fragment reads over all 64 banks of
    // a 64-bank, 4-byte model (checked for KT = 32 and 64; the hardware
    // counts 0.7 conflict cycles per LDS instruction, the change measured
    // +4 % for bf16 W = 1).  Other paired tiles (summed operands, whose
    // staging needs the registers that swizzled fragment addresses would
    // take, and narrower or compensated ones) give each wave an 8 x 8 block
    // of (k row pair, x unit): lanes 0-7 step through the row pairs, so one
    // load instruction covers 8 rows of 128 contiguous bytes (8 cache
    // lines; the earlier k-major order spread it over 16-32 rows).
    // Measured +4 % (2,2,1), +6 % (2,2,2), +2 % (1,2,2), +2-3 % for the
    // four-term operands, results bit-identical.  The hardware counts 0.9
    // bank-conflict cycles per LDS instruction for these kernels (0 for the
    // k-major order): lanes x units 4 apart share banks, and the store of
    // lanes 0-15 appears to be served together with lanes 32-47.  Reordering
    // the x units across lanes to separate them measured no faster.
    static constexpr bool SWZ = !DIRECT && NV == 8 && X >= 256 && ONE_TERM;

    // Unit p of thread tid: first (x, k) it covers.
    __device__ static void coords(int tid, int p, int &x, int &k) {
        const int u = tid + p * C::THREADS;
        if (DIRECT) {
            constexpr int PER_ROW = C::KT / NV;
            x = u / PER_ROW;
            k = (u % PER_ROW) * NV;
        } else if (SWZ) {
            constexpr int PER_ROW = X / NV;
            x = (u % PER_ROW) * NV;
            k = 2 * (u / PER_ROW);
        } else {
            // each wave: 8 row pairs x 8 consecutive 16-byte x units
            constexpr int XB = X / NV / 8;
            const int b = u / 64, lane = u % 64;
            x = NV * (8 * (b % XB) + lane / 8);
            k = 2 * (8 * (b / XB) + lane % 8);
        }
    }
    // Offset of element (x, k) in the tile (paired layouts: k even or a
    // multiple of 4).  Rows x .. x + 7 of one staging unit (x a multiple of
    // 8) share the swizzle, so their offsets are at(x, k) + e * LDX.
    __device__ static int at(int x, int k) {
        if (SWZ) return x * LDX + 4 * ((k >> 2) ^ ((x >> 5) & 7)) + (k & 3);
        return x * LDX + k;
    }
};

// Loads NV consecutive elements of a block starting at (line, run), zero
// outside lines x runs.  fast: the whole run is inside and aligned.  Lanes
// whose elements are outside never access memory.
// Waits until at most N vector-memory loads of this wave are in flight
// (expcnt and lgkmcnt are left alone).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Waits until none of this wave's vector-memory loads and LDS reads is in
// flight (expcnt is left alone).
__device__ __forceinline__ void wait_vmcnt_lgkmcnt0() { __builtin_amdgcn_s_waitcnt(7 << 4); }

typedef short i16x4 __attribute__((ext_vector_type(4)));

// PRE: a pre-split operand (whole 16-byte units only: a unit that crosses the
// extent is loaded whole and its hi and lo halves of the elements outside are
// cleared).
template <class Ops, bool PRE = false>
__device__ __forceinline__ typename Ops::Vec load_vec(const typename Ops::In *__restrict__ base,
                                                      int64_t ld, int line, int run, int lines,
                                                      int runs, bool fast, bool vec) {
    using V = typename Ops::Vec;
    constexpr int NV = Ops::NV;
    V v;
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = 0;
    const typename Ops::In *p = base + (int64_t)line * ld + run;
    if constexpr (PRE) {
        static_assert(NV == 4, "pre-split units hold four elements");
        if (fast || (line < lines && run + NV - 1 < runs)) return *reinterpret_cast<const V *>(p);
        if (line < lines && run < runs) {
            u32x4 w = __builtin_bit_cast(u32x4, *reinterpret_cast<const V *>(p));
#pragma unroll
            for (int e = 0; e < NV; ++e)
                if (run + e >= runs) {
                    const unsigned keep = (e & 1) ? 0x0000ffffu : 0xffff0000u;
                    w[e >> 1] &= keep;
                    w[2 + (e >> 1)] &= keep;
                }
            v = __builtin_bit_cast(V, w);
        }
        return v;
    }
    if (fast || (line < lines && vec && run + NV - 1 < runs)) {
        v = *reinterpret_cast<const V *>(p);
    } else if (line < lines) {
#pragma unroll
        for (int e = 0; e < NV; ++e)
            if (run + e < runs) v[e] = p[e];
    }
    return v;
}

// CHAIN: a workgroup computes two products of one chain (prod[2z] and
// prod[2z + 1], single-term operands) into one accumulator: the first
// product's outputs except the carried one are written after its k loop, the
// accumulator (negated when the signs require it) then collects the second
// product, and the sum goes to the carried C block in one update.  A product
// with a single output thus costs no read-modify-write of C of its own.
template <class C, class Ops, bool A_KC, bool B_KC, int WA, int WB, int WC, bool CHAIN = false>
__global__ __launch_bounds__(C::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void strassen_m16_kernel(const LaunchArgs args, const int vec) {
    using In = typename Ops::In;
    using V = typename Ops::Vec;
    constexpr int NV = Ops::NV;
    constexpr int NPLANES = Ops::kX3 ? 2 : 1;  // hi (and lo) tiles
    using SA = Stage<C, Ops, C::MT, A_KC, WA == 1>;
    using SB = Stage<C, Ops, C::NT, B_KC, WB == 1>;
    static_assert(!Ops::kPreA || (A_KC && WA == 1), "pre-split A: single term, stored as is");
    static_assert(!Ops::kPreB || (!B_KC && WB == 1), "pre-split B: single term, stored as is");
    __shared__ __attribute__((aligned(16))) unsigned short As[2][NPLANES][SA::SIZE];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NPLANES][SB::SIZE];

    int tm, tn;
    tile_coords<C::GROUP>(args.tiles_m, args.tiles_n, tm, tn);
    const int row0 = tm * C::MT, col0 = tn * C::NT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % C::WAVES_M, wn = wave / C::WAVES_M;

    f32x16 acc[C::BM][C::BN];
#pragma unroll
    for (int i = 0; i < C::BM; ++i)
#pragma unroll
        for (int j = 0; j < C::BN; ++j) acc[i][j] = f32x16{};

    // One product into acc, then its epilogue (phase 1 of a chain: all
    // outputs but the carried one).
    auto product = [&](const ProductArg &P, const int phase) __attribute__((always_inline)) {
    const In *__restrict__ A = static_cast<const In *>(P.a_base ? P.a_base : args.A);
    const In *__restrict__ B = static_cast<const In *>(P.b_base ? P.b_base : args.B);
    const int64_t lda = P.a_base ? P.lda : args.lda;
    const int64_t ldb = P.b_base ? P.ldb : args.ldb;
    const int nc = CHAIN ? P.nc : WC;  // outputs in use
    const int skip = phase == 1 ? P.carry - 1 : -1;

    // Extents shared by every term: x (m for A, n for B) and k.
    int a_x, a_k, b_k, b_x;
    min_extent(P.a, WA, a_x, a_k);  // A terms: rows = m extent, cols = k extent
    min_extent(P.b, WB, b_k, b_x);  // B terms: rows = k extent, cols = n extent
    const bool a_x_full = row0 + C::MT <= a_x;
    const bool b_x_full = col0 + C::NT <= b_x;

    V raw_a[WA][SA::VECS][SA::LOADS];
    V raw_b[WB][SB::VECS][SB::LOADS];

    // One operand's loads.  terms[t].rows / .cols are the term's x / k
    // extents.  KC (direct units): element (x, k) at off + x*ld + k, vectors
    // along k; XC (paired units): element (x, k) at off + k*ld + x, vectors
    // along x, two consecutive k rows per unit.
    auto load_operand = [&](auto &raw, const In *base, const TermArg *terms, auto stage, auto kc,
                            auto nterms, int64_t ld, int x0, int k0, bool fast, auto pre) __attribute__((always_inline)) {
        using S = decltype(stage);
        constexpr bool KC = decltype(kc)::value;
        constexpr int NT_ = decltype(nterms)::value;
        constexpr bool PRE = decltype(pre)::value;
#pragma unroll
        for (int p = 0; p < S::VECS; ++p) {
            int x, k;
            S::coords(tid, p, x, k);
#pragma unroll
            for (int t = 0; t < NT_; ++t)
#pragma unroll
                for (int l = 0; l < S::LOADS; ++l) {
                    // direct (KC): line x, run k; paired (XC): line k + l, run x
                    const int line = KC ? x0 + x : k0 + k + l;
                    const int run = KC ? k0 + k : x0 + x;
                    const int lines = KC ? terms[t].rows : terms[t].cols;
                    const int runs = KC ? terms[t].cols : terms[t].rows;
                    raw[t][p][l] = load_vec<Ops, PRE>(base + terms[t].off, ld, line, run, lines, runs,
                                                      fast, vec != 0);
                }
        }
    };

    // Issue the global loads of every term of the k-tile starting at k0.  The
    // extents passed for B are (rows, cols) = (k, n); for the paired layout
    // the line is k and the run is n, for direct (B^T stored) line n, run k.
    auto stage_load = [&](int k0) __attribute__((always_inline)) {
        const bool fast = vec && a_x_full && b_x_full && (k0 + C::KT <= a_k) && (k0 + C::KT <= b_k);
        // A terms carry (rows, cols) = (m, k) = (x, k) extents
        load_operand(raw_a, A, P.a, SA{}, std::integral_constant<bool, A_KC>{},
                     std::integral_constant<int, WA>{}, lda, row0, k0, fast,
                     std::integral_constant<bool, Ops::kPreA>{});
        // B terms carry (rows, cols) = (k, n): swap to (x, k) extents
        TermArg bt[WB];
#pragma unroll
        for (int t = 0; t < WB; ++t) {
            bt[t] = P.b[t];
            bt[t].rows = P.b[t].cols;
            bt[t].cols = P.b[t].rows;
        }
        load_operand(raw_b, B, bt, SB{}, std::integral_constant<bool, B_KC>{},
                     std::integral_constant<int, WB>{}, ldb, col0, k0, fast,
                     std::integral_constant<bool, Ops::kPreB>{});
    };

    // In-bounds k-tiles [0, nfast): unguarded loads from a uniform per-term
    // base (advanced one k-tile per step) plus a per-thread 32-bit byte
    // offset that does not change along k.
    // (The compensated mode with four terms on both operands has no
    // registers to spare for the offsets and keeps the guarded loop.)
    constexpr bool kFastLoop = !(Ops::kX3 && WA + WB >= 8);
    // The compensated mode with at most four terms on 256x256 tiles loads
    // two k-tiles ahead (a second set of staging registers): its 16-deep
    // k-tile is ~1500 MFMA cycles per SIMD, shorter than the latency of the
    // next tile's loads.  Measured +4-6 % for (1,1,1), (2,1,2), (2,2,1) and
    // (2,2,2).  For bf16/fp16 operands it is used for (1,2,2) only, on
    // 32-deep k-tiles (the same registers as one 64-deep set): +6-9 %
    // against the 64-deep one-ahead loop in three A/B runs; (2,1,2) and
    // (2,2,2) measured 3-5 % slower with it, (2,2,1) within 1 %, W = 1 1-3 %
    // slower.
    constexpr bool kDeep = kFastLoop && C::MT == 256 &&
                           (Ops::kX3 ? (WA + WB <= 4 && C::KT == 16) : (WA == 1 && WB == 2 && C::KT == 32));
    // In the two-ahead loop the stores of the tile loaded one trip earlier
    // go to the buffer whose last reads ended at the previous barrier, so
    // they are woven between the MFMA rows (A's after the second row, B's
    // after the row past the middle) instead of following them: for the
    // compensated mode +2.6-3.0 % (2,1,2), +0.7-0.8 % (2,2,x) with A and B
    // as stored, +0.7 % / +5.6 % with both transposed, -1 % (1,2,2) and
    // -0.1 to -1.1 % with exactly one operand transposed; bit-identical.
    // Used where W_A >= W_B and either both or neither operand is
    // transposed.
    constexpr bool kWeaveDeep = kDeep && Ops::kX3 && WA >= WB && A_KC != B_KC;
    // Compensated products with A as stored and B summed: a 16-deep fp32
    // k-tile makes A's rows 64 bytes, half a cache line, and the two-ahead
    // loop requested the two halves of each line a trip apart, so the L2
    // served every line of A twice.  Here A's loads of the two k-tiles of
    // one trip pair are issued back to back (both halves of a line requested
    // together) into one register set holding both tiles; B keeps its
    // per-tile sets.  Measured -10 % for (2,2,x) and -3 to -4 % for (1,2,2)
    // at 8192^3 per product, A/B in one process, bit-identical; (2,1,2)
    // measured 1-2 % slower this way and keeps the per-tile loads; the
    // two-level variants were not measured and keep them too.
    constexpr bool kPairA = kDeep && Ops::kX3 && A_KC && !B_KC && WB == 2 && WC <= 2 && C::KT == 16 &&
                            C::BM == 4 && SA::VECS == 2 && SA::LOADS == 1;
    // Buffer loads for single-term operands and the two-ahead loop (measured
    // faster there); otherwise plain global loads measured faster.
    constexpr bool kBufferLoads = WA + WB <= 2 || kDeep;
    constexpr uint64_t kOffLimit = 1ull << 32;
    const bool off32 = (uint64_t)(A_KC ? C::MT : C::KT) * (uint64_t)lda * sizeof(In) < kOffLimit &&
                       (uint64_t)(B_KC ? C::NT : C::KT) * (uint64_t)ldb * sizeof(In) < kOffLimit;
    const int nfast = (kFastLoop && vec && a_x_full && b_x_full && off32)
                          ? (a_k < b_k ? a_k : b_k) / C::KT : 0;
    uint32_t a_off[SA::VECS][SA::LOADS], b_off[SB::VECS][SB::LOADS];
    auto unit_offsets = [&](auto &off, auto stage, auto kc, int64_t ld) __attribute__((always_inline)) {
        using S = decltype(stage);
        constexpr bool KC = decltype(kc)::value;
#pragma unroll
        for (int p = 0; p < S::VECS; ++p) {
            int x, k;
            S::coords(tid, p, x, k);
#pragma unroll
            for (int l = 0; l < S::LOADS; ++l)
                off[p][l] = (uint32_t)sizeof(In) *
                            (KC ? (uint32_t)x * (uint32_t)ld + k : (uint32_t)(k + l) * (uint32_t)ld + x);
        }
    };
    if constexpr (kFastLoop) {
        unit_offsets(a_off, SA{}, std::integral_constant<bool, A_KC>{}, lda);
        unit_offsets(b_off, SB{}, std::integral_constant<bool, B_KC>{}, ldb);
    }
    const int64_t a_org = A_KC ? (int64_t)row0 * lda : row0;
    const int64_t b_org = B_KC ? (int64_t)col0 * ldb : col0;
    const int64_t a_step = (int64_t)sizeof(In) * (A_KC ? (int64_t)C::KT : (int64_t)C::KT * lda);
    const int64_t b_step = (int64_t)sizeof(In) * (B_KC ? (int64_t)C::KT : (int64_t)C::KT * ldb);

    // Loads number (t * VECS + p) * LOADS + l of one operand, those in
    // [lo, hi) only (the steady loop spreads one k-tile's loads over the
    // MFMA steps of the previous one).
    auto load_fast = [&](auto &raw, const In *base, const TermArg *terms, auto stage, auto nterms,
                         const auto &off, int64_t org, int64_t step, int kt, int lo = 0,
                         int hi = 1 << 20) __attribute__((always_inline)) {
        using S = decltype(stage);
        constexpr int NT_ = decltype(nterms)::value;
#pragma unroll
        for (int t = 0; t < NT_; ++t) {
            const char *tb = reinterpret_cast<const char *>(base + terms[t].off + org) + step * kt;
            if constexpr (kBufferLoads) {
                const auto r = raw_rsrc(tb);
#pragma unroll
                for (int p = 0; p < S::VECS; ++p)
#pragma unroll
                    for (int l = 0; l < S::LOADS; ++l) {
                        const int idx = (t * S::VECS + p) * S::LOADS + l;
                        if (idx >= lo && idx < hi) raw[t][p][l] = buffer_load16<V>(r, off[p][l]);
                    }
            } else {
#pragma unroll
                for (int p = 0; p < S::VECS; ++p)
#pragma unroll
                    for (int l = 0; l < S::LOADS; ++l) {
                        const int idx = (t * S::VECS + p) * S::LOADS + l;
                        if (idx >= lo && idx < hi) raw[t][p][l] = *reinterpret_cast<const V *>(tb + off[p][l]);
                    }
            }
        }
    };
    constexpr int NLA = WA * SA::VECS * SA::LOADS, NLB = WB * SB::VECS * SB::LOADS;
    // Loads [lo, hi) of the k-tile's flat list (A's, then B's) into ra / rb.
    auto load_fast_range_into = [&](int kt, auto &ra, auto &rb, int lo, int hi) __attribute__((always_inline)) {
        if constexpr (kFastLoop) {
            if (lo < NLA)
                load_fast(ra, A, P.a, SA{}, std::integral_constant<int, WA>{}, a_off, a_org, a_step, kt,
                          lo, hi);
            if (hi > NLA)
                load_fast(rb, B, P.b, SB{}, std::integral_constant<int, WB>{}, b_off, b_org, b_step, kt,
                          lo - NLA, hi - NLA);
        }
    };
    auto load_fast_range = [&](int kt, int lo, int hi) __attribute__((always_inline)) {
        load_fast_range_into(kt, raw_a, raw_b, lo, hi);
    };
    auto stage_load_fast_into = [&](int kt, auto &ra, auto &rb) __attribute__((always_inline)) {
        if constexpr (kFastLoop) {
            load_fast(ra, A, P.a, SA{}, std::integral_constant<int, WA>{}, a_off, a_org, a_step, kt);
            load_fast(rb, B, P.b, SB{}, std::integral_constant<int, WB>{}, b_off, b_org, b_step, kt);
        }
    };
    auto stage_load_fast = [&](int kt) __attribute__((always_inline)) { stage_load_fast_into(kt, raw_a, raw_b); };

    // Sign of the first term of each operand: factored out of the operand
    // sum and applied in the epilogue instead (signs are +-1 and rounding to
    // nearest even is symmetric, so the staged values are the same up to
    // that exact negation).  The staged sum is x_0 + sum_t (s_t s_0) x_t.
    const float sa0 = P.a[0].sign, sb0 = P.b[0].sign;

    // Relative-signed sum of element e of load l of unit p over the terms,
    // in fp32.
    auto sum_elem = [&](auto &raw, const TermArg *terms, float s0, auto nterms, int p, int l, int e) __attribute__((always_inline)) {
        constexpr int NT_ = decltype(nterms)::value;
        float s = Ops::to_f32(raw[0][p][l][e]);
#pragma unroll
        for (int t = 1; t < NT_; ++t) s += (terms[t].sign * s0) * Ops::to_f32(raw[t][p][l][e]);
        return s;
    };

    // One stored operand value needs no arithmetic: its bits go to LDS as
    // they are (the 16-bit operand types only; the compensated mode splits).
    constexpr bool kCopyA = WA == 1 && !Ops::kX3;
    constexpr bool kCopyB = WB == 1 && !Ops::kX3;

    // Paired layout from raw rows k and k+1 of NV consecutive x: the word of
    // x + 2j (x + 2j + 1) holds the low (high) halves of word j of both rows.
    auto pair_words = [&](const V &row0, const V &row1, int e) __attribute__((always_inline)) -> unsigned {
        const u32x4 r0 = __builtin_bit_cast(u32x4, row0), r1 = __builtin_bit_cast(u32x4, row1);
        return __builtin_amdgcn_perm(r1[e >> 1], r0[e >> 1], (e & 1) ? 0x07060302u : 0x05040100u);
    };

    // Signed sums of the raw terms ra / rb rounded to the MFMA type (split
    // into hi/lo for the compensated mode), stored into LDS buffer `buf`.
    // part: 0 both operands, 1 A only, 2 B only.
    auto stage_store_from = [&](int buf, auto &ra, auto &rb, int part = 0) __attribute__((always_inline)) {
        // ---- A ----
        if (part != 2)
#pragma unroll
        for (int p = 0; p < SA::VECS; ++p) {
            int x, k;
            SA::coords(tid, p, x, k);
            if constexpr (A_KC && kCopyA) {
                *reinterpret_cast<V *>(&As[buf][0][x * SA::LDX + k]) = ra[0][p][0];
            } else if constexpr (A_KC && Ops::kPreA) {
                // pre-split: the unit's halves are the hi and lo rows of NV k
                const u32x4 w = __builtin_bit_cast(u32x4, ra[0][p][0]);
                *reinterpret_cast<u32x2 *>(&As[buf][0][x * SA::LDX + k]) = u32x2{w[0], w[1]};
                *reinterpret_cast<u32x2 *>(&As[buf][1][x * SA::LDX + k]) = u32x2{w[2], w[3]};
            } else if constexpr (A_KC) {
                // direct: NV consecutive k of row x
                unsigned short hi[NV], lo[NV];
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const float s = sum_elem(ra, P.a, sa0, std::integral_constant<int, WA>{}, p, 0, e);
                    hi[e] = Ops::from_f32(s);
                    if constexpr (Ops::kX3) lo[e] = Ops::from_f32(s - Ops::bf16_to_f32(hi[e]));
                }
                const int off = x * SA::LDX + k;
#pragma unroll
                for (int q = 0; q < NPLANES; ++q) {
                    const unsigned short *src = q == 0 ? hi : lo;
                    if constexpr (NV == 8) {
                        u16x8 w;
#pragma unroll
                        for (int e = 0; e < 8; ++e) w[e] = src[e];
                        *reinterpret_cast<u16x8 *>(&As[buf][q][off]) = w;
                    } else {
                        u16x4 w;
#pragma unroll
                        for (int e = 0; e < 4; ++e) w[e] = src[e];
                        *reinterpret_cast<u16x4 *>(&As[buf][q][off]) = w;
                    }
                }
            } else if constexpr (kCopyA) {
                const int base = SA::at(x, k);
#pragma unroll
                for (int e = 0; e < NV; ++e)
                    *reinterpret_cast<unsigned *>(&As[buf][0][base + e * SA::LDX]) =
                        pair_words(ra[0][p][0], ra[0][p][1], e);
            } else {
                // paired: k rows k, k+1 of NV consecutive x
                const int base = SA::at(x, k);
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const float s0 = sum_elem(ra, P.a, sa0, std::integral_constant<int, WA>{}, p, 0, e);
                    const float s1 = sum_elem(ra, P.a, sa0, std::integral_constant<int, WA>{}, p, 1, e);
                    const unsigned hw = Ops::pack2(s0, s1);
                    const int off = base + e * SA::LDX;
                    *reinterpret_cast<unsigned *>(&As[buf][0][off]) = hw;
                    if constexpr (Ops::kX3) {
                        const float r0 = s0 - __uint_as_float(hw << 16);
                        const float r1 = s1 - __uint_as_float(hw & 0xffff0000u);
                        *reinterpret_cast<unsigned *>(&As[buf][NPLANES - 1][off]) = Ops::pack2(r0, r1);
                    }
                }
            }
        }
        // ---- B ----
        if (part != 1)
#pragma unroll
        for (int p = 0; p < SB::VECS; ++p) {
            int x, k;
            SB::coords(tid, p, x, k);
            if constexpr (B_KC && kCopyB) {
                *reinterpret_cast<V *>(&Bs[buf][0][x * SB::LDX + k]) = rb[0][p][0];
            } else if constexpr (B_KC) {
                unsigned short hi[NV], lo[NV];
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const float s = sum_elem(rb, P.b, sb0, std::integral_constant<int, WB>{}, p, 0, e);
                    hi[e] = Ops::from_f32(s);
                    if constexpr (Ops::kX3) lo[e] = Ops::from_f32(s - Ops::bf16_to_f32(hi[e]));
                }
                const int off = x * SB::LDX + k;
#pragma unroll
                for (int q = 0; q < NPLANES; ++q) {
                    const unsigned short *src = q == 0 ? hi : lo;
                    if constexpr (NV == 8) {
                        u16x8 w;
#pragma unroll
                        for (int e = 0; e < 8; ++e) w[e] = src[e];
                        *reinterpret_cast<u16x8 *>(&Bs[buf][q][off]) = w;
                    } else {
                        u16x4 w;
#pragma unroll
                        for (int e = 0; e < 4; ++e) w[e] = src[e];
                        *reinterpret_cast<u16x4 *>(&Bs[buf][q][off]) = w;
                    }
                }
            } else if constexpr (kCopyB) {
                const int base = SB::at(x, k);
#pragma unroll
                for (int e = 0; e < NV; ++e)
                    *reinterpret_cast<unsigned *>(&Bs[buf][0][base + e * SB::LDX]) =
                        pair_words(rb[0][p][0], rb[0][p][1], e);
            } else if constexpr (Ops::kPreB) {
                // pre-split rows k and k+1 of NV consecutive x: the word of
                // x + e in each plane pairs element e's halves of both rows
                const int base = SB::at(x, k);
                const u32x4 r0 = __builtin_bit_cast(u32x4, rb[0][p][0]);
                const u32x4 r1 = __builtin_bit_cast(u32x4, rb[0][p][1]);
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const unsigned sel = (e & 1) ? 0x07060302u : 0x05040100u;
                    const int off = base + e * SB::LDX;
                    *reinterpret_cast<unsigned *>(&Bs[buf][0][off]) =
                        __builtin_amdgcn_perm(r1[e >> 1], r0[e >> 1], sel);
                    *reinterpret_cast<unsigned *>(&Bs[buf][1][off]) =
                        __builtin_amdgcn_perm(r1[2 + (e >> 1)], r0[2 + (e >> 1)], sel);
                }
            } else {
                const int base = SB::at(x, k);
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const float s0 = sum_elem(rb, P.b, sb0, std::integral_constant<int, WB>{}, p, 0, e);
                    const float s1 = sum_elem(rb, P.b, sb0, std::integral_constant<int, WB>{}, p, 1, e);
                    const unsigned hw = Ops::pack2(s0, s1);
                    const int off = base + e * SB::LDX;
                    *reinterpret_cast<unsigned *>(&Bs[buf][0][off]) = hw;
                    if constexpr (Ops::kX3) {
                        const float r0 = s0 - __uint_as_float(hw << 16);
                        const float r1 = s1 - __uint_as_float(hw & 0xffff0000u);
                        *reinterpret_cast<unsigned *>(&Bs[buf][NPLANES - 1][off]) = Ops::pack2(r0, r1);
                    }
                }
            }
        }
    };

    auto stage_store = [&](int buf) __attribute__((always_inline)) { stage_store_from(buf, raw_a, raw_b); };

    // In MFMA step s of a k-tile, lanes 0-31 supply k = 16s + 0..7 and lanes
    // 32-63 supply k = 16s + 8..15, for A and B alike.
    const int h = lane >> 5, l32 = lane & 31;
    auto mfma = [&](const u32x4 &a, const u32x4 &b, f32x16 c) __attribute__((always_inline)) -> f32x16 {
        if constexpr (std::is_same<Ops, F16Ops>::value)
            return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                          __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                           __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    };
    // Eight consecutive k of tile row x: one 16-byte read (direct stride is a
    // multiple of 16 bytes) or two 8-byte reads (paired stride is a multiple
    // of 8 bytes).
    auto frag = [&](const unsigned short *tile, auto stage, int x, int k) __attribute__((always_inline)) -> u32x4 {
        using S = decltype(stage);
        if constexpr (S::LOADS == 1) return *reinterpret_cast<const u32x4 *>(tile + x * S::LDX + k);
        const u32x2 lo2 = *reinterpret_cast<const u32x2 *>(tile + S::at(x, k));
        const u32x2 hi2 = *reinterpret_cast<const u32x2 *>(tile + S::at(x, k + 4));
        return u32x4{lo2.x, lo2.y, hi2.x, hi2.y};
    };
    // MFMA step s (16 consecutive k) of the k-tile in LDS buffer `buf`.
    auto compute_step = [&](int buf, int s) __attribute__((always_inline)) {
        {
            u32x4 af[NPLANES][C::BM], bf[NPLANES][C::BN];
#pragma unroll
            for (int q = 0; q < NPLANES; ++q) {
#pragma unroll
                for (int i = 0; i < C::BM; ++i)
                    af[q][i] = frag(&As[buf][q][0], SA{}, wm * C::WM + i * 32 + l32, 16 * s + 8 * h);
#pragma unroll
                for (int j = 0; j < C::BN; ++j)
                    bf[q][j] = frag(&Bs[buf][q][0], SB{}, wn * C::WN + j * 32 + l32, 16 * s + 8 * h);
            }
#pragma unroll
            for (int i = 0; i < C::BM; ++i)
#pragma unroll
                for (int j = 0; j < C::BN; ++j) {
                    acc[i][j] = mfma(af[0][i], bf[0][j], acc[i][j]);
                    if constexpr (Ops::kX3) {
                        acc[i][j] = mfma(af[0][i], bf[NPLANES - 1][j], acc[i][j]);
                        acc[i][j] = mfma(af[NPLANES - 1][i], bf[0][j], acc[i][j]);
                    }
                }
        }
    };
    auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < C::KT / 16; ++s) compute_step(buf, s);
    };
    // The same MFMA block with the loads of k-tile `lkt` into ra / rb issued
    // in groups between its rows of MFMAs (fragments are read first); with
    // sa / sb given, the staged sums of sa / sb are stored into LDS buffer
    // `sbuf` between the rows too (A's after the second row, B's after the
    // row past the middle).
    auto compute_loading = [&](int buf, int lkt, auto &ra, auto &rb, int sbuf = -1,
                               V (*sa)[SA::VECS][SA::LOADS] = nullptr,
                               V (*sb)[SB::VECS][SB::LOADS] = nullptr) __attribute__((always_inline)) {
        constexpr int NG = (C::KT / 16) * C::BM, NL = NLA + NLB;
#pragma unroll
        for (int s = 0; s < C::KT / 16; ++s) {
            u32x4 af[NPLANES][C::BM], bf[NPLANES][C::BN];
#pragma unroll
            for (int q = 0; q < NPLANES; ++q) {
#pragma unroll
                for (int i = 0; i < C::BM; ++i)
                    af[q][i] = frag(&As[buf][q][0], SA{}, wm * C::WM + i * 32 + l32, 16 * s + 8 * h);
#pragma unroll
                for (int j = 0; j < C::BN; ++j)
                    bf[q][j] = frag(&Bs[buf][q][0], SB{}, wn * C::WN + j * 32 + l32, 16 * s + 8 * h);
            }
#pragma unroll
            for (int i = 0; i < C::BM; ++i) {
                const int g = s * C::BM + i;
                load_fast_range_into(lkt, ra, rb, g * NL / NG, (g + 1) * NL / NG);
                if (sa != nullptr && g == 1) stage_store_from(sbuf, sa, sb, 1);
                if (sa != nullptr && g == NG / 2 + 1) stage_store_from(sbuf, sa, sb, 2);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int j = 0; j < C::BN; ++j) {
                    acc[i][j] = mfma(af[0][i], bf[0][j], acc[i][j]);
                    if constexpr (Ops::kX3) {
                        acc[i][j] = mfma(af[0][i], bf[NPLANES - 1][j], acc[i][j]);
                        acc[i][j] = mfma(af[NPLANES - 1][i], bf[0][j], acc[i][j]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    const int nk = (args.sk + C::KT - 1) / C::KT;
    int kt = 0;

    // Single-term products with A and B as stored on 256x256 tiles -- 16-bit
    // operands on 64-deep k-tiles, and pre-split compensated operands (both
    // pre-split) on 32-deep ones: the in-bounds k-tiles [0, nfast) are loaded
    // straight into LDS by the load unit (16-byte global_load_lds, no staging
    // registers, no LDS stores), two tiles in flight in the two LDS buffers,
    // one barrier per tile.  Both tiles are kept as stored and unpadded: A
    // [m][k] (128-byte rows) and B [k][n] (512-byte rows of 16-bit data,
    // 1024-byte rows of pre-split units), their 16-byte units XOR-swizzled by
    // row ((row / 2) mod 8 for A, 4 (k mod 4) for B) so that a fragment read
    // cycle hits distinct banks; each lane's load address picks the unit that
    // lands at its LDS slot.  B's fragments (8 consecutive k of one column)
    // come from two 16-bit transpose reads (ds_read_b64_tr_b16: within each
    // 16 lanes, lane s reads 4 consecutive n of k row s/4, and lane L
    // receives column L of those four rows), per plane for pre-split data
    // (the hi and lo halves of each unit).  Same MFMAs on the same values in
    // the same order as the staged loop, so results are bit-identical; the
    // remaining k-tiles (a ragged end) take the staged loop.  The loads are
    // issued in inline assembly so that the compiler does not hold every LDS
    // read behind them; the loop's own vmcnt wait and barrier order them.
    constexpr bool kDirect16 = !Ops::kX3 && WA == 1 && WB == 1 && A_KC && !B_KC && C::MT == 256 &&
                               C::NT == 256 && C::KT == 64 && C::WAVES_M == 2 && C::WAVES_N == 4;
    constexpr bool kDirectPre = Ops::kPreA && Ops::kPreB && WA == 1 && WB == 1 && A_KC && !B_KC &&
                                C::MT == 256 && C::NT == 256 && C::KT == 32 && C::WAVES_M == 2 &&
                                C::WAVES_N == 4;
    constexpr bool kDirect = kDirect16 || kDirectPre;
    if constexpr (kDirect) {
        constexpr int EPU = 16 / (int)sizeof(In);  // elements per 16-byte unit
        constexpr int BRB = 256 * (int)sizeof(In);  // bytes per B k row
        constexpr int BRI = 1024 / BRB;             // B k rows per 1 KB load instruction
        constexpr int BUR = BRB / 16;               // units per B k row
        constexpr int NST = C::KT / 16;             // MFMA steps per k-tile
        static_assert(C::KT * (int)sizeof(In) == 128, "128-byte A rows");
        static_assert((int)sizeof(As[0]) >= 256 * 128 && (int)sizeof(Bs[0]) >= C::KT * BRB,
                      "direct tiles fit the buffers");
        if (nfast >= 1) {
            const int wv = __builtin_amdgcn_readfirstlane(wave);
            const int g16 = lane >> 4, s16 = lane & 15;
            const char *Ab = reinterpret_cast<const char *>(A + P.a[0].off + a_org);
            const char *Bb = reinterpret_cast<const char *>(B + P.b[0].off + b_org);
            // load slots: instruction i of wave wv fills 1 KB of each tile,
            // A rows 8 (4 wv + i) .. + 7, B k rows BRI (4 wv + i) ..; each
            // lane's byte offset from the tile's base (below 2^32: nfast
            // requires it)
            uint32_t a_ld[4], b_ld[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 8 * (4 * wv + i) + lane / 8;
                a_ld[i] = (uint32_t)sizeof(In) * ((uint32_t)r * (uint32_t)lda + EPU * ((lane % 8) ^ ((r >> 1) & 7)));
                const int kr = BRI * (4 * wv + i) + lane / BUR;
                b_ld[i] = (uint32_t)sizeof(In) * ((uint32_t)kr * (uint32_t)ldb + EPU * ((lane % BUR) ^ (4 * (kr & 3))));
            }
            const uint32_t lds_a[2] = {(uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned short *)&As[0][0][0],
                                       (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned short *)&As[1][0][0]};
            const uint32_t lds_b[2] = {(uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned short *)&Bs[0][0][0],
                                       (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned short *)&Bs[1][0][0]};
            // 16 bytes per lane from base + off into LDS at lds + 16 lane
            auto dma = [&](const char *base, uint32_t off, uint32_t lds) __attribute__((always_inline)) {
                asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
                             :: "s"(lds), "v"(off), "s"(base) : "memory", "m0");
            };
            auto issue = [&](int t) __attribute__((always_inline)) {
                const int b = t & 1;
                const char *at = Ab + (int64_t)t * C::KT * (int64_t)sizeof(In);
                const char *bt = Bb + (int64_t)t * C::KT * ldb * (int64_t)sizeof(In);
#pragma unroll
                for (int i = 0; i < 4; ++i) dma(at, a_ld[i], lds_a[b] + (4 * wv + i) * 1024);
#pragma unroll
                for (int i = 0; i < 4; ++i) dma(bt, b_ld[i], lds_b[b] + (4 * wv + i) * 1024);
            };
            // fragment byte offsets within a tile.  A: row ra + 32 i, 16-byte
            // unit (2 st + h) of 16-bit data or (4 st + 2 h + u) of pre-split
            // data; rows 32 apart share the swizzle, so i adds 4096 bytes.
            // B: k row kr0 + 16 st + 4 q (kr mod 4 = s16 / 4 for every st, q),
            // column block nc of fragment j.
            constexpr int AU = kDirectPre ? 2 : 1;
            const int ra = wm * C::WM + l32;
            int a_rd[NST][AU], b_rd[C::BN];
#pragma unroll
            for (int st = 0; st < NST; ++st)
#pragma unroll
                for (int u = 0; u < AU; ++u) {
                    const int unit = kDirectPre ? 4 * st + 2 * h + u : 2 * st + h;
                    a_rd[st][u] = ra * 128 + 16 * (unit ^ ((ra >> 1) & 7));
                }
            const int kr0 = 8 * h + s16 / 4;
#pragma unroll
            for (int j = 0; j < C::BN; ++j) {
                const int nc = wn * C::WN + j * 32 + 16 * (g16 & 1) + 4 * (s16 % 4);
                b_rd[j] = kr0 * BRB + 16 * ((nc / EPU) ^ (4 * (s16 / 4))) + 2 * (nc % EPU);
            }
            typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
            auto tr = [&](const unsigned char *p) __attribute__((always_inline)) -> u32x2 {
                return __builtin_bit_cast(
                    u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                               (lds_i16x4 *)(__attribute__((address_space(3))) const unsigned char *)p));
            };
            // fragments of MFMA step st of the tile in LDS buffer b
            auto read_frags = [&](int b, int st, u32x4 (&af)[NPLANES][C::BM], u32x4 (&bf)[NPLANES][C::BN])
                __attribute__((always_inline)) {
                const unsigned char *ta = reinterpret_cast<const unsigned char *>(&As[b][0][0]);
                const unsigned char *tb = reinterpret_cast<const unsigned char *>(&Bs[b][0][0]);
#pragma unroll
                for (int i = 0; i < C::BM; ++i) {
                    if constexpr (kDirectPre) {
                        const u32x4 u0 = *reinterpret_cast<const u32x4 *>(ta + a_rd[st][0] + 4096 * i);
                        const u32x4 u1 = *reinterpret_cast<const u32x4 *>(ta + a_rd[st][1] + 4096 * i);
                        af[0][i] = u32x4{u0[0], u0[1], u1[0], u1[1]};
                        af[NPLANES - 1][i] = u32x4{u0[2], u0[3], u1[2], u1[3]};
                    } else {
                        af[0][i] = *reinterpret_cast<const u32x4 *>(ta + a_rd[st][0] + 4096 * i);
                    }
                }
#pragma unroll
                for (int j = 0; j < C::BN; ++j)
#pragma unroll
                    for (int q = 0; q < NPLANES; ++q) {  // plane q: the unit's half at byte 8 q
                        const unsigned char *pb = tb + b_rd[j] + 16 * st * BRB + 8 * q;
                        const u32x2 l2 = tr(pb), h2 = tr(pb + 4 * BRB);
                        bf[q][j] = u32x4{l2.x, l2.y, h2.x, h2.y};
                    }
            };
            // every wave's loads into LDS have landed and every wave is past
            // the reads of the buffer the next loads overwrite
            auto tile_barrier = [&]() __attribute__((always_inline)) {
                wait_vmcnt<0>();
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("s_barrier" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            };
            issue(0);
            if constexpr (kDirect16) {
                // 16-bit data: the fragments of step st + 1 are read while
                // step st's MFMAs run, one read per MFMA (+1-3 % bf16 plain),
                // and the tile boundary sits inside the last step: its
                // fragments are already in registers, so after its first row
                // of MFMAs the wave waits for its own LDS reads and loads,
                // meets the others at the barrier, issues the loads of tile
                // t + 2 into the buffer just read, and reads step 0 of tile
                // t + 1 while the rest of the step's MFMAs run.  The barrier,
                // the load issue and the first reads' latency no longer leave
                // the matrix cores idle between tiles (+2.7-3.8 % bf16 and
                // fp16 plain; both measured A/B in alternating processes).
                constexpr int kReads = C::BM + 2 * C::BN;
                constexpr int kMfmas = C::BM * C::BN;
                constexpr int kLast = (NST - 1) & 1;
                static_assert(NST % 2 == 0 && C::BM >= 2, "step 0 of a tile reads into fragment set 0");
                u32x4 fa[2][NPLANES][C::BM], fb[2][NPLANES][C::BN];
                tile_barrier();
                if (1 < nfast) issue(1);
                read_frags(0, 0, fa[0], fb[0]);
                auto tile = [&](int t, auto more) __attribute__((always_inline)) {
                    const int b = t & 1;
#pragma unroll
                    for (int st = 0; st + 1 < NST; ++st) {
                        read_frags(b, st + 1, fa[(st + 1) & 1], fb[(st + 1) & 1]);
#pragma unroll
                        for (int i = 0; i < C::BM; ++i)
#pragma unroll
                            for (int j = 0; j < C::BN; ++j)
                                acc[i][j] = mfma(fa[st & 1][0][i], fb[st & 1][0][j], acc[i][j]);
#pragma unroll
                        for (int g = 0; g < kReads; ++g) {
                            __builtin_amdgcn_sched_group_barrier(0x008, kMfmas / kReads > 0 ? kMfmas / kReads : 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (decltype(more)::value) {
#pragma unroll
                        for (int j = 0; j < C::BN; ++j)
                            acc[0][j] = mfma(fa[kLast][0][0], fb[kLast][0][j], acc[0][j]);
                        __builtin_amdgcn_sched_barrier(0);
                        // tile t + 1 has landed and this wave's reads of
                        // tile t have returned
                        wait_vmcnt_lgkmcnt0();
                        __builtin_amdgcn_sched_barrier(0);
                        asm volatile("s_barrier" ::: "memory");
                        __builtin_amdgcn_sched_barrier(0);
                        if (t + 2 < nfast) issue(t + 2);
                        read_frags(b ^ 1, 0, fa[0], fb[0]);
#pragma unroll
                        for (int i = 1; i < C::BM; ++i)
#pragma unroll
                            for (int j = 0; j < C::BN; ++j)
                                acc[i][j] = mfma(fa[kLast][0][i], fb[kLast][0][j], acc[i][j]);
                        constexpr int kRest = kMfmas - C::BN;
                        __builtin_amdgcn_sched_group_barrier(0x100, kReads > kRest ? kReads - kRest : 0, 0);
#pragma unroll
                        for (int g = 0; g < (kReads < kRest ? kReads : kRest); ++g) {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    } else {
#pragma unroll
                        for (int i = 0; i < C::BM; ++i)
#pragma unroll
                            for (int j = 0; j < C::BN; ++j)
                                acc[i][j] = mfma(fa[kLast][0][i], fb[kLast][0][j], acc[i][j]);
                    }
                };
                int t = 0;
                for (; t + 1 < nfast; ++t) tile(t, std::true_type{});
                tile(t, std::false_type{});
            } else {
                // pre-split data: each step's fragments are read before its
                // MFMAs (reading the next step's during them, with fragment
                // pairs taking twice the reads and registers, measured 3-8 %
                // slower)
                for (int t = 0; t < nfast; ++t) {
                    tile_barrier();
                    if (t + 1 < nfast) issue(t + 1);
#pragma unroll
                    for (int st = 0; st < NST; ++st) {
                        u32x4 af[NPLANES][C::BM], bf[NPLANES][C::BN];
                        read_frags(t & 1, st, af, bf);
#pragma unroll
                        for (int i = 0; i < C::BM; ++i)
#pragma unroll
                            for (int j = 0; j < C::BN; ++j) {
                                acc[i][j] = mfma(af[0][i], bf[0][j], acc[i][j]);
                                acc[i][j] = mfma(af[0][i], bf[NPLANES - 1][j], acc[i][j]);
                                acc[i][j] = mfma(af[NPLANES - 1][i], bf[0][j], acc[i][j]);
                            }
                    }
                }
            }
            kt = nfast;
            if (kt < nk) {
                // the ragged end: staged loop, tile kt in buffer kt & 1
                __syncthreads();
                stage_load(kt * C::KT);
                stage_store(kt & 1);
                __syncthreads();
            }
        }
    }
    bool a_pairs_done = false;
    if constexpr (kPairA) {
        if (nfast >= 3) {
            // Two-ahead loop with A's k-tiles loaded in pairs.  pa[t][2u + w]
            // holds unit u of term t of tile kt0 + w (kt0 even); B's sets
            // alternate, bq holding odd tiles and raw_b even ones.  At the
            // top of a trip tile kt is in LDS buffer 0, tile kt + 1 in pa
            // (w = 1) and bq.
            a_pairs_done = true;
            uint32_t pa_off[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                int x, k;
                SA::coords(tid, p >> 1, x, k);
                pa_off[p] = (uint32_t)sizeof(In) * ((uint32_t)x * (uint32_t)lda + (uint32_t)(k + C::KT * (p & 1)));
            }
            V pa[WA][4];
            V bq[WB][SB::VECS][SB::LOADS];
            constexpr int NPA = 4 * WA;
            // loads [lo, hi) of A's pair of k-tiles kt0, kt0 + 1
            auto load_pair = [&](int kt0, int lo, int hi) __attribute__((always_inline)) {
#pragma unroll
                for (int t = 0; t < WA; ++t) {
                    const char *tb = reinterpret_cast<const char *>(A + P.a[t].off + a_org) + a_step * kt0;
                    const auto r = raw_rsrc(tb);
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const int idx = t * 4 + p;
                        if (idx >= lo && idx < hi) pa[t][p] = buffer_load16<V>(r, pa_off[p]);
                    }
                }
            };
            auto load_b = [&](auto &rb, int ktb, int lo, int hi) __attribute__((always_inline)) {
                load_fast(rb, B, P.b, SB{}, std::integral_constant<int, WB>{}, b_off, b_org, b_step, ktb,
                          lo, hi);
            };
            // A's signed sum of tile kt0 + w, split hi/lo, into LDS buffer buf
            auto store_a = [&](int buf, int w) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    int x, k;
                    SA::coords(tid, u, x, k);
                    u16x4 wh, wl;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float s = pa[0][2 * u + w][e];
#pragma unroll
                        for (int t = 1; t < WA; ++t) s += (P.a[t].sign * sa0) * pa[t][2 * u + w][e];
                        wh[e] = Ops::from_f32(s);
                        wl[e] = Ops::from_f32(s - Ops::bf16_to_f32(wh[e]));
                    }
                    const int off = x * SA::LDX + k;
                    *reinterpret_cast<u16x4 *>(&As[buf][0][off]) = wh;
                    *reinterpret_cast<u16x4 *>(&As[buf][1][off]) = wl;
                }
            };
            // The MFMA rows of the k-tile in buffer buf, hook(g) before row g.
            auto rows_hooked = [&](int buf, auto hook) __attribute__((always_inline)) {
                u32x4 af[NPLANES][C::BM], bf[NPLANES][C::BN];
#pragma unroll
                for (int q = 0; q < NPLANES; ++q) {
#pragma unroll
                    for (int i = 0; i < C::BM; ++i)
                        af[q][i] = frag(&As[buf][q][0], SA{}, wm * C::WM + i * 32 + l32, 8 * h);
#pragma unroll
                    for (int j = 0; j < C::BN; ++j)
                        bf[q][j] = frag(&Bs[buf][q][0], SB{}, wn * C::WN + j * 32 + l32, 8 * h);
                }
#pragma unroll
                for (int i = 0; i < C::BM; ++i) {
                    hook(i);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int j = 0; j < C::BN; ++j) {
                        acc[i][j] = mfma(af[0][i], bf[0][j], acc[i][j]);
                        acc[i][j] = mfma(af[0][i], bf[NPLANES - 1][j], acc[i][j]);
                        acc[i][j] = mfma(af[NPLANES - 1][i], bf[0][j], acc[i][j]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            load_pair(0, 0, NPA);
            load_b(raw_b, 0, 0, NLB);
            store_a(0, 0);
            stage_store_from(0, raw_a, raw_b, 2);
            load_b(bq, 1, 0, NLB);
            __syncthreads();
            for (; kt + 3 < nfast; kt += 2) {
                // tile kt: store tile kt + 1 into buffer 1, load A's tiles
                // kt + 2 and kt + 3 and B's tile kt + 2
                rows_hooked(0, [&](int g) __attribute__((always_inline)) {
                    if (g == 0) load_b(raw_b, kt + 2, 0, NLB / 2);
                    if (g == 1) {
                        store_a(1, 1);
                        load_pair(kt + 2, 0, NPA / 2);
                    }
                    if (g == 2) {
                        load_pair(kt + 2, NPA / 2, NPA);
                        load_b(raw_b, kt + 2, NLB / 2, NLB);
                    }
                    if (g == 3) stage_store_from(1, raw_a, bq, 2);
                });
                __syncthreads();
                // tile kt + 1: store tile kt + 2 into buffer 0, load B's tile kt + 3
                rows_hooked(1, [&](int g) __attribute__((always_inline)) {
                    if (g == 0) load_b(bq, kt + 3, 0, NLB / 2);
                    if (g == 1) store_a(0, 0);
                    if (g == 2) load_b(bq, kt + 3, NLB / 2, NLB);
                    if (g == 3) stage_store_from(0, raw_a, raw_b, 2);
                });
                __syncthreads();
            }
            compute(0);
            store_a(1, 1);
            stage_store_from(1, raw_a, bq, 2);
            __syncthreads();
            kt += 1;
        }
    }
    if (a_pairs_done) {
        // the one-ahead loop below goes on from tile kt in buffer 1
    } else if (kDeep && nfast >= 3) {
        // Two k-tiles per trip, the register sets alternating: tile kt is in
        // LDS buffer 0 and tile kt + 1 in raw_a/raw_b at the top of a trip.
        // The loop ends with tile kt in buffer 1; the loops below go on.
        V q_a[WA][SA::VECS][SA::LOADS];
        V q_b[WB][SB::VECS][SB::LOADS];
        stage_load_fast(0);
        stage_store(0);
        stage_load_fast(1);
        __syncthreads();
        for (; kt + 3 < nfast; kt += 2) {
            if constexpr (kWeaveDeep) {
                compute_loading(0, kt + 2, q_a, q_b, 1, raw_a, raw_b);
                __syncthreads();
                compute_loading(1, kt + 3, raw_a, raw_b, 0, q_a, q_b);
                __syncthreads();
            } else {
                compute_loading(0, kt + 2, q_a, q_b);
                stage_store_from(1, raw_a, raw_b);
                __syncthreads();
                compute_loading(1, kt + 3, raw_a, raw_b);
                stage_store_from(0, q_a, q_b);
                __syncthreads();
            }
        }
        compute(0);
        stage_store_from(1, raw_a, raw_b);
        __syncthreads();
        kt += 1;
    } else if (!(kDirect && nfast >= 1)) {
        if (nfast > 0)
            stage_load_fast(0);
        else
            stage_load(0);
        stage_store(0);
        __syncthreads();
    }
    // Steady state: the next k-tile is in bounds.  Its loads are spread
    // evenly over the MFMA steps of the current one (issued all at once,
    // they filled the texture-address queue and stalled the waves' MFMA
    // issue: +4-11 % measured), and its sums follow the whole MFMA block;
    // the scheduling barriers hold that order.
    // Single-term 16-bit products on 64-deep k-tiles: A's loads are issued
    // in the first steps, so its LDS stores are woven between the MFMAs of
    // the last step (per 16-byte store: a share of the step's MFMAs, up to
    // 8 VALU instructions, the store) and only B's follow the MFMA block:
    // +4-5 % bf16 and fp16 in short runs, about +1 % in long ones, where the
    // power limit takes part of it back through the clock; results
    // bit-identical.  Elsewhere it measured 10-17 %
    // slower ((2,2,x), (4,4,2)), -1 % (128x128 tiles) or within the noise
    // (other summed operands, the compensated mode), so those keep the
    // stores after the block.
    constexpr bool kWeaveA = WA + WB == 2 && !Ops::kX3 && C::KT == 64;
    if constexpr (kFastLoop)
    for (; kt + 1 < nfast; ++kt) {
        const int cur = kt & 1;
        constexpr int NS = C::KT / 16, NL = NLA + NLB;
#pragma unroll
        for (int s = 0; s < (kWeaveA ? NS - 1 : NS); ++s) {
            load_fast_range(kt + 1, s * NL / NS, (s + 1) * NL / NS);
            __builtin_amdgcn_sched_barrier(0);
            compute_step(cur, s);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (kWeaveA) {
            load_fast_range(kt + 1, (NS - 1) * NL / NS, NL);
            __builtin_amdgcn_sched_barrier(0);
            compute_step(cur, NS - 1);
            stage_store_from(cur ^ 1, raw_a, raw_b, 1);
            constexpr int kFrags = NPLANES * (C::BM * SA::LOADS + C::BN * SB::LOADS);
            constexpr int kStoresA = SA::VECS * NPLANES * (SA::LOADS == 1 ? 1 : NV);
            constexpr int kMfmas = C::BM * C::BN * (Ops::kX3 ? 3 : 1);
            constexpr int kMfmaPerStore = kMfmas / kStoresA > 0 ? kMfmas / kStoresA : 1;
            __builtin_amdgcn_sched_group_barrier(0x100, kFrags, 0);
#pragma unroll
            for (int i = 0; i < kStoresA; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, kMfmaPerStore, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, kMfmas, 0);
            __builtin_amdgcn_sched_barrier(0);
            stage_store_from(cur ^ 1, raw_a, raw_b, 2);
        } else {
            stage_store(cur ^ 1);
        }
        __syncthreads();
    }
    // Remaining k-tiles (fringe workgroups, a ragged last k-tile).
    for (; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) stage_load((kt + 1) * C::KT);
        compute(cur);
        if (more) stage_store(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: as in the fp32 kernel (same 32x32 accumulator layout); each
    // accumulator element is scattered to all outputs before the next one.
    float *__restrict__ Cm = args.C;
    int64_t ldc = args.ldc;
    // The two epilogues of a chain address the same C tile: an opaque copy
    // of ldc keeps their addresses from being computed once and held (in
    // spilled registers) across the second k loop.
    if constexpr (CHAIN) asm volatile("" : "+s"(ldc));
    const float alpha = args.alpha, beta = args.beta;
    float g[WC];
    int64_t coff[WC];
    int crows[WC], ccols[WC], cfirst[WC];
#pragma unroll
    for (int o = 0; o < WC; ++o) {
        const bool used = o < nc && o != skip;  // an unused output is an empty block
        g[o] = P.c[o].sign * (sa0 * sb0) * alpha;
        coff[o] = P.c[o].off;
        crows[o] = used ? P.c[o].rows : 0;
        ccols[o] = used ? P.c[o].cols : 0;
        cfirst[o] = P.c[o].first;
    }
    // Interior tiles (every output block covers the whole tile): no
    // per-element guards, so each block's 16 reads of C per output are issued
    // together before its stores.
    bool c_full = true;
#pragma unroll
    for (int o = 0; o < WC; ++o)
        c_full = c_full && (crows[o] == 0 || (row0 + C::MT <= crows[o] && col0 + C::NT <= ccols[o]));
    // With up to two outputs on 256-wide tiles the reads of the next 32x32
    // block are issued before the stores of the current one (the staging
    // registers are free after the k loop), so one block's read latency
    // overlaps the previous block's stores: -1 % (4096^2 blocks) to -2 %
    // (8192^2) for the single-term compensated products with two outputs,
    // bit-identical.  With four outputs the second register set spills.
    if (c_full && WC <= 2 && C::MT == 256) {
        constexpr int NB = C::BM * C::BN;
        float cv[2][WC][16];
        auto cptr = [&](int b, int o) __attribute__((always_inline)) {
            const int cj = col0 + wn * C::WN + (b % C::BN) * 32 + l32;
            const int ci0 = row0 + wm * C::WM + (b / C::BN) * 32 + 4 * h;
            return Cm + coff[o] + (int64_t)ci0 * ldc + cj;
        };
        auto cload = [&](int b) __attribute__((always_inline)) {
#pragma unroll
            for (int o = 0; o < WC; ++o) {
                if (crows[o] == 0 || (cfirst[o] && beta == 0.f)) continue;
                const float *pc = cptr(b, o);
#pragma unroll
                for (int r = 0; r < 16; ++r) cv[b & 1][o][r] = pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc];
            }
        };
        cload(0);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b + 1 < NB) cload(b + 1);
            const int i = b / C::BN, j = b % C::BN;
#pragma unroll
            for (int o = 0; o < WC; ++o) {
                if (crows[o] == 0) continue;
                float *pc = cptr(b, o);
                const bool read = !(cfirst[o] && beta == 0.f);
                const float cb = cfirst[o] ? beta : 1.f;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] =
                        read ? cb * cv[b & 1][o][r] + g[o] * acc[i][j][r] : g[o] * acc[i][j][r];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    if (c_full) {
        // Per 32x32 block, every output's C reads are issued before any of
        // its stores (the outputs are distinct blocks), so one read latency
        // is exposed per block instead of one per output.
#pragma unroll
        for (int i = 0; i < C::BM; ++i)
#pragma unroll
            for (int j = 0; j < C::BN; ++j) {
                const int cj = col0 + wn * C::WN + j * 32 + l32;
                const int ci0 = row0 + wm * C::WM + i * 32 + 4 * h;
                float cv[WC][16];
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    if (crows[o] == 0 || (cfirst[o] && beta == 0.f)) continue;
                    const float *pc = Cm + coff[o] + (int64_t)ci0 * ldc + cj;
#pragma unroll
                    for (int r = 0; r < 16; ++r) cv[o][r] = pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc];
                }
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    if (crows[o] == 0) continue;
                    float *pc = Cm + coff[o] + (int64_t)ci0 * ldc + cj;
                    const bool read = !(cfirst[o] && beta == 0.f);
                    const float cb = cfirst[o] ? beta : 1.f;
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        pc[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] =
                            read ? cb * cv[o][r] + g[o] * acc[i][j][r] : g[o] * acc[i][j][r];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < C::BM; ++i)
#pragma unroll
        for (int j = 0; j < C::BN; ++j) {
            const int cj = col0 + wn * C::WN + j * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ci = row0 + wm * C::WM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int64_t e = (int64_t)ci * ldc + cj;
                const float m = acc[i][j][r];
#pragma unroll
                for (int o = 0; o < WC; ++o) {
                    if (ci < crows[o] && cj < ccols[o]) {
                        float *pc = Cm + coff[o] + e;
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
    };

    if constexpr (CHAIN) {
        const ProductArg &P1 = args.prod[2 * blockIdx.z];
        const ProductArg &P2 = args.prod[2 * blockIdx.z + 1];
        product(P1, 1);
        // acc = s1 M1 (s = product of the first-term signs); the carried block
        // needs c1 M1 + c2 M2 and the second epilogue scales by c2 s2, so acc
        // is negated when c1 s1 != c2 s2.  The barrier keeps the second
        // product's staging stores behind the first one's last LDS reads.
        const TermArg &out1 = P1.c[P1.carry - 1];
        const float k1 = out1.sign * P1.a[0].sign * P1.b[0].sign;
        const float k2 = P2.c[0].sign * P2.a[0].sign * P2.b[0].sign;
        if (k1 != k2)
#pragma unroll
            for (int i = 0; i < C::BM; ++i)
#pragma unroll
                for (int j = 0; j < C::BN; ++j) acc[i][j] = -acc[i][j];
        __syncthreads();
        product(P2, 2);
    } else {
        product(args.prod[blockIdx.z], 0);
    }
}

// Chained launch (CHAIN): nchains workgroup grids of two single-term
// products each, prod[2z] carrying output prod[2z].carry - 1 into
// prod[2z + 1], whose single output is that same C block.
template <class C, class Ops>
hipError_t launch_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s) {
    if (nchains < 1 || 2 * nchains > kMaxBatchArgs) return hipErrorInvalidValue;
    const dim3 grid(a.tiles_m * a.tiles_n, 1, nchains);
    const dim3 block(C::THREADS);
    hipLaunchKernelGGL((strassen_m16_kernel<C, Ops, true, false, 1, 1, 2, true>), grid, block, 0, s, a,
                       vec ? 1 : 0);
    return hipGetLastError();
}

template <class C, class Ops, bool A_KC, bool B_KC, int WA, int WB, int WC>
hipError_t launch_variant(const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    const dim3 grid(a.tiles_m * a.tiles_n, 1, batch);
    const dim3 block(C::THREADS);
    hipLaunchKernelGGL((strassen_m16_kernel<C, Ops, A_KC, B_KC, WA, WB, WC>), grid, block, 0, s, a,
                       vec ? 1 : 0);
    return hipGetLastError();
}

// 16-bit large tiles stage 64-deep k-tiles when the variant has at most four
// operand terms: one k-tile is then about 2000 MFMA cycles per SIMD, which
// amortises the barrier and the first LDS reads of each k-tile; with more
// terms the staging registers allow 32, and (1,2,2) takes 32 for its
// two-ahead loop.  The compensated mode's single-term
// product with A and B as stored takes a 32-deep k-tile with the loads
// spread over its two MFMA steps (A, k-contiguous, then loads whole 128-byte
// rows: +3 % against the 16-deep two-ahead loop, which stays faster, by
// 6-8 %, for the multi-term products; the transposed layouts were not
// measured and keep 16).
template <class C, class Ops, int WA, int WB, bool A_KC = false, bool B_KC = true>
using TileFor = typename std::conditional<
    std::is_same<C, Large>::value && !Ops::kX3 && WA + WB <= 4 && !(WA == 1 && WB == 2), LargeK64,
    typename std::conditional<std::is_same<C, LargeX3>::value && WA + WB == 2 && A_KC && !B_KC, Large,
                              C>::type>::type;

template <class C, class Ops, bool A_KC, bool B_KC>
hipError_t dispatch(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                    hipStream_t s) {
#define STRASSEN_CASE(X, Y, Z)        \
    if (wa == X && wb == Y && wc == Z) \
        return launch_variant<TileFor<C, Ops, X, Y, A_KC, B_KC>, Ops, A_KC, B_KC, X, Y, Z>(a, batch, vec, s);
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

// Pre-split compensated operands (the formed one-level schedule, A and B as
// stored): single-term products with one, two or four outputs.
template <class C, class Ops>
hipError_t dispatch_pre(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    using T = TileFor<C, Ops, 1, 1, true, false>;
    if (wa != 1 || wb != 1) return hipErrorInvalidValue;
    switch (wc) {
        case 1: return launch_variant<T, Ops, true, false, 1, 1, 1>(a, batch, vec, s);
        case 2: return launch_variant<T, Ops, true, false, 1, 1, 2>(a, batch, vec, s);
        case 4: return launch_variant<T, Ops, true, false, 1, 1, 4>(a, batch, vec, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace m16k
}  // namespace strassen
