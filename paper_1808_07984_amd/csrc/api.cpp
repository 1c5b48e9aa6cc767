// C ABI of the library (include/strassen.h): argument validation, planning,
// and one kernel launch per race-free batch of Strassen products.
#include "strassen.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernel_args.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace {

using strassen::LaunchArgs;
using strassen::Plan;
using strassen::ProductArg;
using strassen::TermArg;

thread_local hipStream_t g_stream = nullptr;

// ---------------------------------------------------------------------------
// Launch recording (strassen_profile_start / strassen_profile_stop).
// ---------------------------------------------------------------------------
struct Record {
    strassen_launch_record_t info;
    hipEvent_t e0, e1;
};

struct Recorder {
    std::mutex mu;
    bool on = false;
    int total = 0;
    std::vector<Record> recs;
    std::vector<hipEvent_t> pool;

    hipError_t take(hipEvent_t *e) {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
};

Recorder &recorder() {
    static Recorder r;
    return r;
}

// ---------------------------------------------------------------------------
// Validation.
// ---------------------------------------------------------------------------
constexpr int64_t kMaxDim = (int64_t)1 << 31;  // block extents are int32 in the kernels

size_t elem_size(strassen_dtype_t t) { return t == STRASSEN_F32 ? 4 : 2; }

bool valid_dtype(int t) { return t == STRASSEN_F32 || t == STRASSEN_BF16 || t == STRASSEN_F16; }

// Bytes spanned by an r x c row-major matrix with leading dimension ld.
uint64_t span_bytes(int64_t r, int64_t c, int64_t ld, size_t es) {
    if (r <= 0 || c <= 0) return 0;
    return ((uint64_t)(r - 1) * (uint64_t)ld + (uint64_t)c) * es;
}

bool overlap(const void *p, uint64_t np, const void *q, uint64_t nq) {
    if (np == 0 || nq == 0) return false;
    const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + nq && b < a + np;
}

struct Call {
    int64_t m, n, k;
    const void *A;
    int64_t lda;
    strassen_dtype_t a_type;
    int trans_a;
    const void *B;
    int64_t ldb;
    strassen_dtype_t b_type;
    int trans_b;
    float *C;
    int64_t ldc;
    float alpha, beta;
    int levels;
    strassen_mode_t mode;
    hipStream_t stream;
};

// Returns 0 or -(index of the offending argument in strassen_gemm_ex order).
int validate(const Call &c) {
    if (c.m < 0 || c.m >= kMaxDim) return -1;
    if (c.n < 0 || c.n >= kMaxDim) return -2;
    if (c.k < 0 || c.k >= kMaxDim) return -3;
    // A and B are read only when the product term is present.
    const bool product = c.m > 0 && c.n > 0 && c.k > 0 && c.alpha != 0.f;
    if (!valid_dtype(c.a_type)) return -6;
    if (c.trans_a != 0 && c.trans_a != 1) return -7;
    if (!valid_dtype(c.b_type) || c.b_type != c.a_type) return -10;
    if (c.trans_b != 0 && c.trans_b != 1) return -11;
    // stored shapes: A is m x k (k x m if transposed), B is k x n (n x k)
    const int64_t a_rows = c.trans_a ? c.k : c.m, a_cols = c.trans_a ? c.m : c.k;
    const int64_t b_rows = c.trans_b ? c.n : c.k, b_cols = c.trans_b ? c.k : c.n;
    if (product && c.A == nullptr) return -4;
    if (c.lda < (a_cols > 1 ? a_cols : 1)) return -5;
    if (product && c.B == nullptr) return -8;
    if (c.ldb < (b_cols > 1 ? b_cols : 1)) return -9;
    if (c.m > 0 && c.n > 0 && c.C == nullptr) return -12;
    if (c.ldc < (c.n > 1 ? c.n : 1)) return -13;
    if (c.levels < 0 || c.levels > STRASSEN_MAX_LEVELS) return -16;
    if (c.mode != STRASSEN_MODE_PLAIN && c.mode != STRASSEN_MODE_BF16X3) return -17;
    if (c.mode == STRASSEN_MODE_BF16X3 && c.a_type != STRASSEN_F32) return -17;
    if (product) {
        const uint64_t nc = span_bytes(c.m, c.n, c.ldc, 4);
        const size_t es = elem_size(c.a_type);
        if (overlap(c.A, span_bytes(a_rows, a_cols, c.lda, es), c.C, nc)) return -12;
        if (overlap(c.B, span_bytes(b_rows, b_cols, c.ldb, es), c.C, nc)) return -12;
    }
    // Transposed operands exist for fp32 data (plain and compensated) only.
    if (c.a_type != STRASSEN_F32 && c.trans_a) return -7;
    if (c.a_type != STRASSEN_F32 && c.trans_b) return -11;
    return 0;
}

// ---------------------------------------------------------------------------
// Execution.
// ---------------------------------------------------------------------------
TermArg term(int64_t off, int64_t rows, int64_t cols, int sign, bool first) {
    TermArg t;
    t.off = off;
    t.rows = (int32_t)rows;
    t.cols = (int32_t)cols;
    t.sign = (float)sign;
    t.first = first ? 1 : 0;
    return t;
}

// Tile choice of the product kernels (strassen_set_tile): automatic, or
// forced to 128x128 / 256x256 for tuning and testing.  Per calling thread,
// like the stream, so concurrent callers do not change each other's calls.
thread_local int g_tile = STRASSEN_TILE_AUTO;

// Schedule of the products (strassen_set_schedule), per calling thread.
thread_local int g_schedule = STRASSEN_SCHEDULE_BATCHED;

bool use_large(int64_t sm, int64_t sn, int64_t sk, int batch, bool f32) {
    const int mode = g_tile;
    if (mode == STRASSEN_TILE_128) return false;
    if (mode == STRASSEN_TILE_256) return true;
    const int64_t per_product = ((sm + 255) / 256) * ((sn + 255) / 256);
    if (!f32) {
        // 16-bit operands: the 128x128 tile measured 25-40 % slower per flop,
        // so the 256x256 tile is kept whenever it fills the CUs once.
        return per_product >= 128 && per_product * batch >= 256;
    }
    // fp32: the launch runs in waves of workgroups (256 slots for the
    // 256x256 tile, one per CU; 512 for the 128x128 tile, two per CU).  Cost
    // of a wave in units of one k step of a 256x256 tile, fitted to MI355X
    // measurements (squares 4096-16384, rank-k 16384^2 x 1024 and 2048,
    // levels 0-2): sk + 62.5 for the 256x256 tile; 0.5 (1.045 sk + 16.5) for
    // two 128x128 tiles sharing a CU (a quarter of the work each, 4.5 %
    // slower per flop in the k loop, less fixed cost per tile), and 0.65 of
    // that for a last wave with at most one of them per CU.  The cheaper
    // shape is taken.
    const int64_t tiles256 = per_product * batch;
    const int64_t tiles128 = ((sm + 127) / 128) * ((sn + 127) / 128) * batch;
    const double k = (double)sk;
    const double cost256 = (double)((tiles256 + 255) / 256) * (k + 62.5);
    const double pair = 0.5 * (1.045 * k + 16.5);
    const int64_t full128 = tiles128 / 512, rest128 = tiles128 % 512;
    const double cost128 = (double)full128 * pair +
                           (rest128 == 0 ? 0.0 : rest128 <= 256 ? 0.65 * pair : pair);
    return cost256 <= cost128;
}

// Kernel family of a call: fp32 MFMA, or the 16-bit MFMA path.
struct Family {
    bool m16;
    strassen::Operand16 op;
    int vec;  // elements per aligned vector load
};

Family family(strassen_dtype_t t, strassen_mode_t mode) {
    using strassen::Operand16;
    if (t == STRASSEN_F32 && mode == STRASSEN_MODE_PLAIN) return Family{false, Operand16::kBf16, 4};
    const Operand16 op = (t == STRASSEN_BF16) ? Operand16::kBf16
                         : (t == STRASSEN_F16) ? Operand16::kF16
                                               : Operand16::kBf16x3;
    return Family{true, op, strassen::m16_tile_shape(op == Operand16::kBf16x3, false).vec};
}

strassen::KernelShape shape_of(const Family &f, bool large, int wa, int wb, int wc, bool untransposed) {
    return f.m16 ? strassen::m16_tile_shape(f.op == strassen::Operand16::kBf16x3, large, wa, wb, untransposed)
                 : strassen::f32_tile_shape(large, wa, wb, wc, untransposed);
}

// Task-parallel schedule for small problems (Task Parallelism section,
// element-wise atomic update with batching): beta is applied to C first, then
// the products are launched up to eight at a time regardless of variant and
// every output is added with fp32 atomics, so one launch covers all seven
// products at one level and seven launches the 49 at two.  The order of the
// atomic additions is not fixed: results differ between runs in the last bits.
int run_concurrent(const Call &c, const Plan &plan, bool vec) {
    const int d = plan.d;
    hipError_t err = strassen::launch_scale(c.C, c.ldc, c.m, c.n, c.beta, c.stream);
    if (err != hipSuccess) return (int)err;
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = c.A;
    a.B = c.B;
    a.C = c.C;
    a.lda = c.lda;
    a.ldb = c.ldb;
    a.ldc = c.ldc;
    a.sm = (int32_t)plan.sm;
    a.sn = (int32_t)plan.sn;
    a.sk = (int32_t)plan.sk;
    a.alpha = c.alpha;
    a.beta = 1.f;
    const int total = (int)plan.products.size();
    const int wmax = plan.levels >= 2 ? 4 : 2;
    Recorder &rec = recorder();
    for (int first = 0, launch = 0; first < total; first += strassen::kMaxBatchArgs, ++launch) {
        const int batch = std::min(strassen::kMaxBatchArgs, total - first);
        const bool large = use_large(plan.sm, plan.sn, plan.sk, batch, true);
        const strassen::KernelShape ks = strassen::f32_tile_shape(large);
        a.tiles_m = (int32_t)((plan.sm + ks.mt - 1) / ks.mt);
        a.tiles_n = (int32_t)((plan.sn + ks.nt - 1) / ks.nt);
        for (int z = 0; z < batch; ++z) {
            const strassen::Product &p = plan.products[first + z];
            ProductArg &pa = a.prod[z];
            std::memset(&pa, 0, sizeof(pa));
            pa.na = p.na;
            pa.nb = p.nb;
            pa.nc = p.nc;
            for (int t = 0; t < p.na; ++t) {
                const int R = p.a[t].block / d, Cc = p.a[t].block % d;
                pa.a[t] = term(R * plan.sm * c.lda + Cc * plan.sk,
                               strassen::block_extent(c.m, plan.sm, R),
                               strassen::block_extent(c.k, plan.sk, Cc), p.a[t].sign, false);
            }
            for (int t = 0; t < p.nb; ++t) {
                const int R = p.b[t].block / d, Cc = p.b[t].block % d;
                pa.b[t] = term(R * plan.sk * c.ldb + Cc * plan.sn,
                               strassen::block_extent(c.k, plan.sk, R),
                               strassen::block_extent(c.n, plan.sn, Cc), p.b[t].sign, false);
            }
            for (int t = 0; t < p.nc; ++t) {
                const int R = p.c[t].block / d, Cc = p.c[t].block % d;
                pa.c[t] = term(R * plan.sm * c.ldc + Cc * plan.sn,
                               strassen::block_extent(c.m, plan.sm, R),
                               strassen::block_extent(c.n, plan.sn, Cc), p.c[t].sign, false);
            }
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool timed = false;
        {
            std::lock_guard<std::mutex> lk(rec.mu);
            if (rec.on) {
                hipError_t e = rec.take(&e0);
                if (e == hipSuccess) e = rec.take(&e1);
                if (e != hipSuccess) return (int)e;
                timed = true;
            }
        }
        if (timed && (err = hipEventRecord(e0, c.stream)) != hipSuccess) return (int)err;
        err = large ? strassen::launch_f32_conc_l(wmax, a, batch, vec, c.stream)
                    : strassen::launch_f32_conc_s(wmax, a, batch, vec, c.stream);
        if (err != hipSuccess) return (int)err;
        if (timed) {
            if ((err = hipEventRecord(e1, c.stream)) != hipSuccess) return (int)err;
            Record r;
            std::memset(&r.info, 0, sizeof(r.info));
            std::snprintf(r.info.kernel, sizeof(r.info.kernel), "%s<concurrent,%d>",
                          strassen::f32_kernel_name(large), wmax);
            r.info.launch = launch;
            r.info.batch = batch;
            r.info.workgroups = a.tiles_m * a.tiles_n * batch;
            r.info.flops = 2.0 * batch * (double)plan.sm * (double)plan.sn * (double)plan.sk;
            r.e0 = e0;
            r.e1 = e1;
            std::lock_guard<std::mutex> lk(rec.mu);
            rec.recs.push_back(r);
            ++rec.total;
        }
    }
    return 0;
}

// Starts the launch record of one kernel when recording is on.
int record_begin(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1, bool *timed) {
    Recorder &rec = recorder();
    *timed = false;
    {
        std::lock_guard<std::mutex> lk(rec.mu);
        if (!rec.on) return 0;
        hipError_t e = rec.take(e0);
        if (e == hipSuccess) e = rec.take(e1);
        if (e != hipSuccess) return (int)e;
    }
    *timed = true;
    return (int)hipEventRecord(*e0, s);
}

int record_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1, const char *kernel, int launch, int batch,
               int workgroups, double flops) {
    const hipError_t err = hipEventRecord(e1, s);
    if (err != hipSuccess) return (int)err;
    Record r;
    std::memset(&r.info, 0, sizeof(r.info));
    std::snprintf(r.info.kernel, sizeof(r.info.kernel), "%s", kernel);
    r.info.launch = launch;
    r.info.batch = batch;
    r.info.workgroups = workgroups;
    r.info.flops = flops;
    r.e0 = e0;
    r.e1 = e1;
    Recorder &rec = recorder();
    std::lock_guard<std::mutex> lk(rec.mu);
    rec.recs.push_back(r);
    ++rec.total;
    return 0;
}

// A second stream of the calling thread on one device, with a fork and a
// join event, on which the formed schedule runs B's form beside the product
// launches that need no formed B operand.  Created on first use (default
// priority, non-blocking) and kept until the thread ends.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t ready[16] = {};  // formed two-level: one per sum-forming launch
};
constexpr int kSideDevices = 64;
thread_local SideStream g_side[kSideDevices];

hipError_t side_stream(hipStream_t caller, SideStream **out) {
    int dev = 0;
    hipError_t err = caller ? hipStreamGetDevice(caller, &dev) : hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kSideDevices) return hipErrorInvalidDevice;
    SideStream &ss = g_side[dev];
    if (ss.s == nullptr) {
        int cur = 0;
        if ((err = hipGetDevice(&cur)) != hipSuccess) return err;
        if (cur != dev && (err = hipSetDevice(dev)) != hipSuccess) return err;
        err = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming);
        for (int i = 0; i < 16 && err == hipSuccess; ++i)
            err = hipEventCreateWithFlags(&ss.ready[i], hipEventDisableTiming);
        const hipError_t back = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (err != hipSuccess) return err;
        if (back != hipSuccess) return back;
    }
    *out = &ss;
    return hipSuccess;
}

int run_streams(const Call &c, const Plan &plan, const Family &fam, bool vec);

int run(const Call &c) {
    if (c.m == 0 || c.n == 0) return 0;
    if (c.k == 0 || c.alpha == 0.f)
        return (int)strassen::launch_scale(c.C, c.ldc, c.m, c.n, c.beta, c.stream);

    const Family fam = family(c.a_type, c.mode);
    const Plan plan = strassen::make_plan(c.m, c.n, c.k, c.levels, fam.vec, c.trans_a != 0);
    const int d = plan.d;

    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = c.A;
    a.B = c.B;
    a.C = c.C;
    a.lda = c.lda;
    a.ldb = c.ldb;
    a.ldc = c.ldc;
    a.sm = (int32_t)plan.sm;
    a.sn = (int32_t)plan.sn;
    a.sk = (int32_t)plan.sk;
    a.alpha = c.alpha;
    a.beta = c.beta;
    a.trans_a = c.trans_a;
    a.trans_b = c.trans_b;

    // 16-byte loads need aligned bases, leading dimensions and block offsets
    // (make_plan rounds block extents to the vector width).
    const bool vec = (c.lda % fam.vec == 0) && (c.ldb % fam.vec == 0) &&
                     ((uintptr_t)c.A % 16 == 0) && ((uintptr_t)c.B % 16 == 0);

    if (g_schedule == STRASSEN_SCHEDULE_CONCURRENT && !fam.m16 &&
        !c.trans_a && !c.trans_b && c.levels > 0)
        return run_concurrent(c, plan, vec);
    if (g_schedule == STRASSEN_SCHEDULE_STREAMS && c.levels == 1) return run_streams(c, plan, fam, vec);

    Recorder &rec = recorder();
    for (size_t bi = 0; bi < plan.batches.size(); ++bi) {
        const strassen::Batch &bt = plan.batches[bi];
        const int batch = (int)bt.products.size();
        const bool large = use_large(plan.sm, plan.sn, plan.sk, batch, !fam.m16);
        const strassen::KernelShape ks = shape_of(fam, large, bt.wa, bt.wb, bt.wc, !c.trans_a && !c.trans_b);
        a.tiles_m = (int32_t)((plan.sm + ks.mt - 1) / ks.mt);
        a.tiles_n = (int32_t)((plan.sn + ks.nt - 1) / ks.nt);
        for (int z = 0; z < batch; ++z) {
            const strassen::Product &p = plan.products[bt.products[z]];
            ProductArg &pa = a.prod[z];
            pa.na = p.na;
            pa.nb = p.nb;
            pa.nc = p.nc;
            // Block (R, Cc) of op(X) starts at row R, column Cc of the block
            // grid; a transposed operand stores it at column R, row Cc.
            for (int t = 0; t < p.na; ++t) {
                const int R = p.a[t].block / d, Cc = p.a[t].block % d;
                const int64_t off = c.trans_a ? Cc * plan.sk * c.lda + R * plan.sm
                                              : R * plan.sm * c.lda + Cc * plan.sk;
                pa.a[t] = term(off, strassen::block_extent(c.m, plan.sm, R),
                               strassen::block_extent(c.k, plan.sk, Cc), p.a[t].sign, false);
            }
            for (int t = 0; t < p.nb; ++t) {
                const int R = p.b[t].block / d, Cc = p.b[t].block % d;
                const int64_t off = c.trans_b ? Cc * plan.sn * c.ldb + R * plan.sk
                                              : R * plan.sk * c.ldb + Cc * plan.sn;
                pa.b[t] = term(off, strassen::block_extent(c.k, plan.sk, R),
                               strassen::block_extent(c.n, plan.sn, Cc), p.b[t].sign, false);
            }
            for (int t = 0; t < p.nc; ++t) {
                const int R = p.c[t].block / d, Cc = p.c[t].block % d;
                pa.c[t] = term(R * plan.sm * c.ldc + Cc * plan.sn,
                               strassen::block_extent(c.m, plan.sm, R),
                               strassen::block_extent(c.n, plan.sn, Cc), p.c[t].sign,
                               p.c_first[t]);
            }
        }

        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool timed = false;
        {
            std::lock_guard<std::mutex> lk(rec.mu);
            if (rec.on) {
                hipError_t err = rec.take(&e0);
                if (err == hipSuccess) err = rec.take(&e1);
                if (err != hipSuccess) return (int)err;
                timed = true;
            }
        }
        if (timed) {
            const hipError_t err = hipEventRecord(e0, c.stream);
            if (err != hipSuccess) return (int)err;
        }
        const hipError_t err =
            fam.m16 ? strassen::launch_m16(fam.op, c.trans_a != 0, c.trans_b != 0, large, bt.wa,
                                           bt.wb, bt.wc, a, batch, vec, c.stream)
                    : strassen::launch_f32(c.trans_a != 0, c.trans_b != 0, large, bt.wa, bt.wb,
                                           bt.wc, a, batch, vec, c.stream);
        if (err != hipSuccess) return (int)err;
        if (timed) {
            const hipError_t e2 = hipEventRecord(e1, c.stream);
            if (e2 != hipSuccess) return (int)e2;
            Record r;
            std::memset(&r.info, 0, sizeof(r.info));
            std::snprintf(r.info.kernel, sizeof(r.info.kernel), "%s<%d,%d,%d,%s%s%s>",
                          fam.m16 ? strassen::m16_kernel_name(fam.op, large)
                                  : strassen::f32_kernel_name(large),
                          bt.wa, bt.wb, bt.wc, vec ? "vec" : "scalar", c.trans_a ? ",tA" : "",
                          c.trans_b ? ",tB" : "");
            r.info.launch = (int32_t)bi;
            r.info.batch = batch;
            r.info.workgroups = a.tiles_m * a.tiles_n * batch;
            r.info.flops = 2.0 * (double)batch * (double)plan.sm * (double)plan.sn * (double)plan.sk;
            r.e0 = e0;
            r.e1 = e1;
            std::lock_guard<std::mutex> lk(rec.mu);
            rec.recs.push_back(r);
            ++rec.total;
        }
    }
    return 0;
}

// Stream-by-stage schedule (Task Parallelism section, table tab:gpu_streaming):
// each one-level product is one launch, on the caller's stream (0) or the
// side stream (1) as the table assigns it; the products of a stage run at
// once, and each stage waits for the previous one on both streams (the two
// streams of a stage write disjoint C quadrants).  Beta is applied by the
// first update of each quadrant in this order.
int run_streams(const Call &c, const Plan &plan, const Family &fam, bool vec) {
    SideStream *ss = nullptr;
    hipError_t err = side_stream(c.stream, &ss);
    if (err != hipSuccess) return (int)err;
    const std::vector<strassen::Product> all = strassen::scheme(1);
    const std::vector<strassen::StreamSlot> slots = strassen::stream_stages();
    bool touched[4] = {false, false, false, false};
    // the side stream starts after the caller's earlier work
    if ((err = hipEventRecord(ss->fork, c.stream)) != hipSuccess) return (int)err;
    if ((err = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return (int)err;
    int stage = 0;
    for (size_t i = 0; i < slots.size(); ++i) {
        const strassen::StreamSlot &sl = slots[i];
        if (sl.stage != stage) {
            // stage barrier: each stream waits for the other's work so far
            if ((err = hipEventRecord(ss->fork, c.stream)) != hipSuccess) return (int)err;
            if ((err = hipEventRecord(ss->join, ss->s)) != hipSuccess) return (int)err;
            if ((err = hipStreamWaitEvent(c.stream, ss->join, 0)) != hipSuccess) return (int)err;
            if ((err = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return (int)err;
            stage = sl.stage;
        }
        const strassen::Product &p = all[sl.product];
        const hipStream_t s = sl.stream == 0 ? c.stream : ss->s;
        LaunchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.A = c.A;
        a.B = c.B;
        a.C = c.C;
        a.lda = c.lda;
        a.ldb = c.ldb;
        a.ldc = c.ldc;
        a.sm = (int32_t)plan.sm;
        a.sn = (int32_t)plan.sn;
        a.sk = (int32_t)plan.sk;
        a.alpha = c.alpha;
        a.beta = c.beta;
        a.trans_a = c.trans_a;
        a.trans_b = c.trans_b;
        const bool large = use_large(plan.sm, plan.sn, plan.sk, 1, !fam.m16);
        const strassen::KernelShape ks = shape_of(fam, large, p.na, p.nb, p.nc, !c.trans_a && !c.trans_b);
        a.tiles_m = (int32_t)((plan.sm + ks.mt - 1) / ks.mt);
        a.tiles_n = (int32_t)((plan.sn + ks.nt - 1) / ks.nt);
        ProductArg &pa = a.prod[0];
        pa.na = p.na;
        pa.nb = p.nb;
        pa.nc = p.nc;
        for (int t = 0; t < p.na; ++t) {
            const int R = p.a[t].block / 2, Cc = p.a[t].block % 2;
            const int64_t off = c.trans_a ? Cc * plan.sk * c.lda + R * plan.sm : R * plan.sm * c.lda + Cc * plan.sk;
            pa.a[t] = term(off, strassen::block_extent(c.m, plan.sm, R), strassen::block_extent(c.k, plan.sk, Cc),
                           p.a[t].sign, false);
        }
        for (int t = 0; t < p.nb; ++t) {
            const int R = p.b[t].block / 2, Cc = p.b[t].block % 2;
            const int64_t off = c.trans_b ? Cc * plan.sn * c.ldb + R * plan.sk : R * plan.sk * c.ldb + Cc * plan.sn;
            pa.b[t] = term(off, strassen::block_extent(c.k, plan.sk, R), strassen::block_extent(c.n, plan.sn, Cc),
                           p.b[t].sign, false);
        }
        for (int t = 0; t < p.nc; ++t) {
            const int blk = p.c[t].block, R = blk / 2, Cc = blk % 2;
            pa.c[t] = term(R * plan.sm * c.ldc + Cc * plan.sn, strassen::block_extent(c.m, plan.sm, R),
                           strassen::block_extent(c.n, plan.sn, Cc), p.c[t].sign, !touched[blk]);
            touched[blk] = true;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool timed = false;
        int rc = record_begin(s, &e0, &e1, &timed);
        if (rc != 0) return rc;
        err = fam.m16 ? strassen::launch_m16(fam.op, c.trans_a != 0, c.trans_b != 0, large, p.na, p.nb, p.nc, a, 1,
                                             vec, s)
                      : strassen::launch_f32(c.trans_a != 0, c.trans_b != 0, large, p.na, p.nb, p.nc, a, 1, vec, s);
        if (err != hipSuccess) return (int)err;
        if (timed) {
            char name[64];
            std::snprintf(name, sizeof(name), "%s<%d,%d,%d,stream %d>",
                          fam.m16 ? strassen::m16_kernel_name(fam.op, large) : strassen::f32_kernel_name(large),
                          p.na, p.nb, p.nc, sl.stream);
            rc = record_end(s, e0, e1, name, (int)i, 1, a.tiles_m * a.tiles_n,
                            2.0 * (double)plan.sm * (double)plan.sn * (double)plan.sk);
            if (rc != 0) return rc;
        }
    }
    // the caller's stream waits for the side stream's last work
    if ((err = hipEventRecord(ss->join, ss->s)) != hipSuccess) return (int)err;
    if ((err = hipStreamWaitEvent(c.stream, ss->join, 0)) != hipSuccess) return (int)err;
    return 0;
}

// ---------------------------------------------------------------------------
// Hybrid two-level scheme (Two-Level Strassen's Algorithm section): the top
// level forms each product's signed quadrant sums P (of A) and Q (of B) in
// caller workspace; the fused one-level kernels compute P*Q and scatter it
// straight into the 4x4 grid of C blocks.  Geometry equals the direct two-
// level plan's: C blocks are sm x sn, P is (2 sm) x (2 sk), Q (2 sk) x (2 sn).
// ---------------------------------------------------------------------------
struct HybridGeom {
    Plan two;    // direct two-level plan: block extents sm, sn, sk
    Plan inner;  // one-level plan of the (2sm x 2sn x 2sk) product P*Q
    int64_t p_elems, q_elems;
};

HybridGeom hybrid_geom(int64_t m, int64_t n, int64_t k) {
    HybridGeom g;
    g.two = strassen::make_plan(m, n, k, 2, 4);
    g.inner = strassen::make_plan(2 * g.two.sm, 2 * g.two.sn, 2 * g.two.sk, 1, 4);
    g.p_elems = (2 * g.two.sm) * (2 * g.two.sk);
    g.q_elems = (2 * g.two.sk) * (2 * g.two.sn);
    return g;
}

int run_hybrid(const Call &c, float *ws) {
    if (c.m == 0 || c.n == 0) return 0;
    if (c.k == 0 || c.alpha == 0.f)
        return (int)strassen::launch_scale(c.C, c.ldc, c.m, c.n, c.beta, c.stream);
    const HybridGeom g = hybrid_geom(c.m, c.n, c.k);
    const int64_t sm = g.two.sm, sn = g.two.sn, sk = g.two.sk;
    const float *A = static_cast<const float *>(c.A);
    const float *B = static_cast<const float *>(c.B);
    float *P = ws;
    float *Q = ws + g.p_elems;
    const bool vec_a = (c.lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
    const bool vec_b = (c.ldb % 4 == 0) && ((uintptr_t)B % 16 == 0);
    const std::vector<strassen::Product> top = strassen::scheme(1);
    const Plan &in = g.inner;
    bool touched[16] = {false};

    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = P;
    a.B = Q;
    a.C = c.C;
    a.lda = 2 * sk;
    a.ldb = 2 * sn;
    a.ldc = c.ldc;
    a.sm = (int32_t)sm;
    a.sn = (int32_t)sn;
    a.sk = (int32_t)sk;
    a.alpha = c.alpha;
    a.beta = c.beta;

    Recorder &rec = recorder();
    for (const strassen::Product &tp : top) {
        // P = sum of signed quadrants of A, Q = sum of signed quadrants of B
        strassen::FormTerm ft[2];
        for (int t = 0; t < tp.na; ++t) {
            const int r1 = tp.a[t].block / 2, c1 = tp.a[t].block % 2;
            ft[t].src = A + r1 * 2 * sm * c.lda + c1 * 2 * sk;
            ft[t].rows = (int32_t)strassen::block_extent(c.m, 2 * sm, r1);
            ft[t].cols = (int32_t)strassen::block_extent(c.k, 2 * sk, c1);
            ft[t].sign = (float)tp.a[t].sign;
        }
        hipError_t err = strassen::launch_form(P, 2 * sk, 2 * sm, 2 * sk, c.lda, ft, tp.na, vec_a,
                                               c.stream);
        if (err != hipSuccess) return (int)err;
        for (int t = 0; t < tp.nb; ++t) {
            const int r1 = tp.b[t].block / 2, c1 = tp.b[t].block % 2;
            ft[t].src = B + r1 * 2 * sk * c.ldb + c1 * 2 * sn;
            ft[t].rows = (int32_t)strassen::block_extent(c.k, 2 * sk, r1);
            ft[t].cols = (int32_t)strassen::block_extent(c.n, 2 * sn, c1);
            ft[t].sign = (float)tp.b[t].sign;
        }
        err = strassen::launch_form(Q, 2 * sn, 2 * sk, 2 * sn, c.ldb, ft, tp.nb, vec_b, c.stream);
        if (err != hipSuccess) return (int)err;

        // P*Q by the fused one-level kernels; outputs are the top outputs'
        // quadrants refined by the inner outputs' quadrants.
        for (size_t bi = 0; bi < in.batches.size(); ++bi) {
            const strassen::Batch &bt = in.batches[bi];
            const int batch = (int)bt.products.size();
            const int wc = bt.wc * tp.nc;
            const bool large = use_large(sm, sn, sk, batch, true);
            const strassen::KernelShape ks = strassen::f32_tile_shape(large);
            a.tiles_m = (int32_t)((sm + ks.mt - 1) / ks.mt);
            a.tiles_n = (int32_t)((sn + ks.nt - 1) / ks.nt);
            for (int z = 0; z < batch; ++z) {
                const strassen::Product &p = in.products[bt.products[z]];
                ProductArg &pa = a.prod[z];
                std::memset(&pa, 0, sizeof(pa));
                pa.na = p.na;
                pa.nb = p.nb;
                pa.nc = p.nc * tp.nc;
                for (int t = 0; t < p.na; ++t) {
                    const int R = p.a[t].block / 2, Cc = p.a[t].block % 2;
                    pa.a[t] = term(R * sm * (2 * sk) + Cc * sk, sm, sk, p.a[t].sign, false);
                }
                for (int t = 0; t < p.nb; ++t) {
                    const int R = p.b[t].block / 2, Cc = p.b[t].block % 2;
                    pa.b[t] = term(R * sk * (2 * sn) + Cc * sn, sk, sn, p.b[t].sign, false);
                }
                int o = 0;
                for (int t1 = 0; t1 < tp.nc; ++t1)
                    for (int t2 = 0; t2 < p.nc; ++t2, ++o) {
                        const int q1 = tp.c[t1].block, q2 = p.c[t2].block;
                        const int R = 2 * (q1 / 2) + q2 / 2, Cc = 2 * (q1 % 2) + q2 % 2;
                        const bool first = !touched[R * 4 + Cc];
                        touched[R * 4 + Cc] = true;
                        pa.c[o] = term(R * sm * c.ldc + Cc * sn, strassen::block_extent(c.m, sm, R),
                                       strassen::block_extent(c.n, sn, Cc),
                                       tp.c[t1].sign * p.c[t2].sign, first);
                    }
            }
            hipEvent_t e0 = nullptr, e1 = nullptr;
            bool timed = false;
            {
                std::lock_guard<std::mutex> lk(rec.mu);
                if (rec.on) {
                    hipError_t e = rec.take(&e0);
                    if (e == hipSuccess) e = rec.take(&e1);
                    if (e != hipSuccess) return (int)e;
                    timed = true;
                }
            }
            if (timed && (err = hipEventRecord(e0, c.stream)) != hipSuccess) return (int)err;
            err = strassen::launch_f32(false, false, large, bt.wa, bt.wb, wc, a, batch, true,
                                       c.stream);
            if (err != hipSuccess) return (int)err;
            if (timed) {
                if ((err = hipEventRecord(e1, c.stream)) != hipSuccess) return (int)err;
                Record r;
                std::memset(&r.info, 0, sizeof(r.info));
                std::snprintf(r.info.kernel, sizeof(r.info.kernel), "%s<%d,%d,%d,vec>",
                              strassen::f32_kernel_name(large), bt.wa, bt.wb, wc);
                r.info.launch = (int32_t)bi;
                r.info.batch = batch;
                r.info.workgroups = a.tiles_m * a.tiles_n * batch;
                r.info.flops = 2.0 * batch * (double)sm * (double)sn * (double)sk;
                r.e0 = e0;
                r.e1 = e1;
                std::lock_guard<std::mutex> lk(rec.mu);
                rec.recs.push_back(r);
                ++rec.total;
            }
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// One-level "formed" schedule (the Two-Level section's hybrid idea applied at
// the one level itself): every two-term operand sum of the seven products of
// eq. gpu_allops (five of A, five of B) is written once into caller
// workspace by one streaming pass per operand, which reads each quadrant
// once; each product then runs the single-term kernel, A and B read from the
// workspace or straight from the quadrant, and its accumulator is scattered
// with signs into its C blocks as in the fused schedule, so C needs no
// workspace.  The sums are formed in the fused kernels' order and precision
// (fp32 from the stored values, the first term's sign factored out, 16-bit
// data rounded once), and the product kernels accumulate in the same k
// order, so the result equals the fused one-level result bit for bit --
// except where chains apply (16-bit kernels on 256x256 tiles): there the two
// single-output products M5 and M6 are accumulated after M2 and M3 and added
// into C3 and C0 together with them, saving two read-modify-writes of a C
// block and a launch, and those two blocks can differ in the last bits.
// Two levels: the same for the 49 products on the 4 x 4 block grid, whose
// operands are up to four-term sums (formed by the general-term kernel, one
// launch per level-1 operand), without chains, the batches in the fused
// schedule's order: the result is the fused two-level result bit for bit.
// ---------------------------------------------------------------------------
struct FormedSum {
    int nterms;
    strassen::Term t[strassen::kMaxTerms];  // t[0].sign = +1; the others relative to the first
};

struct FormedGeom {
    Plan plan;                            // one- or two-level plan (block extents)
    std::vector<FormedSum> asums, bsums;  // distinct multi-term operands
    std::vector<int> a_of, b_of;          // per product: its sum, or -1
    size_t es = 4;                        // bytes per workspace element
    int64_t a_bytes = 0, bytes = 0;
    // Compensated mode: the workspace operands are written pre-split, and
    // the single blocks that products take as operands too -- A's at one
    // level (B's single quadrants are read as stored by the products that
    // run beside B's form), A's and B's at two levels and at level 0 (the
    // plain product on pre-split copies of A and B) -- so that products
    // stage pre-split operands.
    bool pre = false;
};

int find_or_add(std::vector<FormedSum> &sums, const strassen::Term *t, int n) {
    FormedSum f;
    f.nterms = n;
    for (int i = 0; i < n; ++i) f.t[i] = strassen::Term{t[i].block, t[i].sign * t[0].sign};
    for (size_t j = 0; j < sums.size(); ++j) {
        bool same = sums[j].nterms == n;
        for (int i = 0; i < n && same; ++i)
            same = sums[j].t[i].block == f.t[i].block && sums[j].t[i].sign == f.t[i].sign;
        if (same) return (int)j;
    }
    sums.push_back(f);
    return (int)sums.size() - 1;
}

FormedGeom formed_geom(int64_t m, int64_t n, int64_t k, const Family &fam, int levels) {
    FormedGeom g;
    g.plan = strassen::make_plan(m, n, k, levels, fam.vec);
    g.pre = fam.m16 && fam.op == strassen::Operand16::kBf16x3;
    if (levels == 0 && g.pre) {
        // pre-split copies need whole 16-byte units per row: the workspace
        // blocks' k and n extents are rounded up (the product's own extents
        // clip at k and n; rounding by less than 4 adds no tile)
        g.plan.sk = (g.plan.sk + fam.vec - 1) / fam.vec * fam.vec;
        g.plan.sn = (g.plan.sn + fam.vec - 1) / fam.vec * fam.vec;
    }
    const bool b_singles = g.pre && levels != 1;
    for (const strassen::Product &p : g.plan.products) {
        g.a_of.push_back(p.na > 1 || g.pre ? find_or_add(g.asums, p.a, p.na) : -1);
        g.b_of.push_back(p.nb > 1 || b_singles ? find_or_add(g.bsums, p.b, p.nb) : -1);
    }
    g.es = (fam.m16 && fam.op != strassen::Operand16::kBf16x3) ? 2 : 4;
    const Plan &pl = g.plan;
    g.a_bytes = (int64_t)g.es * (int64_t)g.asums.size() * pl.sm * pl.sk;
    g.bytes = g.a_bytes + (int64_t)g.es * (int64_t)g.bsums.size() * pl.sk * pl.sn;
    return g;
}

// Forms the sums of one operand X (quadrant (R, Cc) at X + R*srows*ldx +
// Cc*scols, extents clipped to xr x xc) into `out`, one srows x scols block
// per sum, dense with leading dimension scols.
int form_operand(const std::vector<FormedSum> &sums, strassen::FormElem fe, size_t es, const void *X,
                 int64_t ldx, int64_t xr, int64_t xc, int64_t srows, int64_t scols, char *out,
                 bool vec, hipStream_t s, int launch) {
    if (sums.empty()) return 0;
    for (const FormedSum &f : sums)
        if (f.nterms > 2) return (int)hipErrorInvalidValue;  // one level: at most two terms
    strassen::FormSource src[strassen::kFormMaxSources];
    int blocks[strassen::kFormMaxSources];
    int nsrc = 0;
    auto source_of = [&](int block) {
        for (int q = 0; q < nsrc; ++q)
            if (blocks[q] == block) return q;
        const int R = block / 2, Cc = block % 2;
        blocks[nsrc] = block;
        src[nsrc].ptr = static_cast<const char *>(X) + ((uint64_t)R * srows * ldx + (uint64_t)Cc * scols) * es;
        src[nsrc].rows = (int32_t)strassen::block_extent(xr, srows, R);
        src[nsrc].cols = (int32_t)strassen::block_extent(xc, scols, Cc);
        return nsrc++;
    };
    strassen::FormOut o[strassen::kFormMaxOutputs];
    if ((int)sums.size() > strassen::kFormMaxOutputs) return (int)hipErrorInvalidValue;
    for (size_t i = 0; i < sums.size(); ++i) {
        o[i].ptr = out + (uint64_t)i * srows * scols * es;
        o[i].t0 = source_of(sums[i].t[0].block);
        o[i].t1 = sums[i].nterms > 1 ? source_of(sums[i].t[1].block) : -1;
        o[i].s1 = sums[i].nterms > 1 ? (float)sums[i].t[1].sign : 0.f;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool timed = false;
    int rc = record_begin(s, &e0, &e1, &timed);
    if (rc != 0) return rc;
    const hipError_t err = strassen::launch_form_sums(fe, src, nsrc, ldx, o, (int)sums.size(), scols,
                                                      srows, scols, vec, s);
    if (err != hipSuccess) return (int)err;
    if (timed)
        return record_end(s, e0, e1,
                          fe == strassen::FormElem::kF32        ? "form_sums<f32>"
                          : fe == strassen::FormElem::kX3Split ? "form_sums<x3split>"
                                                               : "form_sums<16-bit>",
                          launch, (int)sums.size(), (int)(srows < 65536 ? srows : 65536), 0.0);
    return 0;
}

// Two levels: the sums of one operand on the 4 x 4 block grid, grouped for
// the launches that form them: sums whose terms lie in the same level-1
// quadrants (the operands of one level-1 product: at most seven sums over
// at most eight blocks) form one launch, which reads each block once from
// memory.
std::vector<std::vector<int>> terms_groups(const std::vector<FormedSum> &sums, int d) {
    std::vector<int> masks;
    std::vector<std::vector<int>> groups;
    for (size_t i = 0; i < sums.size(); ++i) {
        int mask = 0;
        for (int t = 0; t < sums[i].nterms; ++t) {
            const int R = sums[i].t[t].block / d, Cc = sums[i].t[t].block % d;
            mask |= 1 << ((R * 2 / d) * 2 + Cc * 2 / d);
        }
        size_t gi = 0;
        while (gi < masks.size() && masks[gi] != mask) ++gi;
        if (gi == masks.size()) {
            masks.push_back(mask);
            groups.emplace_back();
        }
        if (groups[gi].size() == (size_t)strassen::kFormTermsMaxOutputs) {  // not reached at two levels
            masks.push_back(-1);
            groups.emplace_back();
            gi = groups.size() - 1;
        }
        groups[gi].push_back((int)i);
    }
    return groups;
}

// One group of sums of operand X (block (R, Cc) at X + R*srows*ldx +
// Cc*scols, extents clipped to xr x xc) into `out` (sum i at
// i*srows*scols elements, dense, leading dimension scols).  Record: batch =
// sums, workgroups = distinct blocks read.
int form_terms_group(const std::vector<int> &group, const std::vector<FormedSum> &sums, strassen::FormElem fe,
                     size_t es, const void *X, int64_t ldx, int64_t xr, int64_t xc, int64_t srows, int64_t scols,
                     int d, char *out, bool vec, hipStream_t s, int launch) {
    strassen::FormTermsOut o[strassen::kFormTermsMaxOutputs];
    std::vector<int> blocks;
    const size_t nout = group.size();
    for (size_t j = 0; j < nout; ++j) {
        const int i = group[j];
        const FormedSum &f = sums[i];
        o[j].ptr = out + (uint64_t)i * srows * scols * es;
        o[j].n = f.nterms;
        o[j].pad = 0;
        for (int t = 0; t < f.nterms; ++t) {
            const int R = f.t[t].block / d, Cc = f.t[t].block % d;
            o[j].src[t].ptr = static_cast<const char *>(X) + ((uint64_t)R * srows * ldx + (uint64_t)Cc * scols) * es;
            o[j].src[t].rows = (int32_t)strassen::block_extent(xr, srows, R);
            o[j].src[t].cols = (int32_t)strassen::block_extent(xc, scols, Cc);
            o[j].s[t] = (float)f.t[t].sign;
            if (std::find(blocks.begin(), blocks.end(), f.t[t].block) == blocks.end())
                blocks.push_back(f.t[t].block);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool timed = false;
    int rc = record_begin(s, &e0, &e1, &timed);
    if (rc != 0) return rc;
    const hipError_t err = strassen::launch_form_terms(fe, o, (int)nout, ldx, scols, srows, scols, vec, s);
    if (err != hipSuccess) return (int)err;
    if (timed)
        return record_end(s, e0, e1,
                          fe == strassen::FormElem::kF32        ? "form_terms<f32>"
                          : fe == strassen::FormElem::kX3Split ? "form_terms<x3split>"
                                                               : "form_terms<16-bit>",
                          launch, (int)nout, (int)blocks.size(), 0.0);
    return 0;
}

// Two levels: the sum-forming launches in the order of their first use by
// the batches, on a side stream when `side` (each batch waits for the
// launches it reads), the batches in the fused schedule's order on the
// caller's stream, so the result is the fused one's.
template <class RunBatch>
int run_formed_batches_2(const Call &c, const FormedGeom &g, strassen::FormElem fe, size_t in_es, char *wa,
                         char *wb, bool vec_a, bool vec_b, bool side, int &launch, RunBatch &run_batch) {
    const Plan &plan = g.plan;
    const int d = plan.d;
    const std::vector<std::vector<int>> ga = terms_groups(g.asums, d), gb = terms_groups(g.bsums, d);
    std::vector<int> a_group(g.asums.size(), -1), b_group(g.bsums.size(), -1);
    for (size_t gi = 0; gi < ga.size(); ++gi)
        for (int i : ga[gi]) a_group[i] = (int)gi;
    for (size_t gi = 0; gi < gb.size(); ++gi)
        for (int i : gb[gi]) b_group[i] = (int)gi;
    // form launches in first-use order; per batch, the last one it reads
    std::vector<std::pair<int, int>> order;  // (operand 0 = A / 1 = B, group)
    std::vector<int> pos_a(ga.size(), -1), pos_b(gb.size(), -1), wait(plan.batches.size(), -1);
    for (size_t bi = 0; bi < plan.batches.size(); ++bi) {
        for (int pi : plan.batches[bi].products) {
            if (g.a_of[pi] >= 0) {
                int &p = pos_a[a_group[g.a_of[pi]]];
                if (p < 0) {
                    p = (int)order.size();
                    order.push_back({0, a_group[g.a_of[pi]]});
                }
                wait[bi] = std::max(wait[bi], p);
            }
            if (g.b_of[pi] >= 0) {
                int &p = pos_b[b_group[g.b_of[pi]]];
                if (p < 0) {
                    p = (int)order.size();
                    order.push_back({1, b_group[g.b_of[pi]]});
                }
                wait[bi] = std::max(wait[bi], p);
            }
        }
    }
    const Plan &pl = plan;
    auto form = [&](size_t k, hipStream_t s) {
        const int op = order[k].first, gi = order[k].second;
        return op == 0 ? form_terms_group(ga[gi], g.asums, fe, in_es, c.A, c.lda, c.m, c.k, pl.sm, pl.sk, d, wa,
                                          vec_a, s, (int)k)
                       : form_terms_group(gb[gi], g.bsums, fe, in_es, c.B, c.ldb, c.k, c.n, pl.sk, pl.sn, d, wb,
                                          vec_b, s, (int)k);
    };
    SideStream *ss = nullptr;
    if (side && order.size() <= 16) {
        const hipError_t err = side_stream(c.stream, &ss);
        if (err != hipSuccess) return (int)err;
    }
    int rc = 0;
    launch = (int)order.size();
    if (ss == nullptr) {
        for (size_t k = 0; k < order.size(); ++k)
            if ((rc = form(k, c.stream)) != 0) return rc;
        for (size_t bi = 0; bi < plan.batches.size(); ++bi)
            if ((rc = run_batch(bi)) != 0) return rc;
        return 0;
    }
    hipError_t err = hipEventRecord(ss->fork, c.stream);
    if (err == hipSuccess) err = hipStreamWaitEvent(ss->s, ss->fork, 0);
    if (err != hipSuccess) return (int)err;
    for (size_t k = 0; k < order.size(); ++k) {
        if ((rc = form(k, ss->s)) != 0) return rc;
        if ((err = hipEventRecord(ss->ready[k], ss->s)) != hipSuccess) return (int)err;
    }
    if ((err = hipEventRecord(ss->join, ss->s)) != hipSuccess) return (int)err;
    for (size_t bi = 0; bi < plan.batches.size(); ++bi) {
        if (wait[bi] >= 0 && (err = hipStreamWaitEvent(c.stream, ss->ready[wait[bi]], 0)) != hipSuccess)
            return (int)err;
        if ((rc = run_batch(bi)) != 0) return rc;
    }
    // the caller's stream waits for every sum-forming launch
    if ((err = hipStreamWaitEvent(c.stream, ss->join, 0)) != hipSuccess) return (int)err;
    return 0;
}

// side: B's form may run on a side stream (creating it on first use);
// false for callers that must not allocate.
int run_formed(const Call &c, void *ws, bool side = true) {
    if (c.m == 0 || c.n == 0) return 0;
    if (c.k == 0 || c.alpha == 0.f)
        return (int)strassen::launch_scale(c.C, c.ldc, c.m, c.n, c.beta, c.stream);
    const Family fam = family(c.a_type, c.mode);
    const FormedGeom g = formed_geom(c.m, c.n, c.k, fam, c.levels);
    const Plan &plan = g.plan;
    const int d = plan.d;
    const int64_t sm = plan.sm, sn = plan.sn, sk = plan.sk;
    const size_t in_es = elem_size(c.a_type);
    char *wa = static_cast<char *>(ws);
    char *wb = wa + g.a_bytes;
    const strassen::FormElem fe = g.pre                           ? strassen::FormElem::kX3Split
                                  : g.es == 4                     ? strassen::FormElem::kF32
                                  : c.a_type == STRASSEN_BF16 ? strassen::FormElem::kBf16
                                                              : strassen::FormElem::kF16;
    const bool vec_a = (c.lda % fam.vec == 0) && ((uintptr_t)c.A % 16 == 0);
    const bool vec_b = (c.ldb % fam.vec == 0) && ((uintptr_t)c.B % 16 == 0);
    int rc = 0;

    // Operand of product pi: its formed sum in workspace (extent: the union
    // of its terms' extents; beyond it the sum is a virtual zero) or its
    // single quadrant.
    auto operand_a = [&](int pi) {
        const strassen::Product &p = plan.products[pi];
        if (g.a_of[pi] >= 0) {
            int64_t rows = 0, cols = 0;
            for (int t = 0; t < p.na; ++t) {
                rows = std::max(rows, strassen::block_extent(c.m, sm, p.a[t].block / d));
                cols = std::max(cols, strassen::block_extent(c.k, sk, p.a[t].block % d));
            }
            return term((int64_t)g.a_of[pi] * sm * sk, rows, cols, p.a[0].sign, false);
        }
        const int R = p.a[0].block / d, Cc = p.a[0].block % d;
        return term(R * sm * c.lda + Cc * sk, strassen::block_extent(c.m, sm, R),
                    strassen::block_extent(c.k, sk, Cc), p.a[0].sign, false);
    };
    auto operand_b = [&](int pi) {
        const strassen::Product &p = plan.products[pi];
        if (g.b_of[pi] >= 0) {
            int64_t rows = 0, cols = 0;
            for (int t = 0; t < p.nb; ++t) {
                rows = std::max(rows, strassen::block_extent(c.k, sk, p.b[t].block / d));
                cols = std::max(cols, strassen::block_extent(c.n, sn, p.b[t].block % d));
            }
            return term((int64_t)g.b_of[pi] * sk * sn, rows, cols, p.b[0].sign, false);
        }
        const int R = p.b[0].block / d, Cc = p.b[0].block % d;
        return term(R * sk * c.ldb + Cc * sn, strassen::block_extent(c.k, sk, R),
                    strassen::block_extent(c.n, sn, Cc), p.b[0].sign, false);
    };

    // Chains (16-bit kernels): a batch of two-output products each of which
    // shares an output block with a distinct single-output product becomes
    // one chained launch, and those single-output products leave their own
    // batches.  Of the batches that qualify, the one with the most chains,
    // and among those one that reads B's sums anyway (the batches that read
    // B as stored run beside B's form); at one level: {M2, M3} with M5 (C3)
    // and M6 (C0).
    std::vector<int> head_of(plan.products.size(), -1);  // single-output product -> its chain head
    std::vector<int> carry_of(plan.products.size(), 0);  // chain head -> 1 + carried output
    int chained_batch = -1;
    int best_score = 0;
    if (fam.m16 && plan.levels == 1) {
        for (size_t bi = 0; bi < plan.batches.size(); ++bi) {
            const strassen::Batch &bt = plan.batches[bi];
            if (bt.wc != 2 || 2 * bt.products.size() > (size_t)strassen::kMaxBatchArgs ||
                !use_large(sm, sn, sk, (int)bt.products.size(), false))
                continue;  // chained launches use the 256x256 tile
            std::vector<int> pick(plan.products.size(), -1), carry(plan.products.size(), 0);
            std::vector<bool> taken(plan.products.size(), false);
            bool all = true;
            for (int x : bt.products) {
                bool found = false;
                for (size_t y = 0; y < plan.products.size() && !found; ++y) {
                    const strassen::Product &py = plan.products[y];
                    if (py.nc != 1 || taken[y]) continue;
                    for (int o = 0; o < plan.products[x].nc && !found; ++o)
                        if (plan.products[x].c[o].block == py.c[0].block) {
                            taken[y] = true;
                            pick[y] = x;
                            carry[x] = o + 1;
                            found = true;
                        }
                }
                all = all && found;
            }
            if (!all) continue;
            if (g.pre) {  // the chained kernel takes pre-split operands only
                bool pre_b = true;
                for (size_t q = 0; q < pick.size(); ++q)
                    if (pick[q] >= 0) pre_b = pre_b && g.b_of[q] >= 0 && g.b_of[pick[q]] >= 0;
                if (!pre_b) continue;
            }
            bool reads_b_sums = false;
            for (int x : bt.products) reads_b_sums = reads_b_sums || g.b_of[x] >= 0;
            const int score = 2 * (int)bt.products.size() + (reads_b_sums ? 1 : 0);
            if (score <= best_score) continue;
            best_score = score;
            chained_batch = (int)bi;
            head_of = pick;
            carry_of = carry;
        }
    }
    // C blocks written so far (first updates apply beta), in launch order
    bool touched[16] = {false};
    auto first_of = [&](int block) {
        const bool f = !touched[block];
        touched[block] = true;
        return f;
    };
    auto c_term = [&](const strassen::Term &t, bool first) {
        const int R = t.block / d, Cc = t.block % d;
        return term(R * sm * c.ldc + Cc * sn, strassen::block_extent(c.m, sm, R),
                    strassen::block_extent(c.n, sn, Cc), t.sign, first);
    };
    auto set_sources = [&](ProductArg &pa, int pi) {
        pa.a_base = g.a_of[pi] >= 0 ? static_cast<const void *>(wa) : c.A;
        pa.lda = g.a_of[pi] >= 0 ? sk : c.lda;
        pa.b_base = g.b_of[pi] >= 0 ? static_cast<const void *>(wb) : c.B;
        pa.ldb = g.b_of[pi] >= 0 ? sn : c.ldb;
    };

    // Products, batch by batch; a batch whose products take an operand from
    // different places is split by source.
    int launch = 2;
    auto run_batch = [&](size_t bi) -> int {
        const strassen::Batch &bt = plan.batches[bi];
        if ((int)bi == chained_batch) {
            LaunchArgs a;
            std::memset(&a, 0, sizeof(a));
            a.C = c.C;
            a.ldc = c.ldc;
            a.sm = (int32_t)sm;
            a.sn = (int32_t)sn;
            a.sk = (int32_t)sk;
            a.alpha = c.alpha;
            a.beta = c.beta;
            a.tiles_m = (int32_t)((sm + 255) / 256);
            a.tiles_n = (int32_t)((sn + 255) / 256);
            const int nchains = (int)bt.products.size();
            for (int z = 0; z < nchains; ++z) {
                const int x = bt.products[z];
                int y = -1;
                for (size_t q = 0; q < head_of.size(); ++q)
                    if (head_of[q] == x) y = (int)q;
                const strassen::Product &px = plan.products[x], &py = plan.products[y];
                ProductArg &p1 = a.prod[2 * z];
                ProductArg &p2 = a.prod[2 * z + 1];
                p1.na = p1.nb = p2.na = p2.nb = 1;
                p1.nc = px.nc;
                p2.nc = 1;
                p1.carry = carry_of[x];
                set_sources(p1, x);
                set_sources(p2, y);
                p1.a[0] = operand_a(x);
                p1.b[0] = operand_b(x);
                p2.a[0] = operand_a(y);
                p2.b[0] = operand_b(y);
                for (int o = 0; o < px.nc; ++o)
                    p1.c[o] = c_term(px.c[o], o == carry_of[x] - 1 ? false : first_of(px.c[o].block));
                p2.c[0] = c_term(py.c[0], first_of(py.c[0].block));
            }
            const bool vec = vec_a && vec_b;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            bool timed = false;
            rc = record_begin(c.stream, &e0, &e1, &timed);
            if (rc != 0) return rc;
            const hipError_t err = g.pre ? strassen::launch_m16_x3pre_chained(a, nchains, vec, c.stream)
                                         : strassen::launch_m16_chained(fam.op, a, nchains, vec, c.stream);
            if (err != hipSuccess) return (int)err;
            if (timed) {
                char name[64];
                std::snprintf(name, sizeof(name), "%s<chained,%d,%s>",
                              g.pre ? strassen::m16_x3pre_kernel_name(true, true)
                                    : strassen::m16_kernel_name(fam.op, true),
                              nchains, vec ? "vec" : "scalar");
                rc = record_end(c.stream, e0, e1, name, launch, 2 * nchains, a.tiles_m * a.tiles_n * nchains,
                                2.0 * (double)(2 * nchains) * (double)sm * (double)sn * (double)sk);
                if (rc != 0) return rc;
            }
            ++launch;
            return 0;
        }
        for (int pass = 0; pass < 4; ++pass) {
            const bool fa = (pass & 1) != 0, fb = (pass & 2) != 0;
            std::vector<int> sel;
            for (int pi : bt.products)
                if ((g.a_of[pi] >= 0) == fa && (g.b_of[pi] >= 0) == fb && head_of[pi] < 0) sel.push_back(pi);
            if (sel.empty()) continue;
            LaunchArgs a;
            std::memset(&a, 0, sizeof(a));
            a.A = fa ? static_cast<const void *>(wa) : c.A;
            a.B = fb ? static_cast<const void *>(wb) : c.B;
            a.C = c.C;
            a.lda = fa ? sk : c.lda;
            a.ldb = fb ? sn : c.ldb;
            a.ldc = c.ldc;
            a.sm = (int32_t)sm;
            a.sn = (int32_t)sn;
            a.sk = (int32_t)sk;
            a.alpha = c.alpha;
            a.beta = c.beta;
            const int batch = (int)sel.size();
            const bool large = use_large(sm, sn, sk, batch, !fam.m16);
            const strassen::KernelShape ks = shape_of(fam, large, 1, 1, bt.wc, true);
            a.tiles_m = (int32_t)((sm + ks.mt - 1) / ks.mt);
            a.tiles_n = (int32_t)((sn + ks.nt - 1) / ks.nt);
            for (int z = 0; z < batch; ++z) {
                const int pi = sel[z];
                const strassen::Product &p = plan.products[pi];
                ProductArg &pa = a.prod[z];
                pa.na = 1;
                pa.nb = 1;
                pa.nc = p.nc;
                pa.a[0] = operand_a(pi);
                pa.b[0] = operand_b(pi);
                for (int t = 0; t < p.nc; ++t) pa.c[t] = c_term(p.c[t], first_of(p.c[t].block));
            }
            const bool vec = (fa || vec_a) && (fb || vec_b);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            bool timed = false;
            rc = record_begin(c.stream, &e0, &e1, &timed);
            if (rc != 0) return rc;
            const hipError_t err =
                g.pre     ? strassen::launch_m16_x3pre(fb, large, 1, 1, bt.wc, a, batch, vec, c.stream)
                : fam.m16 ? strassen::launch_m16(fam.op, false, false, large, 1, 1, bt.wc, a, batch, vec, c.stream)
                          : strassen::launch_f32(false, false, large, 1, 1, bt.wc, a, batch, vec, c.stream);
            if (err != hipSuccess) return (int)err;
            if (timed) {
                char name[64];
                std::snprintf(name, sizeof(name), "%s<1,1,%d,%s>",
                              g.pre     ? strassen::m16_x3pre_kernel_name(fb, large)
                              : fam.m16 ? strassen::m16_kernel_name(fam.op, large)
                                        : strassen::f32_kernel_name(large),
                              bt.wc, vec ? "vec" : "scalar");
                rc = record_end(c.stream, e0, e1, name, launch, batch, a.tiles_m * a.tiles_n * batch,
                                2.0 * (double)batch * (double)sm * (double)sn * (double)sk);
                if (rc != 0) return rc;
            }
            ++launch;
        }
        return 0;
    };

    // Where chains apply, the batches whose products all take B as stored go
    // first and B's form runs on the side stream beside them (the form
    // kernel's waves fit next to the product workgroups: no LDS, few
    // registers); the caller's stream waits for it before the batches that
    // read it.  Measured at 8192^3, bf16x3: chains alone gave 0.992x the
    // plain product's rate, chains and this 1.012x (forming only the early
    // batches' A sums first and the rest beside them changed nothing more).
    std::vector<size_t> early, late;
    for (size_t bi = 0; bi < plan.batches.size(); ++bi) {
        bool b_formed = false;
        for (int pi : plan.batches[bi].products) {
            b_formed = b_formed || g.b_of[pi] >= 0;
            if (head_of[pi] >= 0) b_formed = b_formed || g.b_of[head_of[pi]] >= 0;
        }
        if ((int)bi == chained_batch)
            for (size_t q = 0; q < head_of.size(); ++q)
                if (head_of[q] >= 0) b_formed = b_formed || g.b_of[q] >= 0;
        (b_formed ? late : early).push_back(bi);
    }
    SideStream *ss = nullptr;
    // (only together with the chains: where neither applies, the launch
    // order, and so the result, is the fused schedule's)
    if (side && fam.m16 && chained_batch >= 0 && !early.empty() && !g.bsums.empty()) {
        const hipError_t err = side_stream(c.stream, &ss);
        if (err != hipSuccess) return (int)err;
    }
    if (ss != nullptr) {
        rc = form_operand(g.asums, fe, in_es, c.A, c.lda, c.m, c.k, sm, sk, wa, vec_a, c.stream, 0);
        if (rc != 0) return rc;
        hipError_t err = hipEventRecord(ss->fork, c.stream);
        if (err == hipSuccess) err = hipStreamWaitEvent(ss->s, ss->fork, 0);
        if (err != hipSuccess) return (int)err;
        rc = form_operand(g.bsums, fe, in_es, c.B, c.ldb, c.k, c.n, sk, sn, wb, vec_b, ss->s, 1);
        if (rc != 0) return rc;
        if ((err = hipEventRecord(ss->join, ss->s)) != hipSuccess) return (int)err;
        for (size_t bi : early)
            if ((rc = run_batch(bi)) != 0) return rc;
        if ((err = hipStreamWaitEvent(c.stream, ss->join, 0)) != hipSuccess) return (int)err;
        for (size_t bi : late)
            if ((rc = run_batch(bi)) != 0) return rc;
        return 0;
    }
    if (plan.levels == 2) return run_formed_batches_2(c, g, fe, in_es, wa, wb, vec_a, vec_b, side, launch, run_batch);
    rc = form_operand(g.asums, fe, in_es, c.A, c.lda, c.m, c.k, sm, sk, wa, vec_a, c.stream, 0);
    if (rc != 0) return rc;
    rc = form_operand(g.bsums, fe, in_es, c.B, c.ldb, c.k, c.n, sk, sn, wb, vec_b, c.stream, 1);
    if (rc != 0) return rc;
    for (size_t bi = 0; bi < plan.batches.size(); ++bi)
        if ((rc = run_batch(bi)) != 0) return rc;
    return 0;
}

// Maps a strassen_gemm_ex argument index to its strassen_gemm_formed position
// (levels and the transpose flags cannot be wrong there).
int to_formed_index(int code) {
    switch (-code) {
        case 7: case 11: case 16: return -1;  // not reachable
        case 8: return -7;
        case 9: return -8;
        case 10: return -9;
        case 12: return -10;
        case 13: return -11;
        case 14: return -12;
        case 15: return -13;
        case 17: return -14;
        default: return code;
    }
}

// Maps a strassen_gemm_ex argument index to its strassen_gemm position.
int to_base_index(int code) {
    switch (-code) {
        case 1: return -1;
        case 2: return -2;
        case 3: return -3;
        case 4: return -4;
        case 5: return -5;
        case 8: return -6;
        case 9: return -7;
        case 12: return -8;
        case 13: return -9;
        case 14: return -10;
        case 15: return -11;
        case 16: return -12;
        default: return code;
    }
}

const char *const kArgMessages[] = {
    "invalid argument 1",  "invalid argument 2",  "invalid argument 3",  "invalid argument 4",
    "invalid argument 5",  "invalid argument 6",  "invalid argument 7",  "invalid argument 8",
    "invalid argument 9",  "invalid argument 10", "invalid argument 11", "invalid argument 12",
    "invalid argument 13", "invalid argument 14", "invalid argument 15", "invalid argument 16",
    "invalid argument 17", "invalid argument 18",
};

}  // namespace

extern "C" {

int strassen_gemm_ex(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                     strassen_dtype_t a_type, int trans_a, const void *B, int64_t ldb,
                     strassen_dtype_t b_type, int trans_b, float *C, int64_t ldc, float alpha,
                     float beta, int levels, strassen_mode_t mode, void *hip_stream) {
    const Call c{m, n, k, A, lda, a_type, trans_a, B, ldb, b_type, trans_b, C, ldc,
                 alpha, beta, levels, mode, (hipStream_t)hip_stream};
    const int v = validate(c);
    if (v != 0) return v;
    try {
        return run(c);
    } catch (...) {
        return (int)hipErrorOutOfMemory;  // host allocation in the planner failed
    }
}

int strassen_gemm(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
                  int64_t ldb, float *C, int64_t ldc, float alpha, float beta, int levels) {
    const int r = strassen_gemm_ex(m, n, k, A, lda, STRASSEN_F32, 0, B, ldb, STRASSEN_F32, 0, C,
                                   ldc, alpha, beta, levels, STRASSEN_MODE_PLAIN, g_stream);
    return r < 0 ? to_base_index(r) : r;
}

int64_t strassen_hybrid_workspace_size(int64_t m, int64_t n, int64_t k) {
    if (m < 0 || m >= kMaxDim) return -1;
    if (n < 0 || n >= kMaxDim) return -2;
    if (k < 0 || k >= kMaxDim) return -3;
    try {
        const HybridGeom g = hybrid_geom(m, n, k);
        return (g.p_elems + g.q_elems) * (int64_t)sizeof(float);
    } catch (...) {
        return -(int64_t)hipErrorOutOfMemory;
    }
}

int strassen_gemm_hybrid(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                         const float *B, int64_t ldb, float *C, int64_t ldc, float alpha,
                         float beta, void *workspace, int64_t workspace_bytes, void *hip_stream) {
    const Call c{m, n, k, A, lda, STRASSEN_F32, 0, B, ldb, STRASSEN_F32, 0, C, ldc,
                 alpha, beta, 2, STRASSEN_MODE_PLAIN, (hipStream_t)hip_stream};
    const int v = validate(c);
    if (v != 0) return to_base_index(v);
    const bool product = m > 0 && n > 0 && k > 0 && alpha != 0.f;
    if (!product) {
        try {
            return run_hybrid(c, nullptr);
        } catch (...) {
            return (int)hipErrorOutOfMemory;
        }
    }
    const int64_t need = strassen_hybrid_workspace_size(m, n, k);
    if (need < 0) return (int)(-need);
    if (workspace == nullptr || (uintptr_t)workspace % 16 != 0) return -12;
    if (workspace_bytes < need) return -13;
    const uint64_t wb = (uint64_t)need;
    if (overlap(workspace, wb, A, span_bytes(m, k, lda, 4)) ||
        overlap(workspace, wb, B, span_bytes(k, n, ldb, 4)) ||
        overlap(workspace, wb, C, span_bytes(m, n, ldc, 4)))
        return -12;
    try {
        return run_hybrid(c, static_cast<float *>(workspace));
    } catch (...) {
        return (int)hipErrorOutOfMemory;
    }
}

}  // extern "C" (reopened below)

namespace {

// Workspace bytes of a formed call, or a negative code: -1 m, -2 n, -3 k,
// -4 levels, -5 dtype, -6 mode.
int64_t formed_size(int64_t m, int64_t n, int64_t k, int levels, strassen_dtype_t dtype,
                    strassen_mode_t mode) {
    if (m < 0 || m >= kMaxDim) return -1;
    if (n < 0 || n >= kMaxDim) return -2;
    if (k < 0 || k >= kMaxDim) return -3;
    if (levels < 0 || levels > 2) return -4;
    if (!valid_dtype(dtype)) return -5;
    if (mode != STRASSEN_MODE_PLAIN && mode != STRASSEN_MODE_BF16X3) return -6;
    if (mode == STRASSEN_MODE_BF16X3 && dtype != STRASSEN_F32) return -6;
    try {
        return formed_geom(m, n, k, family(dtype, mode), levels).bytes;
    } catch (...) {
        return -(int64_t)hipErrorOutOfMemory;
    }
}

// Maps a strassen_gemm_ex argument index to its strassen_gemm_formed_ex
// position (the transpose flags cannot be wrong there).
int to_formed_ex_index(int code) {
    switch (-code) {
        case 7: case 11: return -1;  // not reachable
        case 8: return -7;
        case 9: return -8;
        case 10: return -9;
        case 12: return -10;
        case 13: return -11;
        case 14: return -12;
        case 15: return -13;
        case 16: return -14;
        case 17: return -15;
        default: return code;
    }
}

int formed_call(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, strassen_dtype_t a_type,
                const void *B, int64_t ldb, strassen_dtype_t b_type, float *C, int64_t ldc, float alpha,
                float beta, int levels, strassen_mode_t mode, void *workspace, int64_t workspace_bytes,
                void *hip_stream) {
    const Call c{m, n, k, A, lda, a_type, 0, B, ldb, b_type, 0, C, ldc,
                 alpha, beta, levels, mode, (hipStream_t)hip_stream};
    const int v = validate(c);
    if (v != 0) return to_formed_ex_index(v);
    if (levels < 0 || levels > 2) return -14;
    const bool product = m > 0 && n > 0 && k > 0 && alpha != 0.f;
    try {
        if (!product) return run_formed(c, nullptr);
        const int64_t need = formed_size(m, n, k, levels, a_type, mode);
        if (need < 0) return (int)(-need);
        if (need == 0) return run_formed(c, nullptr);  // level 0 on stored operands: nothing to form
        if (workspace == nullptr || (uintptr_t)workspace % 16 != 0) return -16;
        if (workspace_bytes < need) return -17;
        const uint64_t wbytes = (uint64_t)need;
        const size_t es = elem_size(a_type);
        if (overlap(workspace, wbytes, A, span_bytes(m, k, lda, es)) ||
            overlap(workspace, wbytes, B, span_bytes(k, n, ldb, es)) ||
            overlap(workspace, wbytes, C, span_bytes(m, n, ldc, 4)))
            return -16;
        return run_formed(c, workspace);
    } catch (...) {
        return (int)hipErrorOutOfMemory;
    }
}

}  // namespace

extern "C" {

int64_t strassen_formed_workspace_size_ex(int64_t m, int64_t n, int64_t k, int levels, strassen_dtype_t dtype,
                                          strassen_mode_t mode) {
    return formed_size(m, n, k, levels, dtype, mode);
}

int64_t strassen_formed_workspace_size(int64_t m, int64_t n, int64_t k, strassen_dtype_t dtype,
                                       strassen_mode_t mode) {
    const int64_t r = formed_size(m, n, k, 1, dtype, mode);
    return r == -5 ? -4 : r == -6 ? -5 : r;
}

int strassen_gemm_formed_ex(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                            strassen_dtype_t a_type, const void *B, int64_t ldb, strassen_dtype_t b_type,
                            float *C, int64_t ldc, float alpha, float beta, int levels, strassen_mode_t mode,
                            void *workspace, int64_t workspace_bytes, void *hip_stream) {
    return formed_call(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta, levels, mode, workspace,
                       workspace_bytes, hip_stream);
}

int strassen_gemm_formed(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                         strassen_dtype_t a_type, const void *B, int64_t ldb, strassen_dtype_t b_type,
                         float *C, int64_t ldc, float alpha, float beta, strassen_mode_t mode,
                         void *workspace, int64_t workspace_bytes, void *hip_stream) {
    // the _ex positions from levels on are one further
    const int r = formed_call(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta, 1, mode, workspace,
                              workspace_bytes, hip_stream);
    return r <= -15 ? r + 1 : r;
}

static_assert(strassen::kNoAllocScratchBytes == STRASSEN_NOALLOC_SCRATCH_BYTES,
              "scratch size in the header and the library agree");

int strassen_gemm_formed_noalloc(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                                 strassen_dtype_t a_type, const void *B, int64_t ldb,
                                 strassen_dtype_t b_type, float *C, int64_t ldc, float alpha,
                                 float beta, strassen_mode_t mode, void *hip_stream) {
    const Call c{m, n, k, A, lda, a_type, 0, B, ldb, b_type, 0, C, ldc,
                 alpha, beta, 1, mode, (hipStream_t)hip_stream};
    const int v = validate(c);
    if (v != 0) return to_formed_index(v);
    const bool product = m > 0 && n > 0 && k > 0 && alpha != 0.f;
    try {
        if (!product) return run_formed(c, nullptr);
        const int64_t need = formed_size(m, n, k, 1, a_type, mode);
        if (need < 0) return (int)(-need);
        if (need > strassen::kNoAllocScratchBytes) return STRASSEN_ERROR_SCRATCH_LIMIT;
        void *scratch = nullptr;
        const hipError_t err = strassen::noalloc_scratch(c.stream, &scratch);
        if (err != hipSuccess) return (int)err;
        return run_formed(c, scratch, false);
    } catch (...) {
        return (int)hipErrorOutOfMemory;
    }
}

int strassen_set_stream(void *hip_stream) {
    g_stream = (hipStream_t)hip_stream;
    return 0;
}

int strassen_set_schedule(int schedule) {
    if (schedule != STRASSEN_SCHEDULE_BATCHED && schedule != STRASSEN_SCHEDULE_CONCURRENT &&
        schedule != STRASSEN_SCHEDULE_STREAMS)
        return -1;
    g_schedule = schedule;
    return 0;
}

int strassen_set_tile(int tile) {
    if (tile != STRASSEN_TILE_AUTO && tile != STRASSEN_TILE_128 && tile != STRASSEN_TILE_256)
        return -1;
    g_tile = tile;
    return 0;
}

int strassen_plan_info(int64_t m, int64_t n, int64_t k, int levels, strassen_dtype_t dtype,
                       strassen_mode_t mode, strassen_plan_info_t *out) {
    if (m < 0 || m >= kMaxDim) return -1;
    if (n < 0 || n >= kMaxDim) return -2;
    if (k < 0 || k >= kMaxDim) return -3;
    if (levels < 0 || levels > STRASSEN_MAX_LEVELS) return -4;
    if (!valid_dtype(dtype)) return -5;
    if (mode != STRASSEN_MODE_PLAIN && mode != STRASSEN_MODE_BF16X3) return -6;
    if (mode == STRASSEN_MODE_BF16X3 && dtype != STRASSEN_F32) return -6;
    if (out == nullptr) return -7;
    try {
        const Family fam = family(dtype, mode);
        const Plan p = strassen::make_plan(m, n, k, levels, fam.vec);
        // tile of the launch with the most operand terms
        const strassen::Batch *wide = &p.batches[0];
        for (const strassen::Batch &b : p.batches)
            if (b.wa + b.wb > wide->wa + wide->wb) wide = &b;
        const bool large = use_large(p.sm, p.sn, p.sk, (int)wide->products.size(), !fam.m16);
        const strassen::KernelShape ks = shape_of(fam, large, wide->wa, wide->wb, wide->wc, true);
        std::memset(out, 0, sizeof(*out));
        out->levels = levels;
        out->blocks_per_dim = p.d;
        out->sub_m = p.sm;
        out->sub_n = p.sn;
        out->sub_k = p.sk;
        out->n_instances = (int32_t)p.products.size();
        out->n_launches = (int32_t)p.batches.size();
        out->tile_m = ks.mt;
        out->tile_n = ks.nt;
        out->tile_k = ks.kt;
        out->workgroups_per_instance =
            (int32_t)(((p.sm + ks.mt - 1) / ks.mt) * ((p.sn + ks.nt - 1) / ks.nt));
        out->executed_flops = p.executed_flops;
        out->classical_flops = 2.0 * (double)m * (double)n * (double)k;
    } catch (...) {
        return (int)hipErrorOutOfMemory;
    }
    return 0;
}

int strassen_plan_instances(int levels, strassen_instance_t *out, int capacity) {
    if (levels < 0 || levels > STRASSEN_MAX_LEVELS) return -1;
    if (out == nullptr && capacity > 0) return -2;
    if (capacity < 0) return -3;
    try {
        // Block assignment does not depend on the matrix sizes.
        const Plan p = strassen::make_plan(1 << levels, 1 << levels, 1 << levels, levels, 1);
        int idx = 0;
        for (size_t bi = 0; bi < p.batches.size(); ++bi)
            for (int pi : p.batches[bi].products) {
                if (idx < capacity) {
                    const strassen::Product &q = p.products[pi];
                    strassen_instance_t &o = out[idx];
                    std::memset(&o, 0, sizeof(o));
                    o.launch = (int32_t)bi;
                    o.n_a = q.na;
                    o.n_b = q.nb;
                    o.n_c = q.nc;
                    for (int t = 0; t < q.na; ++t) {
                        o.a_block[t] = q.a[t].block;
                        o.a_sign[t] = q.a[t].sign;
                    }
                    for (int t = 0; t < q.nb; ++t) {
                        o.b_block[t] = q.b[t].block;
                        o.b_sign[t] = q.b[t].sign;
                    }
                    for (int t = 0; t < q.nc; ++t) {
                        o.c_block[t] = q.c[t].block;
                        o.c_sign[t] = q.c[t].sign;
                        o.c_first[t] = q.c_first[t] ? 1 : 0;
                    }
                }
                ++idx;
            }
        return idx;
    } catch (...) {
        return (int)hipErrorOutOfMemory;
    }
}

#ifndef STRASSEN_BUILD_ID
#define STRASSEN_BUILD_ID "unknown"
#endif

const char *strassen_build_id(void) { return STRASSEN_BUILD_ID; }

const char *strassen_error_string(int code) {
    if (code == 0) return "success";
    if (code == STRASSEN_ERROR_SCRATCH_LIMIT)
        return "the call needs more workspace than the no-allocation entry point's fixed scratch holds";
    if (code < 0) {
        const int i = -code;
        if (i >= 1 && i <= (int)(sizeof(kArgMessages) / sizeof(kArgMessages[0])))
            return kArgMessages[i - 1];
        return "invalid argument";
    }
    const char *s = hipGetErrorString((hipError_t)code);
    return s ? s : "HIP runtime error";
}

int strassen_profile_start(void) {
    Recorder &r = recorder();
    std::lock_guard<std::mutex> lk(r.mu);
    for (Record &x : r.recs) {
        r.pool.push_back(x.e0);
        r.pool.push_back(x.e1);
    }
    r.recs.clear();
    r.total = 0;
    r.on = true;
    return 0;
}

int strassen_probe_mfma(int op, int random, int64_t iters, int32_t workgroups, float *out, void *hip_stream) {
    if (op < 0 || op > 2) return -1;
    if (random != 0 && random != 1) return -2;
    if (iters < 0) return -3;
    if (workgroups < 1) return -4;
    if (out == nullptr) return -5;
    return (int)strassen::launch_mfma_probe(op, random, iters, workgroups, out, (hipStream_t)hip_stream);
}

int strassen_profile_stop(strassen_launch_record_t *out, int capacity) {
    if (out == nullptr && capacity > 0) return -1;
    if (capacity < 0) return -2;
    Recorder &r = recorder();
    std::lock_guard<std::mutex> lk(r.mu);
    r.on = false;
    int idx = 0;
    for (Record &x : r.recs) {
        hipError_t err = hipEventSynchronize(x.e1);
        if (err != hipSuccess) return (int)err;
        float ms = 0.f;
        err = hipEventElapsedTime(&ms, x.e0, x.e1);
        if (err != hipSuccess) return (int)err;
        x.info.ms = ms;
        if (idx < capacity) out[idx] = x.info;
        ++idx;
    }
    for (Record &x : r.recs) {
        r.pool.push_back(x.e0);
        r.pool.push_back(x.e1);
    }
    r.recs.clear();
    const int total = r.total;
    r.total = 0;
    return total;
}

}  // extern "C"
