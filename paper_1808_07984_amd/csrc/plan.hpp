// Host-side planner: which Strassen products exist at a given number of
// levels, how the d x d block partition maps onto the matrices, and in which
// race-free batches the products are launched.  Pure C++, no HIP headers, so
// it is testable on a machine without a GPU.
#pragma once

#include <cstdint>
#include <vector>

namespace strassen {

constexpr int kMaxLevels = 2;
constexpr int kMaxTerms = 4;   // operands per matrix at two levels
constexpr int kMaxBatch = 8;   // largest variant count at two levels

struct Term {
    int block;  // row-major index in the d x d block partition
    int sign;   // +1 or -1
};

// One product M = (sum_t sa_t A_{a_t}) (sum_t sb_t B_{b_t});
//             C_{c_o} += sc_o * M  (eq. straprim1, generalised to <= 4 terms).
struct Product {
    int na = 0, nb = 0, nc = 0;
    Term a[kMaxTerms], b[kMaxTerms], c[kMaxTerms];
    bool c_first[kMaxTerms] = {false, false, false, false};
};

struct Batch {
    int wa, wb, wc;              // variant: operand counts shared by the batch
    std::vector<int> products;   // indices into Plan::products, C-disjoint
};

struct Plan {
    int levels = 0;
    int d = 1;                   // blocks per dimension, 2^levels
    int64_t m = 0, n = 0, k = 0;
    int64_t sm = 0, sn = 0, sk = 0;  // block extents (virtual padding)
    std::vector<Product> products;   // in launch order
    std::vector<Batch> batches;
    double executed_flops = 0;
};

// Products of `levels` levels: the levels-fold Kronecker power of the
// one-level scheme, in a fixed canonical order (before batching).
std::vector<Product> scheme(int levels);

// Full plan.  `vec` is the vector width in elements that block offsets along
// n and k (and m when round_m is set: A stored transposed) are rounded to when
// levels >= 1, so vector loads stay aligned.
Plan make_plan(int64_t m, int64_t n, int64_t k, int levels, int vec, bool round_m = false);

// Stream-by-stage schedule of the seven one-level products (Task Parallelism
// section, table "tab:gpu_streaming"): products of one stage run at once on
// streams 0 and 1, products on one stream in the listed order, and every
// stage waits for the previous one on both streams.  Entries are indices
// into scheme(1) (M0..M6), in launch order.
struct StreamSlot {
    int product;
    int stage;
    int stream;
};
std::vector<StreamSlot> stream_stages();

// Rows (or columns) of block index `b` (0 <= b < d) that lie inside a
// dimension of size `dim` when blocks have extent `s`:  clamp(dim - b*s, 0, s).
inline int64_t block_extent(int64_t dim, int64_t s, int b) {
    int64_t r = dim - (int64_t)b * s;
    if (r < 0) r = 0;
    if (r > s) r = s;
    return r;
}

}  // namespace strassen
