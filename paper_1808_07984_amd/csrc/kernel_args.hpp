// Plain-data kernel arguments shared by the host launcher and the device
// kernels.  One launch runs a batch of up to kMaxBatchArgs Strassen products
// of one variant; blockIdx.z selects the product.
#pragma once

#include <cstdint>

namespace strassen {

constexpr int kMaxBatchArgs = 8;

// One operand block: element (r, c) of the block (block-local coordinates)
// lives at base[off + r * ld + c] and is inside the matrix iff r < rows and
// c < cols; outside it is a virtual zero (inputs) or not stored (outputs).
struct TermArg {
    int64_t off;
    int32_t rows;
    int32_t cols;
    float sign;    // +1 or -1
    int32_t first; // outputs only: 1 = first update of this C block (applies beta)
};

struct ProductArg {
    TermArg a[4];
    TermArg b[4];
    TermArg c[4];
    // Operand sources of this product when set (16-bit kernels): its A terms
    // index a_base with leading dimension lda, its B terms b_base with ldb;
    // null: LaunchArgs::A / lda (B / ldb).
    const void *a_base;
    const void *b_base;
    int64_t lda, ldb;
    int32_t na, nb, nc;  // terms in use (kernels compiled for a variant use all)
    int32_t carry;       // chained launches: 1 + the output this product leaves in the
                         // accumulator for the next product of its chain; 0 = none
};

struct LaunchArgs {
    const void *A;
    const void *B;
    float *C;
    int64_t lda, ldb, ldc;
    int32_t sm, sn, sk;        // block extents (rows of A/C, cols of B/C, inner)
    int32_t tiles_m, tiles_n;  // workgroup tiles covering one block
    float alpha, beta;
    int32_t trans_a, trans_b;  // 1: A (B) is stored transposed
    ProductArg prod[kMaxBatchArgs];
};

}  // namespace strassen
