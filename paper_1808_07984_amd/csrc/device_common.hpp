// Device helpers shared by the product kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernel_args.hpp"

namespace strassen {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Maps blockIdx.x to a (tile_m, tile_n) pair of one output block.
//
// Workgroups are handed to the 8 XCDs round-robin by id; each XCD has its own
// L2.  The id is first renumbered so every XCD receives one contiguous range
// of tiles, then tiles are walked in groups of GROUP tile-rows so that
// neighbouring workgroups share rows of A and columns of B.
template <int GROUP>
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int &tm, int &tn) {
    const int nt = tiles_m * tiles_n;
    int bid = blockIdx.x;
    const int xcd = bid & 7, local = bid >> 3;
    const int q = nt >> 3, r = nt & 7;
    bid = xcd * q + (xcd < r ? xcd : r) + local;
    const int per_group = GROUP * tiles_n;
    const int g = bid / per_group;
    const int m0 = g * GROUP;
    const int gs = (tiles_m - m0) < GROUP ? (tiles_m - m0) : GROUP;
    const int in = bid - g * per_group;
    tm = m0 + in % gs;
    tn = in / gs;
}

// Smallest extent over the first n terms (scalar, uniform).
__device__ __forceinline__ void min_extent(const TermArg *t, int n, int &rows, int &cols) {
    rows = t[0].rows;
    cols = t[0].cols;
    for (int i = 1; i < n; ++i) {
        rows = t[i].rows < rows ? t[i].rows : rows;
        cols = t[i].cols < cols ? t[i].cols : cols;
    }
}

}  // namespace strassen
