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

// 16-byte loads through a buffer resource: the base lives in scalar
// registers and each lane supplies a 32-bit byte offset, so a load costs no
// 64-bit address registers.  The record count is 2^32 - 1: no range
// clamping; callers keep every offset (plus 16) below 2^32.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, 0x00020000);
}
template <class V>
__device__ __forceinline__ V buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    static_assert(sizeof(V) == 16, "16-byte vectors");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
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
