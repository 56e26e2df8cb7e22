// Workgroup-to-cell mapping shared by the row-blocked kernels (the step
// passes and the channel-parallel adjoint).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace mlbm {

// Block order.  The grid is one-dimensional and the hardware hands block b to
// XCD b mod 8 (round robin); each XCD has its own L2.  Blocks that cover
// neighbouring x-chunks of one row read the same boundary cache lines (the
// x-shifted pulls).  Three bijections of [0, gridDim.x) onto (chunk, row):
//   kOrderNatural     chunk fastest, rows in order;
//   kOrderXcdRange    every XCD runs one contiguous range of logical blocks,
//                     so the chunks of a row share an L2;
//   kOrderInterleave8 8 consecutive rows go to the 8 XCDs and the chunks of a
//                     row follow 8 blocks apart on the same XCD; rows are
//                     still swept in order across the chip.
// Which is fastest depends on the grid (measured on MI355X; see step_launch).
__device__ __forceinline__ void block_order(int order, int nx, int ny, int bx, int& chunk, int& y, int& z) {
    constexpr unsigned kXcd = 8;
    const unsigned b = blockIdx.x, G = gridDim.x;
    const unsigned nchunk = (static_cast<unsigned>(nx) + bx - 1) / bx;
    unsigned row, ch;
    if (order == kOrderInterleave8) {
        const unsigned grp = kXcd * nchunk, g = b / grp, t = b % grp;
        if (g < G / grp) {
            ch = t / kXcd;
            row = g * kXcd + t % kXcd;
        } else {          // last, partial group of rows: natural order
            ch = t % nchunk;
            row = g * kXcd + t / nchunk;
        }
    } else {
        unsigned L = b;
        if (order == kOrderXcdRange) {
            const unsigned q = G / kXcd, r = G % kXcd, j = b % kXcd;
            L = j * q + (j < r ? j : r) + b / kXcd;
        }
        row = L / nchunk;
        ch = L - row * nchunk;
    }
    chunk = static_cast<int>(ch);
    y = static_cast<int>(row % static_cast<unsigned>(ny));
    z = static_cast<int>(row / static_cast<unsigned>(ny));
}

}  // namespace mlbm
