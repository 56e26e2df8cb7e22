// Deterministic block reduction of kRedSlots doubles per thread.
//
// Every block reduces its threads' values with a fixed LDS tree and writes
// one row of the partials array; launch_finalize then reduces the rows in a
// fixed order.  No atomics: results are bitwise reproducible for a given
// problem size.
#pragma once

#include "common.hpp"

namespace mlbm {

// Reduces acc[0..kRedSlots) over the block (kRedThreads threads, 1-D) into
// out_row.  Bit s of MAXMASK selects max for slot s, otherwise sum.
template <unsigned MAXMASK>
__device__ __forceinline__ void block_reduce_store(double (&acc)[kRedSlots], double* out_row) {
    __shared__ double sh[kRedSlots][kRedThreads];
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) sh[s][t] = acc[s];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int s = 0; s < kRedSlots; ++s) {
                const double o = sh[s][t + w];
                sh[s][t] = ((MAXMASK >> s) & 1u) ? fmax(sh[s][t], o) : sh[s][t] + o;
            }
        }
        __syncthreads();
    }
    if (t < kRedSlots) out_row[t] = sh[t][0];
}

}  // namespace mlbm
