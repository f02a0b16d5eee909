// Device helpers for the deterministic reductions of the pixel-domain kernels.
//
// Every vector kernel runs on a fixed grid (kVecBlocks x kVecThreads) with a
// grid-stride loop, so each partial sum covers a fixed set of elements in a
// fixed order; partials are combined by a fixed tree.  A kernel that needs a
// reduced scalar re-reduces the partials in its prologue (every block the same
// way), which yields bitwise identical scalars in all blocks without an extra
// launch.
#pragma once

#include "mm_internal.h"

namespace mm {

// sum of nb partials, identical in every block; all threads must call
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int nb,
                                                  double* red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// block tree sum of v (one value per thread) written to part[blockIdx.x]
__device__ __forceinline__ void write_partial(double v, double* __restrict__ part, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// slots of the partial buffer
constexpr int kSlotPQ = 0, kSlotRR = 1, kSlotRZ = 2, kSlotAux = 3, kNumSlots = 4;

}  // namespace mm
