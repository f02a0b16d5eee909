// Device helpers for the deterministic reductions of the pixel-domain kernels.
//
// Every vector kernel runs on a fixed grid per problem (at most kVecBlocks blocks of
// kVecThreads, sized by the problem alone) with a grid-stride loop, so each partial sum
// covers a fixed set of elements in a fixed order; partials are combined by a fixed tree.  A kernel that needs a
// reduced scalar re-reduces the partials in its prologue (every block the same
// way), which yields bitwise identical scalars in all blocks without an extra
// launch.
#pragma once

#include "mm_internal.h"

namespace mm {

// block sum of v (one value per thread; blockDim.x a multiple of 64, at most 1024): wave
// shuffle trees, then the per-wave sums in wave order; the same in every block, returned to
// all threads.  All threads must call.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    __syncthreads();  // red may be reused at once
    return r;
}

// sum of nb partials, identical in every block; all threads must call
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int nb,
                                                  double* red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    return block_sum(s, red);
}

// block sum of v written to part[blockIdx.x]
__device__ __forceinline__ void write_partial(double v, double* __restrict__ part, double* red) {
    const double r = block_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// block sum of v written to part[k] (k: the block's index within its problem)
__device__ __forceinline__ void write_partial_at(double v, double* __restrict__ part, int k,
                                                 double* red) {
    const double r = block_sum(v, red);
    if (threadIdx.x == 0) part[k] = r;
}

// slots of the partial buffer
constexpr int kSlotPQ = 0, kSlotRR = 1, kSlotRZ = 2, kSlotAux = 3, kNumSlots = 4;

// problem b of block g given the block offsets off[0..B] (off[0] = 0, non-decreasing):
// the largest b with off[b] <= g
__device__ __forceinline__ int block_problem(const int32_t* __restrict__ off, int B, int g) {
    int a = 0, b = B - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (off[m] <= g) a = m; else b = m - 1;
    }
    return a;
}

// the partials of problem b in a slot
__device__ __forceinline__ double* slot_part(const PcgCtl& c, int slot, int b) {
    return c.part + ((int64_t)slot * c.B + b) * kVecBlocks;
}

// a block's place in a per-problem vector launch
struct VecBlock {
    int b;          // problem
    int k;          // block index within the problem
    int64_t base;   // first element (or pixel) of the problem
    int64_t n;      // elements (or pixels) of the problem
    int64_t stride; // grid stride of the problem's loop: its block count x kVecThreads
};

// elements == true: n_s entries per pixel; false: pixels
__device__ __forceinline__ VecBlock vec_block(const PcgCtl& c, int ns, bool elements) {
    VecBlock v;
    const int32_t* off = elements ? c.eblk : c.pblk;
    v.b = block_problem(off, c.B, blockIdx.x);
    v.k = blockIdx.x - off[v.b];
    v.stride = (int64_t)(off[v.b + 1] - off[v.b]) * kVecThreads;
    const int64_t o0 = c.ooff[v.b], o1 = c.ooff[v.b + 1];
    const int64_t m = elements ? ns : 1;
    v.base = o0 * m;
    v.n = (o1 - o0) * m;
    return v;
}

}  // namespace mm
