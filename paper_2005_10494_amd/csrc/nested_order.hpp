// Launch order for the sweeps whose designs have their own integration rule
// (nested populations cut from one biomarker): the sweep runs every lane of
// a wavefront at the wavefront's largest rule, so designs go to the sweep
// sorted by cost, largest first, those that do not exist last.
#pragma once
#include "bmd_internal.hpp"

namespace bmd {

// Largest value of v over the wavefront, in a scalar register.
__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

// Stable counting sort of designs 0..G-1 by key(g) in [0, NBINS) into order
// (one workgroup of 1024 threads): bin counts by LDS atomics and their
// exclusive scan into bin starts; then, tile by tile of 1,024 designs, each
// wavefront's count per bin, each lane's rank among the lanes of its
// wavefront with the same key (by 63 shuffles), and per bin the wavefronts'
// starts in turn.  Ties keep index order.
template <int NBINS, typename Key>
__device__ void order_by_key(int64_t G, Key key, int32_t* __restrict__ order) {
    __shared__ int start[NBINS];
    __shared__ int wstart[16][NBINS];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    for (int b = t; b < NBINS; b += 1024) start[b] = 0;
    __syncthreads();
    for (int64_t g = t; g < G; g += 1024) atomicAdd(&start[key(g)], 1);
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int b = 0; b < NBINS; ++b) {
            const int c = start[b];
            start[b] = run;
            run += c;
        }
    }
    for (int64_t g0 = 0; g0 < G; g0 += 1024) {
        for (int b = t; b < 16 * NBINS; b += 1024) (&wstart[0][0])[b] = 0;
        __syncthreads();   // also orders the scan above and the previous tile's reads before these writes
        const int64_t g = g0 + t;
        const int k = g < G ? key(g) : -1;
        if (k >= 0) atomicAdd(&wstart[wave][k], 1);
        int rank = 0;
        for (int j = 0; j < 64; ++j) {
            const int kj = __shfl(k, j);
            rank += (j < lane && kj == k) ? 1 : 0;
        }
        __syncthreads();
        for (int b = t; b < NBINS; b += 1024) {
            int run = start[b];
            for (int w = 0; w < 16; ++w) {
                const int c = wstart[w][b];
                wstart[w][b] = run;
                run += c;
            }
            start[b] = run;
        }
        __syncthreads();
        if (k >= 0) order[wstart[wave][k] + rank] = static_cast<int32_t>(g);
        __syncthreads();
    }
}

}  // namespace bmd
