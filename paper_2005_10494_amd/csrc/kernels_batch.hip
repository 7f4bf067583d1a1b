// Many independent grid problems in one persistent launch.
//
// Work item = (scenario, tile of 256 designs, slice of draws).  Workgroups pull
// items from a device counter until the list is exhausted (every workgroup
// reaches the exit), regenerate the slice's draws chunk by chunk in LDS from
// their Philox counters, and write one FP64 partial sum per design and slice.
// The last item of a scenario stamps its completion time.  A finalize kernel
// reduces the slices in fixed order, so results do not depend on scheduling.
#include <climits>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "draw_chunk.hpp"
#include "eval_core.hpp"

namespace bmd {

namespace {

template <typename T, int D, int NMAX>
__device__ void batch_item(const BatchScenario& S, int tile, int slice, char* lds, const BatchArgs& a) {
    const DevProblem& P = S.P;
    const int64_t G = P.G;
    const int64_t g = static_cast<int64_t>(tile) * kEvalBlock + threadIdx.x;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;
    DesignState<T, D, NMAX> s;
    s.init(P, gg, S.r, S.z1, S.z2, a.gl, static_cast<const T*>(S.glw));
    const ChunkView<T> c = carve_chunk<T>(lds, a.chunk, S.K);
    const ChunkDraws<T> src{c, D, S.K};
    const T* A = static_cast<const T*>(S.A);
    const int64_t kb = static_cast<int64_t>(slice) * S.slice_len;
    const int64_t ke = min(S.M, kb + S.slice_len);
    double s1 = 0.0;
    for (int64_t k0 = kb; k0 < ke; k0 += a.chunk) {
        const int nk = static_cast<int>(min<int64_t>(a.chunk, ke - k0));
        regenerate_chunk<T, D>(P, S.gh, S.K, c, k0, nk);
        for (int i = 0; i < nk; ++i) s1 += static_cast<double>(summand<T, D, NMAX>(P, s, src, i, A, S.K));
    }
    if (valid) S.partials[static_cast<int64_t>(slice) * G + g] = s1;
}

// Work loop.  Thread 0 does all of its global bookkeeping in ONE guarded block
// at the top of the iteration (retire the previous item, claim the next), and
// the claimed index is broadcast through LDS and made wave-uniform, so the
// loop exit is a scalar branch.  Two separate thread-0 blocks (claim at the
// top, retire at the bottom) let the compiler thread them together across the
// back edge into a loop nest in which lane 0 waits outside an inner loop that
// the rest of its wave can only leave after lane 0 claims new work: a deadlock
// under SIMT execution.
template <typename T, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int s_item;
    int prev_sc = -1;   // scenario of the item this workgroup finished last (thread 0)
    if (threadIdx.x == 0) atomicMin(a.t_start, static_cast<unsigned long long>(wall_clock64()));
    for (;;) {
        if (threadIdx.x == 0) {
            if (prev_sc >= 0) {
                __threadfence();
                if (atomicSub(&a.left[prev_sc], 1) == 1)
                    a.t_done[prev_sc] = static_cast<unsigned long long>(wall_clock64());
            }
            s_item = atomicAdd(a.counter, 1);
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= a.n_items) break;
        const int4 it = a.items[item];
        const int sc = __builtin_amdgcn_readfirstlane(it.x);
        const int tile = __builtin_amdgcn_readfirstlane(it.y);
        const int slice = __builtin_amdgcn_readfirstlane(it.z);
        const BatchScenario& S = a.sc[sc];
        switch (__builtin_amdgcn_readfirstlane(S.P.d)) {
            case 1: batch_item<T, 1, NMAX>(S, tile, slice, lds, a); break;
            case 2: batch_item<T, 2, NMAX>(S, tile, slice, lds, a); break;
            case 3: batch_item<T, 3, NMAX>(S, tile, slice, lds, a); break;
            case 4: batch_item<T, 4, NMAX>(S, tile, slice, lds, a); break;
            case 5: batch_item<T, 5, NMAX>(S, tile, slice, lds, a); break;
            default: batch_item<T, 6, NMAX>(S, tile, slice, lds, a); break;
        }
        prev_sc = sc;
        __syncthreads();   // item done by every thread; s_item free for the next claim
    }
}

// Counters for one launch (a kernel, so the sequence can live in a graph).
__global__ void k_batch_reset(BatchArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        *a.counter = 0;
        *a.t_start = ULLONG_MAX;
    }
    if (s < a.n_sc) {
        a.left[s] = a.sc[s].n_items;
        a.t_done[s] = 0;
    }
}

__global__ void k_batch_finalize(BatchArgs a) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= a.G_total) return;
    int lo = 0, hi = a.n_sc - 1;   // last scenario with g_offset <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.sc[mid].g_offset <= t) lo = mid; else hi = mid - 1;
    }
    const BatchScenario& S = a.sc[lo];
    const int64_t g = t - S.g_offset;
    double s = 0.0;
    for (int sl = 0; sl < S.n_slices; ++sl) s += S.partials[static_cast<int64_t>(sl) * S.P.G + g];
    S.mean[g] = s / static_cast<double>(S.M);
}

}  // namespace

size_t batch_lds_bytes(int prec, int chunk, int K) {
    return prec == BMD_FP64 ? chunk_bytes<double>(chunk, kMaxDim, K) : chunk_bytes<float>(chunk, kMaxDim, K);
}

int batch_blocks_per_cu(int prec, size_t lds) {
    int nb = 0;
    hipError_t e = prec == BMD_FP64
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<double, 24>, kEvalBlock, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<float, 12>, kEvalBlock, lds);
    if (e != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_batch(int prec, const BatchArgs& a, int grid, size_t lds, bool reset, bool finalize,
                        hipStream_t s) {
    if (reset) {
        hipLaunchKernelGGL(k_batch_reset, dim3((a.n_sc + 255) / 256), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (prec == BMD_FP64)
        hipLaunchKernelGGL((k_batch<double, 24>), dim3(grid), dim3(kEvalBlock), lds, s, a);
    else
        hipLaunchKernelGGL((k_batch<float, 12>), dim3(grid), dim3(kEvalBlock), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !finalize) return e;
    hipLaunchKernelGGL(k_batch_finalize, dim3(static_cast<unsigned>((a.G_total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace bmd
