// LDS layout of a chunk of prior draws (Formula 5's Delta^(k)) staged for the
// gradient kernel: every point of the workgroup reads the same draws.
#pragma once
#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {

// LDS layout of a chunk of C draws:
//   FP64:  tau[C][6]
//   T:     b0[C] b1[C] PR[C] mu1[C] Bt[C][K][d]
template <typename T>
struct ChunkView {
    double* tau;
    T *b0, *b1, *PR, *mu1, *Bt;
};

template <typename T>
__host__ __device__ inline size_t chunk_bytes(int C, int d, int K) {
    return sizeof(double) * static_cast<size_t>(C) * kMaxDim + sizeof(T) * static_cast<size_t>(C) * (4 + static_cast<size_t>(d) * K);
}

template <typename T>
__device__ inline ChunkView<T> carve_chunk(char* base, int C, int K) {
    (void)K;
    ChunkView<T> v;
    double* dp = reinterpret_cast<double*>(base);
    v.tau = dp; dp += C * kMaxDim;
    T* tp = reinterpret_cast<T*>(dp);
    v.b0 = tp; tp += C;
    v.b1 = tp; tp += C;
    v.PR = tp; tp += C;
    v.mu1 = tp; tp += C;
    v.Bt = tp;
    return v;
}

}  // namespace bmd
