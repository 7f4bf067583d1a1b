// In-kernel regeneration of prior draws (Formula 5's Delta^(k)) into LDS,
// chunk by chunk, from their Philox counters: the same arithmetic as the draw
// kernel of the grid sweep (FP64, rounded once to the integrand type T), shared
// by every design of the workgroup.
#pragma once
#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {

// LDS layout of a chunk of C draws:
//   FP64:  b0d[C] b1d[C] tau[C][6] t[C][6] prod[C][K]
//   int32: thr[C][6]
//   T:     b0[C] b1[C] PR[C] mu1[C] tauT[C] e1[C] e2[C] Bt[C][d][K]
template <typename T>
struct ChunkView {
    double *b0d, *b1d, *tau, *t, *prod;
    int32_t* thr;
    T *b0, *b1, *PR, *mu1, *tauT, *e1, *e2, *Bt;
};

template <typename T>
__host__ __device__ inline size_t chunk_bytes(int C, int d, int K) {
    return sizeof(double) * static_cast<size_t>(C) * (2 + 2 * kMaxDim + K) + sizeof(int32_t) * C * kMaxDim +
           sizeof(T) * static_cast<size_t>(C) * (7 + static_cast<size_t>(d) * K);
}

template <typename T>
__device__ inline ChunkView<T> carve_chunk(char* base, int C, int K) {
    ChunkView<T> v;
    double* dp = reinterpret_cast<double*>(base);
    v.b0d = dp; dp += C;
    v.b1d = dp; dp += C;
    v.tau = dp; dp += C * kMaxDim;
    v.t = dp; dp += C * kMaxDim;
    v.prod = dp; dp += static_cast<size_t>(C) * K;
    int32_t* ip = reinterpret_cast<int32_t*>(dp);
    v.thr = ip; ip += C * kMaxDim;
    T* tp = reinterpret_cast<T*>(ip);
    v.b0 = tp; tp += C;
    v.b1 = tp; tp += C;
    v.PR = tp; tp += C;
    v.mu1 = tp; tp += C;
    v.tauT = tp; tp += C;
    v.e1 = tp; tp += C;
    v.e2 = tp; tp += C;
    v.Bt = tp;
    return v;
}

// Number of grid indices i in [0, m_j) with q_{j,i} <= tau (nondecreasing grid).
__device__ __forceinline__ int32_t grid_count_le(const DevProblem& P, int j, double tau) {
    int lo = 0, hi = P.m[j];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (grid_coord(P.q_lo, P.q_hi, mid, P.m[j]) <= tau) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Draws k0 .. k0+nk-1 into the chunk; every thread of the block must call it.
// gh: FP64 Gauss-Hermite rule x[K], w[K].  Grid thresholds are filled when the
// problem has a grid.  Ends with the chunk visible to the whole block.
template <typename T, int D>
__device__ void regenerate_chunk(const DevProblem& P, const double* __restrict__ gh, int K, const ChunkView<T>& c,
                                 int64_t k0, int nk) {
    __syncthreads();   // previous chunk fully consumed
    if (threadIdx.x < nk) {
        const int i = threadIdx.x;
        double u[8];
        draw_uniforms<8>(static_cast<uint64_t>(k0 + i), P.scenario, P.key0, P.key1, P.n_uniform, u);
        if (P.effect == BMD_EFFECT_STEP) {
            const double b0 = P.mu_b0 + P.sd_b0 * norm_quantile(u[0]);
            const double b1 = P.mu_b1 + P.sd_b1 * norm_quantile(u[1]);
            c.b0d[i] = b0;
            c.b1d[i] = b1;
            c.b0[i] = static_cast<T>(b0);
            c.b1[i] = static_cast<T>(b1);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double tau = affine_uniform(P.tau_lo, P.tau_hi, u[2 + j]);
                c.tau[i * kMaxDim + j] = tau;
                c.t[i * kMaxDim + j] = norm_quantile(tau);
                c.thr[i * kMaxDim + j] = P.G > 0 ? grid_count_le(P, j, tau) : 0;
            }
            c.tauT[i] = static_cast<T>(c.tau[i * kMaxDim]);
            if (D == 1) {
                const double PR = 1.0 - c.tau[i * kMaxDim];
                c.PR[i] = static_cast<T>(PR);
                c.mu1[i] = static_cast<T>(P.sqrtI * (b0 + b1 * PR));
            }
        } else {
            const double e1 = norm_quantile(u[0]);
            const double e2 = norm_quantile(u[1]);
            c.e1[i] = static_cast<T>(e1);
            c.e2[i] = static_cast<T>(e2);
            c.mu1[i] = static_cast<T>(P.sqrtI * (P.th1 + P.sg1 * e1));
        }
    }
    if constexpr (D >= 2) {
        if (P.effect == BMD_EFFECT_STEP) {
            __syncthreads();
            for (int e = threadIdx.x; e < nk * K; e += blockDim.x) {
                const int i = e / K, m = e % K;
                const double s = P.sr * gh[m];
                double prod = gh[K + m];
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double v = norm_cdf((s - c.t[i * kMaxDim + j]) / P.sq);
                    c.Bt[(static_cast<size_t>(i) * D + j) * K + m] = static_cast<T>(j == 0 ? gh[K + m] * v : v);
                    prod *= v;
                }
                c.prod[static_cast<size_t>(i) * K + m] = prod;
            }
            __syncthreads();
            if (threadIdx.x < nk) {
                const int i = threadIdx.x;
                double PR = 0.0;
                for (int m = 0; m < K; ++m) PR += c.prod[static_cast<size_t>(i) * K + m];
                c.PR[i] = static_cast<T>(PR);
                c.mu1[i] = static_cast<T>(P.sqrtI * (c.b0d[i] + c.b1d[i] * PR));
            }
        }
    }
    __syncthreads();
}

}  // namespace bmd
