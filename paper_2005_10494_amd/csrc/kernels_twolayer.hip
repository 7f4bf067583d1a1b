// The paper's two-layer sampling estimator of the expected power (Formula 7,
// with the inner layer of Formula 6): N1 outer draws Delta^(k) from the prior,
// N2 inner draws x^(l) of the null statistics (Formula 1), and
//   P = 1 - (1 / (N1 N2)) sum_k sum_l [x^(l)_j <= z_j - sqrt(r_j I) Delta^(k)_j for all j],
// the same inner draws serving every outer draw.  The comparisons are counted in
// A x B blocks (outer-draw groups x inner-draw groups), from which the
// finalize forms the estimate and an unbiased estimate of its variance.
//
// Inner draws: n standard normals e'_1..e'_n per l from the Philox stream whose
// fourth counter word has its top bit set, chained into the nested null
// correlations of Appendix A.1: x_1 = e'_1,
// x_{i+1} = sqrt(r_{i+1}/r_i) x_i + sqrt(1 - r_{i+1}/r_i) e'_{i+1}.
#include <cstdint>

#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {
namespace {

constexpr int kTwoBlock = 256;   // threads per workgroup (and outer draws per LDS chunk)
constexpr int kTwoR = 4;         // inner draws per lane
constexpr uint32_t kInnerStream = 0x80000000u;

// Uniform i (< 4) of inner draw l: Philox counter (l lo, l hi, scenario, top bit | block).
__device__ __forceinline__ double inner_uniform(uint64_t l, const DevProblem& P, int i) {
    const uint4 o = philox4x32_10(make_uint4(static_cast<uint32_t>(l), static_cast<uint32_t>(l >> 32), P.scenario,
                                             kInnerStream | static_cast<uint32_t>(i / 2)),
                                  P.key0, P.key1);
    return (i & 1) ? uniform52(o.z, o.w) : uniform52(o.x, o.y);
}

// e[j * N2 + l] = Phi^-1(u_j(l)), j < n.
__global__ void k_inner_draws(DevProblem P, int n, int64_t N2, double* __restrict__ e) {
    const int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= N2) return;
    for (int j = 0; j < n; ++j) e[j * N2 + l] = norm_quantile(inner_uniform(static_cast<uint64_t>(l), P, j));
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

struct TwoLayerArgs {
    DevProblem P;
    int n;                      // nested populations
    const double* r;            // [G] second fraction (cutoff and two-population alpha designs)
    const double* z[4];         // [G] critical values
    const double* e[4];         // outer draws' normals, FP64 [N1]
    const double* ei;           // inner draws' normals [n][N2]
    int64_t N1, N2;
    int A, B;                   // outer and inner groups
    uint32_t* blocks;           // [G][A][B]
};

// Fractions r_1..r_n of design g (r_1 = 1).
__device__ __forceinline__ void design_fractions(const TwoLayerArgs& a, int64_t g, double* r) {
    r[0] = 1.0;
    r[1] = a.n == 2 ? a.r[g] : a.P.r_lo;
    r[2] = a.P.r_hi;
    r[3] = a.P.r_4;
}

// One workgroup: design blockIdx.x and 1,024 inner draws; wavefront w's lane
// holds the four draws blockIdx.y * 1024 + w * 256 + 64 i + lane (i < 4), so
// a wavefront's draws are contiguous and lie in one inner group.  The outer
// draws' thresholds b_kj = z_j - mu_j^(k) go through LDS in chunks of 256 (one
// per thread) and each read serves the lane's four inner draws (one read per
// comparison would exceed the LDS bandwidth).  Each lane counts, over the
// outer draws of the current group, how often its inner draws stay below the
// thresholds in every coordinate, and at the end of each outer group the
// wavefront's counts go to the design's block (outer group, inner group of the
// wavefront) by one atomic add.  T is the comparison type (FP64, or FP32 with
// both sides rounded).
template <typename T, int N>
__global__ __launch_bounds__(kTwoBlock) void k_two_layer(TwoLayerArgs a) {
    // thresholds of a chunk, each draw's padded to 2 or 4 values so that one
    // vector LDS read fetches them
    constexpr int NP = N == 2 ? 2 : 4;
    __shared__ __align__(16) T sb[kTwoBlock * NP];
    const int64_t g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    double r[4], z[N];
    design_fractions(a, g, r);
    bool skip = false;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        z[j] = a.z[j][g];
        skip = skip || z[j] != z[j];   // no valid level split: the finalize writes NaN
    }
    if (skip) return;
    // Formula 10 means mu_i = sqrt(r_i I) (theta_i + sigma_i Y_i), Y the chain of
    // the outer normals: mu_i = m0_i + sum_{j<=i} mc[i][j] e_j.
    double m0[N], mc[N][N], ch[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double th = -log1p(-(a.P.paper_a - a.P.paper_b * r[i]));
        const double sc = sqrt(r[i] * a.P.info) / sqrt(a.P.paper_events * r[i] / 4.0);
        m0[i] = sqrt(r[i] * a.P.info) * th;
#pragma unroll
        for (int j = 0; j < N; ++j) ch[i][j] = 0.0;
        if (i == 0) {
            ch[0][0] = 1.0;
        } else {
            const double f = sqrt(r[i] / r[i - 1]);
#pragma unroll
            for (int j = 0; j < N; ++j) ch[i][j] = j < i ? f * ch[i - 1][j] : 0.0;
            ch[i][i] = sqrt(1.0 - r[i] / r[i - 1]);
        }
#pragma unroll
        for (int j = 0; j < N; ++j) mc[i][j] = sc * ch[i][j];
    }
    // this lane's inner draws, the same chain of their own normals
    const int64_t l0 = static_cast<int64_t>(blockIdx.y) * (kTwoBlock * kTwoR) + (tid >> 6) * (64 * kTwoR) + lane;
    T x[kTwoR][N];
#pragma unroll
    for (int q = 0; q < kTwoR; ++q) {
        double xd[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double ei = a.ei[i * a.N2 + l0 + 64 * q];
            xd[i] = i == 0 ? ei : sqrt(r[i] / r[i - 1]) * xd[i - 1] + sqrt(1.0 - r[i] / r[i - 1]) * ei;
            x[q][i] = static_cast<T>(xd[i]);
        }
    }
    const int64_t SA = a.N1 / a.A;
    const int bgrp = static_cast<int>(l0 / (a.N2 / a.B));
    uint32_t* blk = a.blocks + (g * a.A) * a.B + bgrp;
    uint32_t cnt = 0;
    for (int64_t k0 = 0; k0 < a.N1; k0 += kTwoBlock) {
        const int nk = static_cast<int>(min<int64_t>(kTwoBlock, a.N1 - k0));
        __syncthreads();   // the previous chunk's thresholds are no longer read
        if (tid < nk) {
            double e[N];
#pragma unroll
            for (int j = 0; j < N; ++j) e[j] = a.e[j][k0 + tid];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double mu = m0[i];
#pragma unroll
                for (int j = 0; j <= i; ++j) mu += mc[i][j] * e[j];
                sb[tid * NP + i] = static_cast<T>(z[i] - mu);
            }
        }
        __syncthreads();
        int kk = 0;
        while (kk < nk) {
            // the outer draws of this chunk up to the end of the current group
            const int64_t k = k0 + kk;
            const int end = static_cast<int>(min<int64_t>(nk, (k / SA + 1) * SA - k0));
            // every coordinate compared, the results combined without branches;
            // two outer draws at a time so that their LDS reads are in flight together
            for (; kk + 2 <= end; kk += 2) {
                T bk[2][NP];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int j = 0; j < NP; ++j) bk[u][j] = sb[(kk + u) * NP + j];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int q = 0; q < kTwoR; ++q) {
                        uint32_t in = 1u;
#pragma unroll
                        for (int j = 0; j < N; ++j) in &= static_cast<uint32_t>(x[q][j] <= bk[u][j]);
                        cnt += in;
                    }
            }
            for (; kk < end; ++kk) {
#pragma unroll
                for (int q = 0; q < kTwoR; ++q) {
                    uint32_t in = 1u;
#pragma unroll
                    for (int j = 0; j < N; ++j) in &= static_cast<uint32_t>(x[q][j] <= sb[kk * NP + j]);
                    cnt += in;
                }
            }
            if ((k0 + kk) % SA == 0) {   // group done: add the wavefront's counts to its block
                uint32_t s = cnt;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
                if (lane == 0) atomicAdd(blk + ((k0 + kk) / SA - 1) * a.B, s);
                cnt = 0;
            }
        }
    }
}

// One workgroup of 64 threads per design: estimate 1 - T / (N1 N2) from the
// block counts and, with block means m_ab, row and column means R_a, C_b and
// grand mean M, the two-way crossed random-effects estimate of its variance
//   (MS_A + MS_B - MS_E) / (A B),
//   MS_A = B sum_a (R_a - M)^2 / (A - 1),  MS_B = A sum_b (C_b - M)^2 / (B - 1),
//   MS_E = sum_ab (m_ab - R_a - C_b + M)^2 / ((A - 1)(B - 1)),
// unbiased for the estimate's variance (the Hoeffding parts of the indicator
// are uncorrelated, so the block means follow that model).  Designs without a
// valid level split get NaN.
__global__ __launch_bounds__(64) void k_two_layer_final(TwoLayerArgs a, double* __restrict__ mean,
                                                        double* __restrict__ var) {
    __shared__ double sR[64], sC[64], sE[64];
    const int64_t g = blockIdx.x;
    const int t = threadIdx.x;
    bool skip = false;
    for (int j = 0; j < a.n; ++j) skip = skip || a.z[j][g] != a.z[j][g];
    if (skip) {
        if (t == 0) {
            mean[g] = NAN;
            if (var) var[g] = NAN;
        }
        return;
    }
    const int A = a.A, B = a.B;
    const uint32_t* n = a.blocks + g * A * B;
    const double cell = static_cast<double>(a.N1 / A) * static_cast<double>(a.N2 / B);
    if (t < A) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += n[t * B + b] / cell;
        sR[t] = s / B;
    }
    if (t < B) {
        double s = 0.0;
        for (int i = 0; i < A; ++i) s += n[i * B + t] / cell;
        sC[t] = s / A;
    }
    __syncthreads();
    double M = 0.0;
    uint64_t T = 0;
    for (int i = 0; i < A; ++i) {
        M += sR[i];
        for (int b = 0; b < B; ++b) T += n[i * B + b];
    }
    M /= A;
    if (t < A) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) {
            const double d = n[t * B + b] / cell - sR[t] - sC[b] + M;
            s += d * d;
        }
        sE[t] = s;
    }
    __syncthreads();
    if (t == 0) {
        mean[g] = 1.0 - static_cast<double>(T) / (static_cast<double>(a.N1) * static_cast<double>(a.N2));
        if (var) {
            double sa = 0.0, sc = 0.0, se = 0.0;
            for (int i = 0; i < A; ++i) sa += (sR[i] - M) * (sR[i] - M);
            for (int b = 0; b < B; ++b) sc += (sC[b] - M) * (sC[b] - M);
            for (int i = 0; i < A; ++i) se += sE[i];
            const double msa = B * sa / (A - 1), msb = A * sc / (B - 1), mse = se / ((A - 1) * (B - 1));
            var[g] = (msa + msb - mse) / (static_cast<double>(A) * B);
        }
    }
}

template <typename T>
hipError_t launch_counts(const TwoLayerArgs& a, int64_t G, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(G), static_cast<unsigned>(a.N2 / (kTwoBlock * kTwoR)));
    switch (a.n) {
        case 2: hipLaunchKernelGGL((k_two_layer<T, 2>), grid, dim3(kTwoBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_two_layer<T, 3>), grid, dim3(kTwoBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_two_layer<T, 4>), grid, dim3(kTwoBlock), 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t two_layer_inner_bytes(int n, int64_t N2) { return sizeof(double) * static_cast<size_t>(n) * N2; }

hipError_t launch_two_layer(const bmd_problem* p, int prec, int n, int64_t N1, int64_t N2, int A, int B,
                            const DrawArrays<double>& outer, double* inner, uint32_t* blocks, double* mean,
                            double* var, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_inner_draws, dim3(static_cast<unsigned>((N2 + 255) / 256)), dim3(256), 0, s, p->P, n, N2,
                       inner);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = G * A * B;
    hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>((nb + 255) / 256)), dim3(256), 0, s, blocks, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    TwoLayerArgs a{};
    a.P = p->P;
    a.n = n;
    a.r = p->d_r;
    a.z[0] = p->d_z1;
    a.z[1] = p->d_z2;
    a.z[2] = p->d_z3 ? p->d_z3 : p->d_z2;
    a.z[3] = p->d_z4 ? p->d_z4 : p->d_z2;
    a.e[0] = outer.e1;
    a.e[1] = outer.e2;
    a.e[2] = outer.e3;
    a.e[3] = outer.e4;
    a.ei = inner;
    a.N1 = N1;
    a.N2 = N2;
    a.A = A;
    a.B = B;
    a.blocks = blocks;
    e = prec == BMD_FP64 ? launch_counts<double>(a, G, s) : launch_counts<float>(a, G, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_two_layer_final, dim3(static_cast<unsigned>(G)), dim3(64), 0, s, a, mean, var);
    return hipGetLastError();
}

}  // namespace bmd
