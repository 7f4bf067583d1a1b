// Device-side numerics for the design-objective kernels (gfx950).
//
// The FP64 normal CDF and quantile come from the device math library (ocml:
// erfc, normcdfinv); the FP32 normal CDF is a fitted tail form (see
// norm_cdf(float)); the bivariate normal CDF is evaluated from Plackett's identity
// d Phi_2 / d rho = phi_2 integrated over the angle theta = asin(rho)
// (Drezner & Wesolowsky 1990, as organised by Genz 2004, Stat. Comput. 14:251),
// with a Gauss-Legendre rule whose node count grows with the correlation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "normal_cdf_fit.hpp"

namespace bmd {

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC 2011).
// Round: multiply words 0 and 2 by fixed constants, xor the high halves into
// words 1 and 3 with the key; the key advances by two Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (n + 1/2) * 2^-52 with n the 52-bit integer made of the top 26 bits of each
// word; exact in FP64, strictly inside (0, 1).
__device__ __forceinline__ double uniform52(uint32_t wa, uint32_t wb) {
#pragma clang fp contract(off)
    const uint64_t n = (static_cast<uint64_t>(wa >> 6) << 26) | static_cast<uint64_t>(wb >> 6);
    const double t = static_cast<double>(n) + 0.5;
    return t * 0x1p-52;
}

// Fill u[0..nu) for draw k: block b uses counter (k lo, k hi, scenario, b).
template <int NU>
__device__ __forceinline__ void draw_uniforms(uint64_t k, uint32_t scenario, uint32_t key0,
                                              uint32_t key1, int nu, double* u) {
    uint32_t w[2 * NU + 4];
#pragma unroll
    for (int b = 0; b < (2 * NU + 3) / 4; ++b) {
        if (4 * b < 2 * nu) {
            const uint4 o = philox4x32_10(
                make_uint4(static_cast<uint32_t>(k), static_cast<uint32_t>(k >> 32), scenario,
                           static_cast<uint32_t>(b)),
                key0, key1);
            w[4 * b + 0] = o.x;
            w[4 * b + 1] = o.y;
            w[4 * b + 2] = o.z;
            w[4 * b + 3] = o.w;
        }
    }
#pragma unroll
    for (int i = 0; i < NU; ++i)
        if (i < nu) u[i] = uniform52(w[2 * i], w[2 * i + 1]);
}

// Grid coordinate q_lo + ((q_hi - q_lo) * i) / (m - 1), each step rounded
// (no fused multiply-add: the value must be bit-identical to a plain IEEE
// evaluation in this order).
__device__ __forceinline__ double grid_coord(double q_lo, double q_hi, int64_t i, int m) {
#pragma clang fp contract(off)
    const double span = q_hi - q_lo;
    const double t = (span * static_cast<double>(i)) / static_cast<double>(m - 1);
    return q_lo + t;
}

// lo + (hi - lo) * u, each step rounded (no fused multiply-add).
__device__ __forceinline__ double affine_uniform(double lo, double hi, double u) {
#pragma clang fp contract(off)
    const double span = hi - lo;
    const double x = span * u;
    return lo + x;
}

// ---------------------------------------------------------------------------
// Univariate normal
// ---------------------------------------------------------------------------
__device__ __forceinline__ double norm_cdf(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }
// Single precision, argument prescaled: for xs = x sqrt(log2(e)/2) and
// y = |xs|, Phi(-|x|) = r' 2^(P(r') - y^2) with r' = 1/(y + 2 sqrt(log2 e))
// (the hardware reciprocal, within one ulp) and P the degree-7 fit of
// normal_cdf_fit.hpp in r' itself (tail relative error within 3e-6 while the
// tail exceeds 1e-9, max abs error of Phi 5.6e-7, unbiased), signed as
// 1/2 + copysign(1/2 - Phi(-|x|), x).  One reciprocal, one exp2 and twelve
// full-rate operations.  Callers that can fold the factor into constants they
// already hold pass xs directly.  xs must be finite: beyond |x| = 14.8 the
// exponent underflows and Phi saturates to 0 or 1.
__device__ __forceinline__ float norm_cdf_scaled(float xs) {
    const float r = __builtin_amdgcn_rcpf(fabsf(xs) + kPhiShift);
    float p = kPhiFit[kPhiFitDeg];
#pragma unroll
    for (int i = kPhiFitDeg - 1; i >= 0; --i) p = fmaf(p, r, kPhiFit[i]);
    const float t = fmaf(-r, __builtin_amdgcn_exp2f(fmaf(-xs, xs, p)), 0.5f);   // 1/2 - Phi(-|x|)
    return 0.5f + __builtin_copysignf(t, xs);
}
__device__ __forceinline__ float norm_cdf(float x) { return norm_cdf_scaled(x * kPhiScale); }
__device__ __forceinline__ double norm_pdf(double x) { return 0.39894228040143267794 * exp(-0.5 * x * x); }
__device__ __forceinline__ float norm_pdf(float x) {
    return 0.39894228040143267794f * __builtin_amdgcn_exp2f(-0.72134752044448170368f * x * x);
}

// Phi^-1(p): the library quantile, then one Newton step on a residual that
// keeps relative accuracy (erf form near 1/2, where p - 1/2 is exact; erfc
// forms in the tails, where p or 1 - p is exact).
__device__ __forceinline__ double norm_quantile(double p) {
    const double x = p <= 0.5 ? normcdfinv(p) : -normcdfinv(1.0 - p);
    const double a = p - 0.5;
    double res;
    if (fabs(a) <= 0.25) res = 0.5 * erf(x * 0.70710678118654752440) - a;
    else if (a < 0.0) res = 0.5 * erfc(-x * 0.70710678118654752440) - p;
    else res = (1.0 - p) - 0.5 * erfc(x * 0.70710678118654752440);
    return x - res / norm_pdf(x);
}

// ---------------------------------------------------------------------------
// Bivariate normal CDF with per-design constants.
//
// Phi_2(h,k;rho) = Phi(h) Phi(k) + (1/2pi) int_0^{asin rho}
//                      exp(-(h^2 + k^2 - 2 h k sin t) / (2 cos^2 t)) dt.
// With Gauss-Legendre nodes x_i on [-1,1], s_i = sin(asin(rho)(1 + x_i)/2):
//   integrand_i = exp(b_i h k - a_i (h^2 + k^2)),  a_i = 1/(2 (1 - s_i^2)), b_i = 2 s_i a_i,
// and the integral is asin(rho)/(4 pi) sum_i w_i integrand_i.
// The per-design constants (a_i, b_i, scale) live in registers; the weights w_i
// belong to the n-point rule shared by the wavefront.
// ---------------------------------------------------------------------------

// Number of Gauss-Legendre nodes for a target accuracy at correlation rho:
// max abs error of the integral <= 1e-14 for FP64 (h, k in [-6, 4]) and
// <= 2e-8 for FP32 (h, k in [-8, 5]), up to rho = 0.975.
__device__ __forceinline__ int bvn_nodes_fp64(double rho) {
    return rho < 0.3 ? 6 : rho < 0.5 ? 8 : rho < 0.75 ? 12 : rho < 0.9 ? 16 : rho < 0.95 ? 20 : 24;
}
__device__ __forceinline__ int bvn_nodes_fp32(double rho) {
    return rho < 0.58 ? 4 : rho < 0.8 ? 6 : rho < 0.91 ? 8 : rho < 0.95 ? 10 : 12;
}

// Offsets of the n-point rules inside the packed Gauss-Legendre table
// (rules for n = 4, 6, 8, 10, 12, 16, 20, 24; x then w, n doubles each).
__device__ __forceinline__ int gl_offset(int n) {
    // 2 * (sum of smaller rule sizes)
    return n == 4 ? 0 : n == 6 ? 8 : n == 8 ? 20 : n == 10 ? 36 : n == 12 ? 56
         : n == 16 ? 80 : n == 20 ? 112 : 152;
}

template <typename T, int NMAX>
struct BvnConst {
    T a[NMAX], b[NMAX];
    T scale;  // asin(rho) / (4 pi)

    // gl: packed table; n: wave-uniform rule size (<= NMAX).  FP32 evaluates
    // exp2 on arguments prescaled by sqrt(log2(e)/2) (norm_cdf_scaled's), so
    // its exponent coefficients become 1/(1 - s^2) and 2 s/(1 - s^2).
    __device__ __forceinline__ void init(double rho, int n, const double* __restrict__ gl) {
        const double th = asin(rho);
        scale = static_cast<T>(th * 0.079577471545947667884);  // 1/(4 pi)
        const double* x = gl + gl_offset(n);
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i < n) {
                const double s = sin(0.5 * th * (1.0 + x[i]));
                const double ai = 1.0 / ((1.0 - s) * (1.0 + s));
                a[i] = static_cast<T>(sizeof(T) == 4 ? ai : 0.5 * ai);
                b[i] = static_cast<T>(sizeof(T) == 4 ? 2.0 * s * ai : s * ai);
            } else {
                a[i] = T(0);
                b[i] = T(0);
            }
        }
    }
};

// Node sum  sum_{i<n} w_i exp(b_i hk - a_i hs)  (FP32: exp2 of prescaled
// arguments, log2(e) folded into a_i, b_i).  Every rule size is even and n is
// wave-uniform, so the nodes go in pairs behind a scalar exit test, unrolled by template
// recursion: only n nodes are evaluated and every coefficient index is a
// compile-time constant (registers, no indexed scratch).  (A guard per node in
// a loop is if-converted into evaluating all NMAX exponentials; a loop with an
// early exit is kept rolled for FP64, its coefficients then indexed in scratch.)
__device__ __forceinline__ double node_exp(double x) { return exp(x); }
__device__ __forceinline__ float node_exp(float x) { return __builtin_amdgcn_exp2f(x); }

template <int I, typename T, int NMAX, typename W>
__device__ __forceinline__ void bvn_node_pairs(int n, T hk, T hs, const BvnConst<T, NMAX>& c, const W& w, T& acc0,
                                               T& acc1) {
    // smallest rule: 4 nodes (FP32 table) or 6 (FP64 table); those need no test
    constexpr int kMinRule = sizeof(T) == 4 ? 4 : 6;
    if constexpr (I < NMAX) {
        if (I >= kMinRule && I >= n) return;
        acc0 = fma(w[I], node_exp(c.b[I] * hk - c.a[I] * hs), acc0);
        acc1 = fma(w[I + 1], node_exp(c.b[I + 1] * hk - c.a[I + 1] * hs), acc1);
        bvn_node_pairs<I + 2>(n, hk, hs, c, w, acc0, acc1);
    }
}

template <typename T, int NMAX, typename W>
__device__ __forceinline__ T bvn_node_sum(int n, T hk, T hs, const BvnConst<T, NMAX>& c, const W& w) {
    T acc0 = T(0), acc1 = T(0);
    bvn_node_pairs<0>(n, hk, hs, c, w, acc0, acc1);
    return acc0 + acc1;
}

// FP64: Phi(h) Phi(k) + asin(rho)/(4 pi) sum_i w_i exp(b_i hk - a_i hs), hs = h^2 + k^2
template <int NMAX>
__device__ __forceinline__ double bvn_cdf(double h, double k, const BvnConst<double, NMAX>& c,
                                          const double* __restrict__ w, int n) {
    const double hk = h * k, hs = fma(h, h, k * k);
    return norm_cdf(h) * norm_cdf(k) + c.scale * bvn_node_sum(n, hk, hs, c, w);
}

// FP32: the same with exp2.  The weights are wave-uniform (one rule per
// wavefront); BvnWeights holds them in scalar registers, read once per design.
template <int NMAX>
struct BvnWeights {
    float w[NMAX];
    __device__ __forceinline__ void load(const float* __restrict__ src, int n) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
            w[i] = i < n ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(src[i]))) : 0.0f;
    }
    __device__ __forceinline__ float operator[](int i) const { return w[i]; }
};

// Arguments prescaled by sqrt(log2(e)/2) (kPhiScale), as norm_cdf_scaled.
template <int NMAX, typename W>
__device__ __forceinline__ float bvn_cdf_scaled(float h, float k, const BvnConst<float, NMAX>& c, const W& w, int n) {
    const float hk = h * k, hs = fmaf(h, h, k * k);
    return fmaf(norm_cdf_scaled(h), norm_cdf_scaled(k), c.scale * bvn_node_sum(n, hk, hs, c, w));
}
template <int NMAX, typename W>
__device__ __forceinline__ float bvn_cdf(float h, float k, const BvnConst<float, NMAX>& c, const W& w, int n) {
    return bvn_cdf_scaled(h * kPhiScale, k * kPhiScale, c, w, n);
}

// Upper complement 1 - Phi_2(h, k; rho) = (1 - scale S) - Phi(h) Phi(k), S the
// node sum: two fused multiply-adds.
template <int NMAX>
__device__ __forceinline__ double bvn_sf(double h, double k, const BvnConst<double, NMAX>& c,
                                         const double* __restrict__ w, int n) {
    const double hk = h * k, hs = fma(h, h, k * k);
    return fma(-norm_cdf(h), norm_cdf(k), fma(-c.scale, bvn_node_sum(n, hk, hs, c, w), 1.0));
}
template <int NMAX, typename W>
__device__ __forceinline__ float bvn_sf_scaled(float h, float k, const BvnConst<float, NMAX>& c, const W& w, int n) {
    const float hk = h * k, hs = fmaf(h, h, k * k);
    return fmaf(-norm_cdf_scaled(h), norm_cdf_scaled(k), fmaf(-c.scale, bvn_node_sum(n, hk, hs, c, w), 1.0f));
}
template <int NMAX, typename W>
__device__ __forceinline__ float bvn_sf(float h, float k, const BvnConst<float, NMAX>& c, const W& w, int n) {
    return bvn_sf_scaled(h * kPhiScale, k * kPhiScale, c, w, n);
}

// Row of the 16x16 result held in accumulator element v of a lane in quarter
// kq = lane / 16 (the column is lane % 16).  Operands: lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  The FP32 16x16x4 instruction gives each quarter four
// consecutive rows; the FP64 one interleaves them with stride 4.
template <typename T>
__device__ __forceinline__ int mfma16_row(int kq, int v) {
    return sizeof(T) == 8 ? kq + 4 * v : 4 * kq + v;
}

}  // namespace bmd
