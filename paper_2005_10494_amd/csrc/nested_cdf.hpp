// Normal CDFs of nested populations (Sec. 2.2 with the null correlations of
// Appendix A.1: corr(Z_i, Z_j) = sqrt(r_j / r_i) for fractions r_i > r_j).
// Each population's statistic is the scaled sum over its members, so the
// statistics form a chain: given one of them, those before it are
// independent of those after it.  The CDFs below condition on the second
// statistic and integrate over it with a panel Gauss-Legendre rule.
//
// Three populations:  given Y2 = y the other two are independent normals
// with means r12 y, r23 y and sds s12 = sqrt(1 - r2), s23 = sqrt(1 - r3/r2):
//   Phi_3(h1, h2, h3) = int_{-inf}^{h2} phi(y) Phi((h1 - r12 y)/s12) Phi((h3 - r23 y)/s23) dy,
// a one-dimensional integral of univariate CDFs only.  It runs over [-L, U],
// U = min(h2, L, the y beyond which either conditional argument falls below
// -L), with L = 8.5 in FP64 (Phi(-8.5) < 1e-17) and 6 in FP32 (Phi(-6) = 1e-9),
// cut into equal panels of an 8-point Gauss-Legendre rule.  The integrand's
// steepest part is the conditional CDF whose scale in y, l = s12 / r12 or
// s23 / r23, is smaller; the panel count is ceil(c / l) with c = 6 (8..128
// panels) in FP64 and c = 2.5 (3..64) in FP32.  Against an adaptive reference
// over 0.1 <= r2 <= 0.9 and r3 / r2 up to 0.99 this keeps the quadrature error
// below 5e-12 (FP64) and 6.2e-8 (FP32: an order below the FP32 Phi's own
// 5.6e-7, which the 1e-5 objective bar already budgets for); the critical
// values use at least 16 panels.
//
// Four populations: given Y2 = y, Y1 is independent of (Y3, Y4), which are
// bivariate normal with means r23 y, r24 y, sds s23, s24 = sqrt(1 - r4/r2)
// and the partial correlation rho = (r34 - r23 r24) / (s23 s24):
//   Phi_4(h) = int_{-inf}^{h2} phi(y) Phi((h1 - r12 y)/s12)
//              Phi_2((h3 - r23 y)/s23, (h4 - r24 y)/s24; rho) dy,
// the bivariate CDF by the node sum of device_math.hpp at that fixed rho.
// Same range rule (the upper limit also where the fourth argument falls
// below -L), panels ceil(c / l) with l the smallest of s12/r12, s23/r23,
// s24/r24, at least 12 panels in FP64 (c = 6) and 3 in FP32 (c = 2.5): against
// the adaptive reference over r2 in [0.15, 0.9] and ratios r3/r2, r4/r3 in
// [0.15, 0.9] the error stays below 4e-13 (FP64) and 1.8e-7 (FP32, below the
// FP32 Phi's own error).
#pragma once
#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {

constexpr int kNodes = 8;          // Gauss-Legendre points per panel
constexpr int kPanelsSetup = 16;   // fewest panels for the critical values (FP64)

// Panels in type T for subgroup fractions r2 > r3.
template <typename T>
__device__ __forceinline__ int tvn_panels(double r2, double r3) {
    const double l = fmin(sqrt((1.0 - r2) / r2), sqrt((r2 - r3) / r3));
    const double c = sizeof(T) == 8 ? 6.0 : 2.5;
    const int lo = sizeof(T) == 8 ? 8 : 3, hi = sizeof(T) == 8 ? 128 : 64;
    return max(lo, min(hi, static_cast<int>(ceil(c / l))));
}

// exp(-x^2 / 2); FP32 through exp2.
__device__ __forceinline__ double half_gauss(double x) { return exp(-0.5 * x * x); }
__device__ __forceinline__ float half_gauss(float x) {
    return __builtin_amdgcn_exp2f(x * x * -0.72134752044448170368f);   // log2(e) / 2
}

// A wave-uniform value moved to a scalar register (FP32 constants only).
template <typename T>
__device__ __forceinline__ T uniform(T x) {
    if constexpr (sizeof(T) == 4)
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
    else
        return x;
}

// Constants of Phi_3 in type T: per problem (UNI: the FP32 ones moved to
// scalar registers), or per lane for sweeps whose designs have their own
// fractions (UNI = false).
template <typename T, bool UNI = true>
struct TvnConst {
    __device__ static T U(T x) { return UNI ? uniform(x) : x; }
    T r12, r23;        // regressions of the first and third coordinates on the second
    T is12, is23;      // 1 / s12, 1 / s23
    T tail;            // L: integration range [-L, U]
    T c1, c3;          // L s12, L s23: offsets of the upper integration limit
    T ir12, ir23;      // 1 / r12, 1 / r23
    T px[kNodes];      // panel nodes on [0, 1]
    T pw[kNodes];      // panel weights with phi's 1/sqrt(2 pi) folded in
    int np;            // panels
    // FP32 integrates in y' = k y, k = sqrt(log2(e)/2) (norm_cdf_scaled's
    // unit): phi(y) dy = 2^(-y'^2) dy' / (k sqrt(2 pi)) and each prescaled
    // conditional argument is one fused multiply-add, u' = k h1 / s12 -
    // (r12 / s12) y'; the panel weights go into the exponent as log2.
    T g1, g3;          // r12 / s12, r23 / s23: slopes in y'
    T k1, k3;          // k / s12, k / s23: scales of h1, h3
    T lw[kNodes];      // log2(w_i / (2 k sqrt(2 pi)))

    __device__ void init(double r2, double r3, int panels, const double* __restrict__ gl) {
        const double L = sizeof(T) == 8 ? 8.5 : 6.0;
        const double a = sqrt(r2), b = sqrt(r3 / r2), sa = sqrt(1.0 - r2), sb = sqrt(1.0 - r3 / r2);
        const double k = static_cast<double>(kPhiScale);
        g1 = U(static_cast<T>(a / sa));
        g3 = U(static_cast<T>(b / sb));
        k1 = U(static_cast<T>(k / sa));
        k3 = U(static_cast<T>(k / sb));
        r12 = static_cast<T>(a);
        r23 = static_cast<T>(b);
        is12 = static_cast<T>(1.0 / sa);
        is23 = static_cast<T>(1.0 / sb);
        tail = uniform(static_cast<T>(L));
        c1 = U(static_cast<T>(L * sa));
        c3 = U(static_cast<T>(L * sb));
        ir12 = U(static_cast<T>(1.0 / a));
        ir23 = U(static_cast<T>(1.0 / b));
        const double* x = gl + gl_offset(kNodes);
        const double* w = x + kNodes;
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            // node constants: the same for every design
            px[i] = uniform(static_cast<T>(0.5 * (1.0 + x[i])));
            pw[i] = static_cast<T>(0.5 * w[i] * 0.39894228040143267794);
            lw[i] = uniform(static_cast<T>(log2(0.5 * w[i] * 0.39894228040143267794 / k)));
        }
        np = panels;
    }
};

// FP32 Phi_3 in y' (see TvnConst): per point one FMA for y', one per
// conditional argument, one for the Gaussian's exponent with the weight, an
// exp2, the two CDFs and two to accumulate.
template <bool UNI>
__device__ __forceinline__ float tvn(float h1, float h2, float h3, const TvnConst<float, UNI>& c) {
    const float k = kPhiScale;
    const float lo = -c.tail * k;
    const float hi = k * fminf(fminf(h2, c.tail), fminf((h1 + c.c1) * c.ir12, (h3 + c.c3) * c.ir23));
    const float width = fmaxf(hi - lo, 0.0f) / static_cast<float>(c.np);
    const float H1 = h1 * c.k1, H3 = h3 * c.k3;
    float acc = 0.0f;
    for (int p = 0; p < c.np; ++p) {
        const float a = fmaf(width, static_cast<float>(p), lo);
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            const float y = fmaf(width, c.px[i], a);
            const float u = fmaf(-c.g1, y, H1);
            const float v = fmaf(-c.g3, y, H3);
            const float e = __builtin_amdgcn_exp2f(fmaf(-y, y, c.lw[i]));
            acc = fmaf(e * norm_cdf_scaled(u), norm_cdf_scaled(v), acc);
        }
    }
    return acc * width;
}

// Phi_3(h1, h2, h3) over c.np panels (wave-uniform).  Every lane runs the
// same node count: an empty range (U <= -L) becomes a zero panel width, and
// NaN inputs give NaN.
template <typename T, bool UNI>
__device__ __forceinline__ T tvn(T h1, T h2, T h3, const TvnConst<T, UNI>& c) {
    const T lo = -c.tail;
    const T hi = fmin(fmin(h2, c.tail), fmin((h1 + c.c1) * c.ir12, (h3 + c.c3) * c.ir23));
    const T width = fmax(hi - lo, T(0)) / static_cast<T>(c.np);
    T acc = T(0);
    for (int p = 0; p < c.np; ++p) {
        const T a = fma(width, static_cast<T>(p), lo);
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            const T y = fma(width, c.px[i], a);
            const T u = (h1 - c.r12 * y) * c.is12;
            const T v = (h3 - c.r23 * y) * c.is23;
            acc = fma(c.pw[i] * half_gauss(y), norm_cdf(u) * norm_cdf(v), acc);
        }
    }
    return acc * width;
}


// ---------------------------------------------------------------------------
// Critical values (FP64, one wavefront per design).  The FWER boundary is a
// root of a falling function of one critical value; each evaluation is one
// Phi_3 or Phi_4 at wave-uniform arguments, whose np x 8 panel points the
// lanes share: lane l takes Gauss-Legendre node l % 8 of panels l / 8,
// l / 8 + 8, ..., and every lane returns lane 0's total of the butterfly, so
// the root finder's branches stay wave-uniform.
// ---------------------------------------------------------------------------

// The lane's panel node: position on [0, 1] and weight with phi's
// 1/sqrt(2 pi) folded in (TvnConst's px, pw of node lane % 8).
struct PanelNode {
    double px, pw;
    int p0;   // first panel of the lane
};

__device__ __forceinline__ PanelNode panel_node(const double* __restrict__ gl, int lane) {
    const int i = lane & (kNodes - 1);
    const double* x = gl + gl_offset(kNodes);
    return {0.5 * (1.0 + x[i]), 0.5 * x[kNodes + i] * 0.39894228040143267794, lane / kNodes};
}

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return __shfl(v, 0);
}

// Phi_3(h1, h2, h3) by the wavefront, the rule of tvn().
__device__ __forceinline__ double tvn_wave(double h1, double h2, double h3, const TvnConst<double>& c,
                                           const PanelNode& nd) {
    const double lo = -c.tail;
    const double hi = fmin(fmin(h2, c.tail), fmin((h1 + c.c1) * c.ir12, (h3 + c.c3) * c.ir23));
    const double width = fmax(hi - lo, 0.0) / static_cast<double>(c.np);
    double acc = 0.0;
    for (int p = nd.p0; p < c.np; p += 64 / kNodes) {
        const double y = fma(width, nd.px, fma(width, static_cast<double>(p), lo));
        const double u = (h1 - c.r12 * y) * c.is12;
        const double v = (h3 - c.r23 * y) * c.is23;
        acc = fma(nd.pw * half_gauss(y), norm_cdf(u) * norm_cdf(v), acc);
    }
    return wave_total(acc) * width;
}

// Root of F, falling, in [lo, hi] by the Illinois variant of false position
// (a retained end has its F halved, so both ends move; a step that leaves the
// bracket bisects); the end itself when F(lo) <= 0 or F(hi) >= 0.  Stops at a
// bracket of 1e-14 relative width or |F| at the rounding level `tiny` of the
// CDF.  F takes and returns wave-uniform values.
template <typename Fn>
__device__ __forceinline__ double falling_root(Fn F, double lo, double hi, double tiny) {
    double Flo = F(lo), Fhi = F(hi);
    double z = Flo <= 0.0 ? lo : Fhi >= 0.0 ? hi : 0.5 * (lo + hi);
    int kept = 0;   // +1: lo kept by the last step, -1: hi kept
    for (int it = 0; it < 100 && Flo > 0.0 && Fhi < 0.0; ++it) {
        double x = (lo * Fhi - hi * Flo) / (Fhi - Flo);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        const double Fx = F(x);
        z = x;
        if (Fx == 0.0 || hi - lo <= 1e-14 * fabs(x)) break;
        if (Fx > 0.0) {
            lo = x;
            Flo = Fx;
            if (kept == -1) Fhi *= 0.5;
            kept = -1;
        } else {
            hi = x;
            Fhi = Fx;
            if (kept == 1) Flo *= 0.5;
            kept = 1;
        }
        if (fabs(Fx) <= tiny) break;
    }
    return z;
}

// Partial correlation of (Y3, Y4) given Y2 for fractions r2 > r3 > r4:
// (sqrt(r4/r3) - sqrt(r3/r2) sqrt(r4/r2)) / (s23 s24) = sqrt(r4 (r2 - r3) / (r3 (r2 - r4))).
__host__ __device__ inline double qvn_partial_rho(double r2, double r3, double r4) {
    return sqrt(r4 * (r2 - r3) / (r3 * (r2 - r4)));
}

// Panels of Phi_4 in type T.
template <typename T>
__device__ __forceinline__ int qvn_panels(double r2, double r3, double r4) {
    const double l = fmin(fmin(sqrt((1.0 - r2) / r2), sqrt((r2 - r3) / r3)), sqrt((r2 - r4) / r4));
    const double c = sizeof(T) == 8 ? 6.0 : 2.5;
    const int lo = sizeof(T) == 8 ? 12 : 3, hi = sizeof(T) == 8 ? 128 : 64;
    return max(lo, min(hi, static_cast<int>(ceil(c / l))));
}

// Per-problem constants of Phi_4 for four nested populations, in type T.
template <typename T, int NMAX, bool UNI = true>
struct QvnConst {
    __device__ static T U(T x) { return UNI ? uniform(x) : x; }
    T r12, r23, r24;     // regressions on the second coordinate
    T is12, is23, is24;  // 1 / s12, 1 / s23, 1 / s24
    T tail;
    T c1, c3, c4;        // L s1j: offsets of the upper integration limit
    T ir12, ir23, ir24;
    T px[kNodes], pw[kNodes];
    int np;              // panels
    BvnConst<T, NMAX> bc;   // Phi_2 at the partial correlation of (Y3, Y4) given Y2
    T bw[NMAX];          // its node weights
    int nb;              // its node count (a rule of the packed table)
    // FP32 in y' as for Phi_3: slopes r1j / s1j, scales k / s1j, log2 weights
    T g1, g3, g4, k1, k3, k4;
    T lw[kNodes];

    __device__ void init(double r2, double r3, double r4, int panels, int bvn_n, const double* __restrict__ gl) {
        const double L = sizeof(T) == 8 ? 8.5 : 6.0;
        const double a = sqrt(r2), b = sqrt(r3 / r2), c = sqrt(r4 / r2);
        const double sa = sqrt(1.0 - r2), sb = sqrt(1.0 - r3 / r2), sc = sqrt(1.0 - r4 / r2);
        r12 = static_cast<T>(a);
        r23 = static_cast<T>(b);
        r24 = static_cast<T>(c);
        // FP32 CDFs take arguments prescaled by sqrt(log2(e)/2) (norm_cdf_scaled)
        const double k = sizeof(T) == 4 ? static_cast<double>(kPhiScale) : 1.0;
        is12 = static_cast<T>(k / sa);
        is23 = static_cast<T>(k / sb);
        is24 = static_cast<T>(k / sc);
        tail = static_cast<T>(L);
        c1 = static_cast<T>(L * sa);
        c3 = static_cast<T>(L * sb);
        c4 = static_cast<T>(L * sc);
        ir12 = static_cast<T>(1.0 / a);
        ir23 = static_cast<T>(1.0 / b);
        ir24 = static_cast<T>(1.0 / c);
        const double* x = gl + gl_offset(kNodes);
        const double* w = x + kNodes;
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            px[i] = static_cast<T>(0.5 * (1.0 + x[i]));
            pw[i] = static_cast<T>(0.5 * w[i] * 0.39894228040143267794);
        }
        {
            const double kk = static_cast<double>(kPhiScale);
            g1 = U(static_cast<T>(a / sa));
            g3 = U(static_cast<T>(b / sb));
            g4 = U(static_cast<T>(c / sc));
            k1 = U(static_cast<T>(kk / sa));
            k3 = U(static_cast<T>(kk / sb));
            k4 = U(static_cast<T>(kk / sc));
#pragma unroll
            for (int i = 0; i < kNodes; ++i) {
                lw[i] = uniform(static_cast<T>(log2(0.5 * w[i] * 0.39894228040143267794 / kk)));
                px[i] = uniform(px[i]);
            }
            tail = uniform(tail);
            c1 = U(c1);
            c3 = U(c3);
            c4 = U(c4);
            ir12 = U(ir12);
            ir23 = U(ir23);
            ir24 = U(ir24);
        }
        np = panels;
        nb = bvn_n;
        bc.init(qvn_partial_rho(r2, r3, r4), bvn_n, gl);
        const double* bwx = gl + gl_offset(bvn_n) + bvn_n;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            bw[i] = uniform(static_cast<T>(i < bvn_n ? bwx[i] : 0.0));
            bc.a[i] = U(bc.a[i]);
            bc.b[i] = U(bc.b[i]);
        }
        bc.scale = U(bc.scale);
    }
};

// Univariate and bivariate CDFs at the arguments QvnConst prepares: FP32
// prescaled, FP64 as they are.
__device__ __forceinline__ float qvn_cdf1(float x) { return norm_cdf_scaled(x); }
__device__ __forceinline__ double qvn_cdf1(double x) { return norm_cdf(x); }
template <int NMAX, bool UNI>
__device__ __forceinline__ float qvn_cdf2(float a, float b, const QvnConst<float, NMAX, UNI>& c) {
    return bvn_cdf_scaled<NMAX>(a, b, c.bc, c.bw, c.nb);
}
template <int NMAX, bool UNI>
__device__ __forceinline__ double qvn_cdf2(double a, double b, const QvnConst<double, NMAX, UNI>& c) {
    return bvn_cdf<NMAX>(a, b, c.bc, c.bw, c.nb);
}

// FP32 Phi_4 in y' (see TvnConst): the three conditional arguments are one
// FMA each and arrive prescaled at the univariate and bivariate CDFs.
template <int NMAX, bool UNI>
__device__ __forceinline__ float qvn(float h1, float h2, float h3, float h4, const QvnConst<float, NMAX, UNI>& c) {
    const float k = kPhiScale;
    const float lo = -c.tail * k;
    const float hi = k * fminf(fminf(fminf(h2, c.tail), (h1 + c.c1) * c.ir12),
                               fminf((h3 + c.c3) * c.ir23, (h4 + c.c4) * c.ir24));
    const float width = fmaxf(hi - lo, 0.0f) / static_cast<float>(c.np);
    const float H1 = h1 * c.k1, H3 = h3 * c.k3, H4 = h4 * c.k4;
    float acc = 0.0f;
    for (int p = 0; p < c.np; ++p) {
        const float a = fmaf(width, static_cast<float>(p), lo);
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            const float y = fmaf(width, c.px[i], a);
            const float u1 = fmaf(-c.g1, y, H1);
            const float u3 = fmaf(-c.g3, y, H3);
            const float u4 = fmaf(-c.g4, y, H4);
            const float e = __builtin_amdgcn_exp2f(fmaf(-y, y, c.lw[i]));
            acc = fmaf(e * norm_cdf_scaled(u1), bvn_cdf_scaled<NMAX>(u3, u4, c.bc, c.bw, c.nb), acc);
        }
    }
    return acc * width;
}

// Phi_4(h1, h2, h3, h4) over c.np panels (wave-uniform); an empty range gives
// zero, NaN inputs NaN.
template <typename T, int NMAX, bool UNI>
__device__ __forceinline__ T qvn(T h1, T h2, T h3, T h4, const QvnConst<T, NMAX, UNI>& c) {
    const T lo = -c.tail;
    const T hi = fmin(fmin(fmin(h2, c.tail), (h1 + c.c1) * c.ir12),
                      fmin((h3 + c.c3) * c.ir23, (h4 + c.c4) * c.ir24));
    const T width = fmax(hi - lo, T(0)) / static_cast<T>(c.np);
    T acc = T(0);
    for (int p = 0; p < c.np; ++p) {
        const T a = fma(width, static_cast<T>(p), lo);
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            const T y = fma(width, c.px[i], a);
            const T u1 = (h1 - c.r12 * y) * c.is12;
            const T u3 = (h3 - c.r23 * y) * c.is23;
            const T u4 = (h4 - c.r24 * y) * c.is24;
            acc = fma(c.pw[i] * half_gauss(y) * qvn_cdf1(u1), qvn_cdf2(u3, u4, c), acc);
        }
    }
    return acc * width;
}

// Phi_4(h1, h2, h3, h4) in FP64 by the wavefront, the rule of qvn().
template <int NMAX>
__device__ __forceinline__ double qvn_wave(double h1, double h2, double h3, double h4,
                                           const QvnConst<double, NMAX>& c, const PanelNode& nd) {
    const double lo = -c.tail;
    const double hi = fmin(fmin(fmin(h2, c.tail), (h1 + c.c1) * c.ir12),
                           fmin((h3 + c.c3) * c.ir23, (h4 + c.c4) * c.ir24));
    const double width = fmax(hi - lo, 0.0) / static_cast<double>(c.np);
    double acc = 0.0;
    for (int p = nd.p0; p < c.np; p += 64 / kNodes) {
        const double y = fma(width, nd.px, fma(width, static_cast<double>(p), lo));
        const double u1 = (h1 - c.r12 * y) * c.is12;
        const double u3 = (h3 - c.r23 * y) * c.is23;
        const double u4 = (h4 - c.r24 * y) * c.is24;
        acc = fma(nd.pw * half_gauss(y) * qvn_cdf1(u1), qvn_cdf2(u3, u4, c), acc);
    }
    return wave_total(acc) * width;
}

}  // namespace bmd
