// One summand of the Formula 5 estimate for a grid design and a prior draw
// (the direct sweep body; the matrix-core body uses its pieces).
//
//   1 - Phi_2(z1 - mu1_k, z2 - mu2_gk; sqrt r_g)
//   step prior:  mu1 = sqrt(I) (b0 + b1 P(R)),  mu2 = sqrt(r I) (b0 + b1 O / r),
//                O = P(x_j > max(c_j, t_j) all j), the responders inside the subgroup
//   paper prior: mu1 = sqrt(I) Delta_1,  mu2 = sqrt(r I) Delta_2  (Formula 10)
#pragma once
#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

template <typename T>
__device__ __forceinline__ T logistic_fn(T x) {
    return T(1) / (T(1) + exp(-x));
}

// Draws read from the per-draw arrays of the draw kernel.
template <typename T>
struct GlobalDraws {
    DrawArrays<T> D;
    int d;
    __device__ T b0(int64_t k) const { return D.b0[k]; }
    __device__ T b1(int64_t k) const { return D.b1[k]; }
    __device__ T mu1(int64_t k) const { return D.mu1[k]; }
    __device__ T PR(int64_t k) const { return D.PR[k]; }
    __device__ T tauT(int64_t k) const { return D.tauT[k]; }
    __device__ T e1(int64_t k) const { return D.e1[k]; }
    __device__ T e2(int64_t k) const { return D.e2[k]; }
    __device__ int thr(int j, int64_t k) const { return D.thr[k * d + j]; }
    __device__ double tau(int j, int64_t k) const { return D.tau[j * D.M + k]; }
    __device__ const T* B(int64_t k) const { return D.B + k * d * D.K; }
};

// Everything about one grid design that the summand needs, held in registers.
template <typename T, int D, int NMAX>
struct DesignState {
    int idx[D];
    double q[D];
    BvnConst<T, NMAX> bc;
    int n;                 // Gauss-Legendre nodes (wave-uniform)
    const T* w;            // their weights
    T z1, z2, srI, invr, rT, omq, c0, c1, c2;
    // FP32 matrix-core sweep: the critical values and drift factors times
    // sqrt(log2(e)/2), so the bivariate normal's arguments arrive prescaled
    T z1s, z2s, a0s, a1s;
    // Derivative of the summand in the first test's level alpha_1 (init_dalpha):
    //   d(1 - Phi_2(h, k))/d alpha_1 = da1 phi(h) Phi((k - rho h)/s) + da2 phi(k) Phi((h - rho k)/s),
    // da1 = 1/phi(z1) from dz1/d alpha_1 = -1/phi(z1); with the second level on
    // the FWER boundary (rule BMD_ALPHA_SPLIT) da2 = (dz2/dz1)/phi(z1),
    // dz2/dz1 = -phi(z1) Phi((z2 - rho z1)/s) / (phi(z2) Phi((z1 - rho z2)/s));
    // with a fixed second level da2 = 0.  da1, da2 carry phi's 1/sqrt(2 pi);
    // rs = rho/s and is = 1/s give the conditional arguments.
    T da1, da2, rs, is;

    __device__ void init(const DevProblem& P, int64_t g, const double* __restrict__ r_arr,
                         const double* __restrict__ z1_arr, const double* __restrict__ z2_arr,
                         const double* __restrict__ gl, const T* __restrict__ glw) {
        int64_t rem = g;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            idx[j] = static_cast<int>(rem / P.stride[j]);
            rem -= static_cast<int64_t>(idx[j]) * P.stride[j];
            q[j] = grid_coord(P.q_lo, P.q_hi, idx[j], P.m[j]);
        }
        const double r = r_arr[g];
        const double rho = sqrt(r);
        n = wave_max_int(sizeof(T) == 8 ? bvn_nodes_fp64(rho) : bvn_nodes_fp32(rho));
        bc.init(rho, n, gl);
        w = glw + gl_offset(n) + n;
        const double srI_d = sqrt(r * P.info);
        z1 = static_cast<T>(z1_arr[g]);
        z2 = static_cast<T>(z2_arr[g]);
        srI = static_cast<T>(srI_d);
        invr = static_cast<T>(1.0 / r);
        rT = static_cast<T>(r);
        omq = static_cast<T>(1.0 - q[0]);
        {
            const double sc = static_cast<double>(kPhiScale);
            z1s = static_cast<T>(sc * z1_arr[g]);
            z2s = static_cast<T>(sc * z2_arr[g]);
            a0s = static_cast<T>(sc * srI_d);
            a1s = static_cast<T>(sc * srI_d / r);
        }
        c0 = c1 = c2 = T(0);
        da1 = da2 = rs = is = T(0);
        if (P.effect == BMD_EFFECT_PAPER_GAUSS) {
            const double th2 = -log1p(-(P.paper_a - P.paper_b * r));
            const double sg2 = 1.0 / sqrt(P.paper_events * r / 4.0);
            c0 = static_cast<T>(srI_d * th2);
            c1 = static_cast<T>(srI_d * sg2 * sqrt(r));
            c2 = static_cast<T>(srI_d * sg2 * sqrt(1.0 - r));
        }
    }

    // The alpha_1-derivative constants for critical values z1, z2 (finite z1).
    __device__ void init_dalpha(const DevProblem& P, double r, double z1d, double z2d) {
        const double rho = sqrt(r), sd = sqrt((1.0 - rho) * (1.0 + rho));
        const double inv_root_2pi = 0.39894228040143267794;
        const double c1d = 1.0 / norm_pdf(z1d);
        double c2d = 0.0;
        if (P.alpha_rule == BMD_ALPHA_SPLIT && z2d < INFINITY) {
            const double dz2 = -norm_pdf(z1d) * norm_cdf((z2d - rho * z1d) / sd) /
                               (norm_pdf(z2d) * norm_cdf((z1d - rho * z2d) / sd));
            c2d = dz2 * c1d;
        }
        da1 = static_cast<T>(c1d * inv_root_2pi);
        da2 = static_cast<T>(c2d * inv_root_2pi);
        rs = static_cast<T>(rho / sd);
        is = static_cast<T>(1.0 / sd);
    }
};

// The alpha_1-derivative of one summand at its arguments h, k (unscaled):
// da1 phi(h) Phi((k - rho h)/s) + da2 phi(k) Phi((h - rho k)/s), each phi
// without its 1/sqrt(2 pi) (carried by da1, da2); a second critical value at
// +infinity (zinf bit 1) leaves phi(h) alone, as the one-test derivative of
// Appendix A.3.
template <typename T, int D, int NMAX>
__device__ __forceinline__ T dalpha_term(const DevProblem& P, const DesignState<T, D, NMAX>& s, T h, T kq) {
    const T g = T(-0.5);
    if (P.zinf & 2) return s.da1 * exp(g * h * h);
    const T ph = exp(g * h * h) * norm_cdf(fma(kq, s.is, -s.rs * h));
    const T pk = exp(g * kq * kq) * norm_cdf(fma(h, s.is, -s.rs * kq));
    return fma(s.da1, ph, s.da2 * pk);
}

// Responder-in-subgroup fraction O for draw k (d >= 2).  A: axis tables
// [d][K][mmax] with the Gauss-Hermite weights folded into axis 0.
template <typename T, int D, int NMAX, typename Src>
__device__ __forceinline__ T overlap(const DevProblem& P, const DesignState<T, D, NMAX>& s, const Src& src,
                                     int64_t k, const T* __restrict__ A, int K) {
    const int mmax = P.mmax;
    const T* Bk = src.B(k);
    if (P.width > 0.0) {
        T sw[D];
#pragma unroll
        for (int j = 0; j < D; ++j) sw[j] = logistic_fn(static_cast<T>((s.q[j] - src.tau(j, k)) / P.width));
        T acc = T(0);
        for (int m = 0; m < K; ++m) {
            T prod = T(1);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const T av = A[(static_cast<int64_t>(j) * K + m) * mmax + s.idx[j]];
                prod *= sw[j] * av + (T(1) - sw[j]) * Bk[m * D + j];
            }
            acc += prod;
        }
        return acc;
    }
    bool fl[D];
    bool all = true, none = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        fl[j] = s.idx[j] >= src.thr(j, k);
        all = all && fl[j];
        none = none && !fl[j];
    }
    if (all) return s.rT;
    if (none) return src.PR(k);
    const T* p[D];
    int64_t st[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        p[j] = fl[j] ? A + static_cast<int64_t>(j) * K * mmax + s.idx[j] : Bk + j;
        st[j] = fl[j] ? mmax : D;
    }
    T acc = T(0);
    for (int m = 0; m < K; ++m) {
        T prod = p[0][m * st[0]];
#pragma unroll
        for (int j = 1; j < D; ++j) prod *= p[j][m * st[j]];
        acc += prod;
    }
    return acc;
}

// 1 - Phi_2(...) for design s and draw k; with dv, also its derivative in
// alpha_1 (dalpha_term; the design's init_dalpha constants).
template <typename T, int D, int NMAX, typename Src>
__device__ __forceinline__ T summand(const DevProblem& P, const DesignState<T, D, NMAX>& s, const Src& src,
                                     int64_t k, const T* __restrict__ A, int K, T* dv = nullptr) {
    const T mu1 = src.mu1(k);
    T mu2;
    if (P.effect == BMD_EFFECT_STEP) {
        T O;
        if constexpr (D == 1) {
            if (P.width > 0.0) {
                const T sw = logistic_fn(static_cast<T>((s.q[0] - src.tau(0, k)) / P.width));
                O = T(1) - (sw * static_cast<T>(s.q[0]) + (T(1) - sw) * src.tauT(k));
            } else {
                O = s.idx[0] >= src.thr(0, k) ? s.omq : T(1) - src.tauT(k);
            }
        } else {
            O = overlap<T, D, NMAX>(P, s, src, k, A, K);
        }
        mu2 = s.srI * (src.b0(k) + src.b1(k) * O * s.invr);
    } else {
        mu2 = s.c0 + s.c1 * src.e1(k) + s.c2 * src.e2(k);
    }
    const T h = s.z1 - mu1, kq = s.z2 - mu2;
    if (dv) *dv = dalpha_term<T, D, NMAX>(P, s, h, kq);
    if (P.zinf == 0) return bvn_sf<NMAX>(h, kq, s.bc, s.w, s.n);
    if (P.zinf == 1) return T(1) - norm_cdf(kq);
    if (P.zinf == 2) return T(1) - norm_cdf(h);
    return T(0);
}

}  // namespace bmd
