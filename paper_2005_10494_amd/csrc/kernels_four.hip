// Four nested populations 1 > r2 > r3 > r4 (n = 4 of Sec. 2.2: the designs
// with three candidate thresholds of Sec. 3, null correlations of Appendix
// A.1, Formula 10 prior): per-design critical values with the fourth on the
// FWER boundary of Formula 2, and the grid sweep of the Formula 5 estimate
// whose summand is 1 - Phi_4(z - mu; R), Phi_4 as in nested_cdf.hpp.
#include <cmath>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "nested_cdf.hpp"

namespace bmd {
namespace {

constexpr int kBvnMax64 = 24;   // largest FP64 rule of the packed table
constexpr int kBvnMax32 = 12;   // largest FP32 rule

// Levels alpha_1, alpha_2, alpha_3 (axes 0, 1, 2) of design g; the fourth
// critical value solves F(z4) = 1 - Phi_4(z1, z2, z3, z4) - alpha0 = 0 (F
// falls in z4) inside the bracket from the fourth test alone at level alpha0
// (F >= 0) to the union bound with the level a123 = 1 - Phi_3(z1, z2, z3) the
// first three spend (F <= 0), by falling_root as for the third level of three
// populations (one wavefront per design).  NaN when a123 >= alpha0.
__global__ __launch_bounds__(64) void k_four_precompute(DevProblem P, const double* __restrict__ gl,
                                                        double* __restrict__ r_out, double* __restrict__ z1_out,
                                                        double* __restrict__ z2_out, double* __restrict__ z3_out,
                                                        double* __restrict__ z4_out) {
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int i0 = static_cast<int>(g / P.stride[0]);
    const int i1 = static_cast<int>((g / P.stride[1]) % P.m[1]);
    const int i2 = static_cast<int>(g % P.m[2]);
    const double z1 = -norm_quantile(grid_coord(P.q_lo, P.q_hi, i0, P.m[0]));
    const double z2 = -norm_quantile(grid_coord(P.q_lo, P.q_hi, i1, P.m[1]));
    const double z3 = -norm_quantile(grid_coord(P.q_lo, P.q_hi, i2, P.m[2]));
    const PanelNode nd = panel_node(gl, lane);
    TvnConst<double> c3;
    c3.init(P.r_lo, P.r_hi, max(kPanelsSetup, tvn_panels<double>(P.r_lo, P.r_hi)), gl);
    const double a123 = 1.0 - tvn_wave(z1, z2, z3, c3, nd);
    double z4 = NAN;
    if (a123 < P.alpha0) {
        QvnConst<double, kBvnMax64> c;
        c.init(P.r_lo, P.r_hi, P.r_4, max(kPanelsSetup, qvn_panels<double>(P.r_lo, P.r_hi, P.r_4)),
               bvn_nodes_fp64(qvn_partial_rho(P.r_lo, P.r_hi, P.r_4)), gl);
        auto F = [&](double z) { return (1.0 - qvn_wave(z1, z2, z3, z, c, nd)) - P.alpha0; };
        z4 = falling_root(F, -norm_quantile(P.alpha0), -norm_quantile(P.alpha0 - a123), 4e-16);
    }
    if (lane == 0) {
        r_out[g] = P.r_lo;
        z1_out[g] = z1;
        z2_out[g] = z2;
        z3_out[g] = z3;
        z4_out[g] = z4;
    }
}

template <typename T>
struct FourArgs {
    int64_t G;
    int m0, m1, m2;     // grid points of alpha_1, alpha_2, alpha_3 (axes 0, 1, 2)
    const double* z1;
    const double* z2;
    const double* z3;
    const double* z4;
    const int32_t* order;   // [G] designs with a fourth level first
    const T* e1;
    const T* e2;
    const T* e3;
    const T* e4;
    int64_t M;
    int64_t slice_len;
    double* partials;   // [n_slices][2][G]: sums, then sums of squares (VAR only)
    const double* gl;   // packed Gauss-Legendre table, FP64
    double r2, r3, r4;
    // Formula 10 means sqrt(r_i I) (theta_i + sigma_i Y_i) of the four statistics,
    // linear in the draw's normals: mu1 = m0 + m1 e1, mu2 = m2 + m3 e1 + m4 e2,
    // mu3 = m5 + m6 e1 + m7 e2 + m8 e3, mu4 = m9 + m10 e1 + m11 e2 + m12 e3 + m13 e4.
    double m[14];
};

// One thread per design (alpha_1, alpha_2, alpha_3), the draws of slice
// blockIdx.y.  The designs go in the problem's order (those with a fourth
// level first), so the wavefronts that compute are full of designs that have
// one, and the designs without one form whole wavefronts that write NaN sums
// and leave without touching the draws.
template <typename T, bool VAR>
__global__ __launch_bounds__(kEvalBlock) void k_eval_four(FourArgs<T> a) {
    constexpr int NB = sizeof(T) == 8 ? kBvnMax64 : kBvnMax32;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kEvalBlock + threadIdx.x;
    const bool valid = idx < a.G;
    // idle lanes shadow the last design of the order
    const int64_t g = a.order[valid ? idx : a.G - 1], gg = g;
    const int slice = blockIdx.y;
    const double z4d = a.z4[gg];
    if (__all(!valid || z4d != z4d)) {
        if (valid) {
            double* out = a.partials + static_cast<int64_t>(slice) * 2 * a.G;
            out[g] = z4d;
            if constexpr (VAR) out[a.G + g] = z4d;
        }
        return;
    }
    QvnConst<T, NB> c;
    const double rho = qvn_partial_rho(a.r2, a.r3, a.r4);
    c.init(a.r2, a.r3, a.r4, qvn_panels<T>(a.r2, a.r3, a.r4), sizeof(T) == 8 ? bvn_nodes_fp64(rho) : bvn_nodes_fp32(rho),
           a.gl);
    const T z1 = static_cast<T>(a.z1[gg]), z2 = static_cast<T>(a.z2[gg]), z3 = static_cast<T>(a.z3[gg]);
    const T z4 = static_cast<T>(z4d);
    T m[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) m[i] = static_cast<T>(a.m[i]);
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(a.M, kb + a.slice_len);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const T e1 = a.e1[k], e2 = a.e2[k], e3 = a.e3[k], e4 = a.e4[k];
        const T h1 = z1 - fma(m[1], e1, m[0]);
        const T h2 = z2 - fma(m[4], e2, fma(m[3], e1, m[2]));
        const T h3 = z3 - fma(m[8], e3, fma(m[7], e2, fma(m[6], e1, m[5])));
        const T h4 = z4 - fma(m[13], e4, fma(m[12], e3, fma(m[11], e2, fma(m[10], e1, m[9]))));
        const double v = static_cast<double>(T(1) - qvn(h1, h2, h3, h4, c));
        s1 += v;
        if constexpr (VAR) s2 = fma(v, v, s2);
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(slice) * 2 * a.G;
        out[g] = s1;
        if constexpr (VAR) out[a.G + g] = s2;
    }
}

template <typename T>
FourArgs<T> four_args(const bmd_problem* p, DrawArrays<T> D, double* partials, int64_t slice_len) {
    const DevProblem& P = p->P;
    FourArgs<T> a{};
    a.G = P.G;
    a.m0 = P.m[0];
    a.m1 = P.m[1];
    a.m2 = P.m[2];
    a.z1 = p->d_z1;
    a.z2 = p->d_z2;
    a.z3 = p->d_z3;
    a.z4 = p->d_z4;
    a.order = p->d_order;
    a.e1 = D.e1;
    a.e2 = D.e2;
    a.e3 = D.e3;
    a.e4 = D.e4;
    a.M = D.M;
    a.slice_len = slice_len;
    a.partials = partials;
    a.gl = p->d_gl;
    a.r2 = P.r_lo;
    a.r3 = P.r_hi;
    a.r4 = P.r_4;
    const double r[4] = {1.0, P.r_lo, P.r_hi, P.r_4};
    double th[4], sc[4];
    for (int i = 0; i < 4; ++i) {
        th[i] = -std::log1p(-(P.paper_a - P.paper_b * r[i]));
        sc[i] = std::sqrt(r[i] * P.info) / std::sqrt(P.paper_events * r[i] / 4.0);   // sqrt(r_i I) sigma_i
    }
    // Y1 = e1 and Y_{i+1} = sqrt(r_{i+1}/r_i) Y_i + sqrt(1 - r_{i+1}/r_i) e_{i+1}:
    // coefficient of e_j in Y_i, row by row.
    double Y[4][4] = {};
    Y[0][0] = 1.0;
    for (int i = 1; i < 4; ++i) {
        for (int j = 0; j < i; ++j) Y[i][j] = std::sqrt(r[i] / r[i - 1]) * Y[i - 1][j];
        Y[i][i] = std::sqrt(1.0 - r[i] / r[i - 1]);
    }
    int k = 0;
    for (int i = 0; i < 4; ++i) {
        a.m[k++] = std::sqrt(r[i] * P.info) * th[i];
        for (int j = 0; j <= i; ++j) a.m[k++] = sc[i] * Y[i][j];
    }
    return a;
}

template <typename T>
hipError_t launch_typed(const FourArgs<T>& a, int n_slices, bool var, hipStream_t s) {
    const void* k = var ? reinterpret_cast<const void*>(k_eval_four<T, true>)
                        : reinterpret_cast<const void*>(k_eval_four<T, false>);
    void* args[] = {const_cast<FourArgs<T>*>(&a)};
    return hipLaunchKernel(k, dim3(static_cast<unsigned>((a.G + kEvalBlock - 1) / kEvalBlock), static_cast<unsigned>(n_slices)),
                           dim3(kEvalBlock), args, 0, s);
}

}  // namespace

hipError_t launch_four_precompute(const bmd_problem* p, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_four_precompute, dim3(static_cast<unsigned>(G)), dim3(64), 0, s, p->P,
                       p->d_gl, p->d_r, p->d_z1, p->d_z2, p->d_z3, p->d_z4);
    return hipGetLastError();
}

int four_blocks_per_cu(int prec) {
    const void* k = prec == BMD_FP64 ? reinterpret_cast<const void*>(k_eval_four<double, false>)
                                     : reinterpret_cast<const void*>(k_eval_four<float, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kEvalBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_eval_four(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, bool want_var, hipStream_t s) {
    if (prec == BMD_FP64)
        return launch_typed<double>(four_args<double>(p, draws_fp64(p, M, ws), partials, slice_len), n_slices,
                                    want_var, s);
    return launch_typed<float>(four_args<float>(p, draws_fp32(p, M, ws), partials, slice_len), n_slices, want_var,
                               s);
}

}  // namespace bmd
