// Three nested populations 1 > r2 > r3 (n = 3 of Sec. 2.2, with the null
// correlations of Appendix A.1 and the Formula 10 prior; Sec. 3 condition
// (c)): per-design critical values with the third on the FWER boundary of
// Formula 2, and the grid sweep of the Formula 5 estimate whose summand is
// 1 - Phi_3(z - mu; R), Phi_3 as in nested_cdf.hpp.
#include <cmath>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "nested_cdf.hpp"

namespace bmd {
namespace {

// Levels alpha_1 (axis 0) and alpha_2 (axis 1) of design g; the third critical
// value solves F(z3) = 1 - Phi_3(z1, z2, z3) - alpha0 = 0 (F falls in z3)
// inside the bracket from the third test alone at level alpha0 (F >= 0) to the
// union bound with the level a12 = 1 - Phi_2(z1, z2; sqrt r2) the first two
// spend (F <= 0), by falling_root with Phi_3 shared by the wavefront's lanes
// (one wavefront per design).  NaN when a12 >= alpha0.
__global__ __launch_bounds__(64) void k_three_precompute(DevProblem P, const double* __restrict__ gl,
                                                         double* __restrict__ r_out, double* __restrict__ z1_out,
                                                         double* __restrict__ z2_out, double* __restrict__ z3_out) {
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int i0 = static_cast<int>(g / P.stride[0]);
    const int i1 = static_cast<int>(g - static_cast<int64_t>(i0) * P.stride[0]);
    const double z1 = -norm_quantile(grid_coord(P.q_lo, P.q_hi, i0, P.m[0]));
    const double z2 = -norm_quantile(grid_coord(P.q_lo, P.q_hi, i1, P.m[1]));
    constexpr int n = 24;
    const double* w = gl + gl_offset(n) + n;
    BvnConst<double, n> b12;
    b12.init(sqrt(P.r_lo), n, gl);
    const double a12 = 1.0 - bvn_cdf<n>(z1, z2, b12, w, n);
    double z3 = NAN;
    if (a12 < P.alpha0) {
        TvnConst<double> c;
        c.init(P.r_lo, P.r_hi, max(kPanelsSetup, tvn_panels<double>(P.r_lo, P.r_hi)), gl);
        const PanelNode nd = panel_node(gl, lane);
        auto F = [&](double z) { return (1.0 - tvn_wave(z1, z2, z, c, nd)) - P.alpha0; };
        z3 = falling_root(F, -norm_quantile(P.alpha0), -norm_quantile(P.alpha0 - a12), 4e-16);
    }
    if (lane == 0) {
        r_out[g] = P.r_lo;
        z1_out[g] = z1;
        z2_out[g] = z2;
        z3_out[g] = z3;
    }
}

template <typename T>
struct ThreeArgs {
    int64_t G;
    int m0, m1;         // grid points of alpha_1 (axis 0) and alpha_2 (axis 1)
    const double* z1;
    const double* z2;
    const double* z3;
    const int32_t* order;   // [G] designs with a third level first
    const T* e1;
    const T* e2;
    const T* e3;
    int64_t M;
    int64_t slice_len;
    double* partials;   // [n_slices][2][G]: sums, then sums of squares (VAR only)
    const double* gl;   // packed Gauss-Legendre table, FP64
    double r2, r3;
    // Formula 10 means of the three statistics, sqrt(r_i I) (theta_i + sigma_i Y_i):
    // mu1 = m0 + m1 e1, mu2 = m2 + m3 e1 + m4 e2, mu3 = m5 + m6 e1 + m7 e2 + m8 e3.
    double m[9];
};

// One thread per design (alpha_1, alpha_2), the draws of slice blockIdx.y.
// The designs go in the problem's order (those with a third level first), so
// the wavefronts that compute are full of designs that have one, and the
// designs without one (the corner where both levels are large) form whole
// wavefronts that write NaN sums and leave without touching the draws.
template <typename T, bool VAR>
__global__ __launch_bounds__(kEvalBlock) void k_eval_three(ThreeArgs<T> a) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kEvalBlock + threadIdx.x;
    const bool valid = idx < a.G;
    // idle lanes shadow the last design of the order
    const int64_t g = a.order[valid ? idx : a.G - 1], gg = g;
    const int slice = blockIdx.y;
    const double z3d = a.z3[gg];
    if (__all(!valid || z3d != z3d)) {
        if (valid) {
            double* out = a.partials + static_cast<int64_t>(slice) * 2 * a.G;
            out[g] = z3d;
            if constexpr (VAR) out[a.G + g] = z3d;
        }
        return;
    }
    TvnConst<T> c;
    c.init(a.r2, a.r3, tvn_panels<T>(a.r2, a.r3), a.gl);
    const T z1 = static_cast<T>(a.z1[gg]), z2 = static_cast<T>(a.z2[gg]), z3 = static_cast<T>(z3d);
    T m[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = static_cast<T>(a.m[i]);
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(a.M, kb + a.slice_len);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const T e1 = a.e1[k], e2 = a.e2[k], e3 = a.e3[k];
        const T h1 = z1 - fma(m[1], e1, m[0]);
        const T h2 = z2 - fma(m[4], e2, fma(m[3], e1, m[2]));
        const T h3 = z3 - fma(m[8], e3, fma(m[7], e2, fma(m[6], e1, m[5])));
        const double v = static_cast<double>(T(1) - tvn(h1, h2, h3, c));
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
ThreeArgs<T> three_args(const bmd_problem* p, DrawArrays<T> D, double* partials, int64_t slice_len) {
    const DevProblem& P = p->P;
    ThreeArgs<T> a{};
    a.G = P.G;
    a.m0 = P.m[0];
    a.m1 = P.m[1];
    a.z1 = p->d_z1;
    a.z2 = p->d_z2;
    a.z3 = p->d_z3;
    a.order = p->d_order;
    a.e1 = D.e1;
    a.e2 = D.e2;
    a.e3 = D.e3;
    a.M = D.M;
    a.slice_len = slice_len;
    a.partials = partials;
    a.gl = p->d_gl;
    a.r2 = P.r_lo;
    a.r3 = P.r_hi;
    const double r[3] = {1.0, P.r_lo, P.r_hi};
    double th[3], sc[3];
    for (int i = 0; i < 3; ++i) {
        th[i] = -std::log1p(-(P.paper_a - P.paper_b * r[i]));
        sc[i] = std::sqrt(r[i] * P.info) / std::sqrt(P.paper_events * r[i] / 4.0);   // sqrt(r_i I) sigma_i
    }
    // Y1 = e1, Y2 = sqrt(r2) e1 + sqrt(1 - r2) e2,
    // Y3 = sqrt(r3) e1 + sqrt(r3 (1 - r2) / r2) e2 + sqrt(1 - r3 / r2) e3
    a.m[0] = std::sqrt(P.info) * th[0];
    a.m[1] = sc[0];
    a.m[2] = std::sqrt(r[1] * P.info) * th[1];
    a.m[3] = sc[1] * std::sqrt(r[1]);
    a.m[4] = sc[1] * std::sqrt(1.0 - r[1]);
    a.m[5] = std::sqrt(r[2] * P.info) * th[2];
    a.m[6] = sc[2] * std::sqrt(r[2]);
    a.m[7] = sc[2] * std::sqrt(r[2] * (1.0 - r[1]) / r[1]);
    a.m[8] = sc[2] * std::sqrt(1.0 - r[2] / r[1]);
    return a;
}

template <typename T>
hipError_t launch_typed(const ThreeArgs<T>& a, int n_slices, bool var, hipStream_t s) {
    const void* k = var ? reinterpret_cast<const void*>(k_eval_three<T, true>)
                        : reinterpret_cast<const void*>(k_eval_three<T, false>);
    void* args[] = {const_cast<ThreeArgs<T>*>(&a)};
    return hipLaunchKernel(k, dim3(static_cast<unsigned>((a.G + kEvalBlock - 1) / kEvalBlock), static_cast<unsigned>(n_slices)),
                           dim3(kEvalBlock), args, 0, s);
}

}  // namespace

hipError_t launch_three_precompute(const bmd_problem* p, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_three_precompute, dim3(static_cast<unsigned>(G)), dim3(64), 0, s, p->P,
                       p->d_gl, p->d_r, p->d_z1, p->d_z2, p->d_z3);
    return hipGetLastError();
}

int three_blocks_per_cu(int prec) {
    const void* k = prec == BMD_FP64 ? reinterpret_cast<const void*>(k_eval_three<double, false>)
                                     : reinterpret_cast<const void*>(k_eval_three<float, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kEvalBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_eval_three(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                             int n_slices, int64_t slice_len, bool want_var, hipStream_t s) {
    if (prec == BMD_FP64)
        return launch_typed<double>(three_args<double>(p, draws_fp64(p, M, ws), partials, slice_len), n_slices,
                                    want_var, s);
    return launch_typed<float>(three_args<float>(p, draws_fp32(p, M, ws), partials, slice_len), n_slices, want_var,
                               s);
}

}  // namespace bmd
