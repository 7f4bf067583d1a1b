// Four nested populations cut from one biomarker by three cutoffs (n = 4 of
// Sec. 2.2 in the cutoff design space): design (q_1, q_2, q_3), q_1 < q_2 <
// q_3, tests the full population and {x > Phi^-1(q_i)} (fractions r_{i+1} =
// 1 - q_i), with the null correlations of Appendix A.1.  Under the step prior
// with one true cutoff tau the responders inside population i are a fraction
// 1 - max(q_i, tau) of all patients, so
//   Delta_i = b0 + b1 (1 - max(q_i, tau)) / r_i   (q = 0 for the full population)
// and the Formula 5 summand is 1 - Phi_4(z - sqrt(r_i I) Delta_i; R), Phi_4 as
// in nested_cdf.hpp with the design's own fractions.
#include <cmath>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "nested_cdf.hpp"
#include "nested_order.hpp"

namespace bmd {
namespace {

constexpr int kN4Bvn64 = 24;   // largest FP64 bivariate rule of the packed table
constexpr int kN4Bvn32 = 12;   // largest FP32 rule

// Cutoff quantiles of design g.
__device__ __forceinline__ void nested4_q(const DevProblem& P, int64_t g, double* q) {
    const int i0 = static_cast<int>(g / P.stride[0]);
    const int i1 = static_cast<int>((g / P.stride[1]) % P.m[1]);
    const int i2 = static_cast<int>(g % P.m[2]);
    q[0] = grid_coord(P.q_lo, P.q_hi, i0, P.m[0]);
    q[1] = grid_coord(P.q_lo, P.q_hi, i1, P.m[1]);
    q[2] = grid_coord(P.q_lo, P.q_hi, i2, P.m[2]);
}

// A design exists when q_1 < q_2 < q_3, the partial correlations of the
// third statistic on the second (given the first) and of the third and fourth
// (given the second) are at most 0.975, and r_3 <= 0.95 r_2: the range of the
// four-population panel and node rules.
__device__ __forceinline__ bool nested4_exists(const double* q) {
    const double r2 = 1.0 - q[0], r3 = 1.0 - q[1], r4 = 1.0 - q[2];
    return q[0] < q[1] && q[1] < q[2] && r3 * (1.0 - r2) <= 0.975 * 0.975 * r2 * (1.0 - r3) &&
           r4 * (r2 - r3) <= 0.975 * 0.975 * r3 * (r2 - r4) && r3 <= 0.95 * r2;
}

// One wavefront per design.  Rule FWER_EQUAL: z* on the FWER boundary
// 1 - Phi_4(z*, z*, z*, z*) = alpha0 by falling_root between one test at
// level alpha0 and the Bonferroni value (FP64 Phi_4 of at least 16 panels,
// its points shared by the lanes); rule BONFERRONI: z = Phi^-1(1 - alpha0 / 4).
// NaN for designs that do not exist.
__global__ __launch_bounds__(64) void k_nested4_precompute(DevProblem P, const double* __restrict__ gl,
                                                           double* __restrict__ r_out, double* __restrict__ z1_out,
                                                           double* __restrict__ z2_out, double* __restrict__ z3_out,
                                                           double* __restrict__ z4_out) {
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    double q[3];
    nested4_q(P, g, q);
    const double r2 = 1.0 - q[0], r3 = 1.0 - q[1], r4 = 1.0 - q[2];
    double z = NAN;
    if (nested4_exists(q)) {
        if (P.alpha_rule == BMD_ALPHA_BONFERRONI) {
            z = -norm_quantile(P.alpha0 / 4.0);
        } else {
            QvnConst<double, kN4Bvn64> c;
            c.init(r2, r3, r4, max(kPanelsSetup, qvn_panels<double>(r2, r3, r4)),
                   bvn_nodes_fp64(qvn_partial_rho(r2, r3, r4)), gl);
            const PanelNode nd = panel_node(gl, lane);
            auto F = [&](double x) { return (1.0 - qvn_wave(x, x, x, x, c, nd)) - P.alpha0; };
            z = falling_root(F, -norm_quantile(P.alpha0), -norm_quantile(P.alpha0 / 4.0), 4e-16);
        }
    }
    if (lane == 0) {
        r_out[g] = r2;
        z1_out[g] = z;
        z2_out[g] = z;
        z3_out[g] = z;
        z4_out[g] = z;
    }
}

// Launch order: existing designs by their FP32 work, largest first (panel
// count, then bivariate node count), ties in index order; designs that do
// not exist last, by the stable counting sort of nested_order.hpp.
constexpr int kN4Nodes = 5;   // FP32 rules of 4, 6, 8, 10 and 12 nodes
constexpr int kN4Bins = (64 - 3 + 1) * kN4Nodes + 1;

__device__ __forceinline__ int nested4_key(const DevProblem& P, const double* z, int64_t g) {
    const double zg = z[g];
    if (zg != zg) return kN4Bins - 1;
    double q[3];
    nested4_q(P, g, q);
    const double r2 = 1.0 - q[0], r3 = 1.0 - q[1], r4 = 1.0 - q[2];
    const int np = qvn_panels<float>(r2, r3, r4);
    const int nb = bvn_nodes_fp32(qvn_partial_rho(r2, r3, r4));
    return kN4Bins - 2 - ((np - 3) * kN4Nodes + (nb - 4) / 2);
}

__global__ __launch_bounds__(1024) void k_order_nested4(DevProblem P, const double* __restrict__ z,
                                                        int32_t* __restrict__ order) {
    order_by_key<kN4Bins>(P.G, [&](int64_t g) { return nested4_key(P, z, g); }, order);
}

template <typename T>
struct Nested4Args {
    DevProblem P;
    const double* z;        // [G] the common critical value (NaN: no design)
    const int32_t* order;   // [G] launch order (k_order_nested4)
    const T* b0;
    const T* b1;
    const T* tau;           // [M] true cutoff quantile
    int64_t M;
    int64_t slice_len;
    double* partials;       // [n_slices][2][G]: sums, then sums of squares (VAR only)
    const double* gl;
};

// One thread per design in the launch order: tile blockIdx.y of kEvalBlock
// designs, the draws of slice blockIdx.x (slices along x: every XCD gets each
// tile, the costliest start first).  Panels and bivariate nodes are the
// wavefront's largest; the Phi_4 constants are the lane's own.  Wavefronts
// whose designs all do not exist write NaN sums and leave.
template <typename T, int NB, bool VAR>
__global__ __launch_bounds__(kEvalBlock) void k_eval_nested4(Nested4Args<T> a) {
    const int64_t G = a.P.G;
    const int64_t idx = static_cast<int64_t>(blockIdx.y) * kEvalBlock + threadIdx.x;
    const bool valid = idx < G;
    const int64_t g = a.order[valid ? idx : G - 1];
    const int slice = blockIdx.x;
    const double zd = a.z[g];
    if (__all(!valid || zd != zd)) {
        if (valid) {
            double* out = a.partials + static_cast<int64_t>(slice) * 2 * G;
            out[g] = zd;
            if constexpr (VAR) out[G + g] = zd;
        }
        return;
    }
    double q[3];
    nested4_q(a.P, g, q);
    const bool exists = zd == zd;
    if (!exists) {   // a harmless stand-in, its sums replaced by NaN
        q[0] = 0.3;
        q[1] = 0.5;
        q[2] = 0.7;
    }
    const double r2 = 1.0 - q[0], r3 = 1.0 - q[1], r4 = 1.0 - q[2];
    const double rho = qvn_partial_rho(r2, r3, r4);
    const int np = wave_max_i32(qvn_panels<T>(r2, r3, r4));
    const int nb = wave_max_i32(sizeof(T) == 8 ? bvn_nodes_fp64(rho) : bvn_nodes_fp32(rho));
    QvnConst<T, NB, false> c;
    c.init(r2, r3, r4, np, nb, a.gl);
    const T z = static_cast<T>(exists ? zd : 2.0);
    const T s1 = static_cast<T>(a.P.sqrtI), s2 = static_cast<T>(sqrt(r2 * a.P.info)),
            s3 = static_cast<T>(sqrt(r3 * a.P.info)), s4 = static_cast<T>(sqrt(r4 * a.P.info));
    const T ir2 = static_cast<T>(1.0 / r2), ir3 = static_cast<T>(1.0 / r3), ir4 = static_cast<T>(1.0 / r4);
    const T tq1 = static_cast<T>(q[0]), tq2 = static_cast<T>(q[1]), tq3 = static_cast<T>(q[2]);
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(a.M, kb + a.slice_len);
    double sum1 = 0.0, sum2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const T b0 = a.b0[k], b1 = a.b1[k], tau = a.tau[k];
        const T h1 = z - s1 * (b0 + b1 * (T(1) - tau));
        const T h2 = z - s2 * (b0 + b1 * (T(1) - fmax(tq1, tau)) * ir2);
        const T h3 = z - s3 * (b0 + b1 * (T(1) - fmax(tq2, tau)) * ir3);
        const T h4 = z - s4 * (b0 + b1 * (T(1) - fmax(tq3, tau)) * ir4);
        const double v = static_cast<double>(T(1) - qvn(h1, h2, h3, h4, c));
        sum1 += v;
        if constexpr (VAR) sum2 = fma(v, v, sum2);
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(slice) * 2 * G;
        out[g] = exists ? sum1 : zd;
        if constexpr (VAR) out[G + g] = exists ? sum2 : zd;
    }
}

template <typename T, int NB>
hipError_t launch_typed(const bmd_problem* p, const DrawArrays<T>& D, double* partials, int n_slices,
                        int64_t slice_len, bool var, hipStream_t s) {
    Nested4Args<T> a{};
    a.P = p->P;
    a.z = p->d_z4;
    a.order = p->d_order;
    a.b0 = D.b0;
    a.b1 = D.b1;
    a.tau = D.tauT;
    a.M = D.M;
    a.slice_len = slice_len;
    a.partials = partials;
    a.gl = p->d_gl;
    const void* k = var ? reinterpret_cast<const void*>(k_eval_nested4<T, NB, true>)
                        : reinterpret_cast<const void*>(k_eval_nested4<T, NB, false>);
    void* args[] = {&a};
    const int64_t tiles = (p->P.G + kEvalBlock - 1) / kEvalBlock;
    if (tiles > kNested3MaxTiles) return hipErrorInvalidConfiguration;   // creation keeps G within this
    return hipLaunchKernel(k, dim3(static_cast<unsigned>(n_slices), static_cast<unsigned>(tiles)), dim3(kEvalBlock),
                           args, 0, s);
}

}  // namespace

hipError_t launch_nested4_precompute(const bmd_problem* p, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_nested4_precompute, dim3(static_cast<unsigned>(G)), dim3(64), 0, s, p->P, p->d_gl, p->d_r,
                       p->d_z1, p->d_z2, p->d_z3, p->d_z4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_nested4, dim3(1), dim3(1024), 0, s, p->P, p->d_z4, p->d_order);
    return hipGetLastError();
}

int nested4_blocks_per_cu(int prec) {
    const void* k = prec == BMD_FP64 ? reinterpret_cast<const void*>(k_eval_nested4<double, kN4Bvn64, false>)
                                     : reinterpret_cast<const void*>(k_eval_nested4<float, kN4Bvn32, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kEvalBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_eval_nested4(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                               int n_slices, int64_t slice_len, bool want_var, hipStream_t s) {
    if (prec == BMD_FP64)
        return launch_typed<double, kN4Bvn64>(p, draws_fp64(p, M, ws), partials, n_slices, slice_len, want_var, s);
    return launch_typed<float, kN4Bvn32>(p, draws_fp32(p, M, ws), partials, n_slices, slice_len, want_var, s);
}

}  // namespace bmd
