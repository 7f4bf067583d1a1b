// Three nested populations cut from one biomarker by two cutoffs (n = 3 of
// Sec. 2.2 in the cutoff design space): design (q_1, q_2), q_1 < q_2, tests
// the full population, {x > Phi^-1(q_1)} (fraction r_2 = 1 - q_1) and
// {x > Phi^-1(q_2)} (r_3 = 1 - q_2), with the null correlations of Appendix
// A.1.  Under the step prior with one true cutoff tau the responders inside
// population i are a fraction 1 - max(q_i, tau) of all patients, so
//   Delta_i = b0 + b1 (1 - max(q_i, tau)) / r_i   (q_1 = 0 for the full population)
// and the Formula 5 summand is 1 - Phi_3(z - sqrt(r_i I) Delta_i; R), Phi_3 as
// in nested_cdf.hpp with the design's own fractions.
#include <cmath>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "nested_cdf.hpp"
#include "nested_order.hpp"

namespace bmd {
namespace {

// Cutoff quantiles of design g.
__device__ __forceinline__ void nested3_q(const DevProblem& P, int64_t g, double* q1, double* q2) {
    const int i0 = static_cast<int>(g / P.stride[0]);
    const int i1 = static_cast<int>(g - static_cast<int64_t>(i0) * P.stride[0]);
    *q1 = grid_coord(P.q_lo, P.q_hi, i0, P.m[0]);
    *q2 = grid_coord(P.q_lo, P.q_hi, i1, P.m[1]);
}

// A design exists when q_1 < q_2 and the partial correlation of the third
// statistic on the second given the first, sqrt(r_3 (1 - r_2) / (r_2 (1 - r_3))),
// is at most 0.975 (the range of the panel rule).  Rule FWER_EQUAL: one z* for
// the three tests on the FWER boundary 1 - Phi_3(z*, z*, z*) = alpha0, by
// falling_root between one test at level alpha0 and the Bonferroni value
// (FP64 Phi_3 of at least 16 panels shared by the wavefront's lanes, one
// wavefront per design); rule BONFERRONI: z = Phi^-1(1 - alpha0 / 3).  NaN for
// designs that do not exist.
__global__ __launch_bounds__(64) void k_nested3_precompute(DevProblem P, const double* __restrict__ gl,
                                                           double* __restrict__ r_out, double* __restrict__ z1_out,
                                                           double* __restrict__ z2_out,
                                                           double* __restrict__ z3_out) {
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    double q1, q2;
    nested3_q(P, g, &q1, &q2);
    const double r2 = 1.0 - q1, r3 = 1.0 - q2;
    double z = NAN;
    if (q1 < q2 && r3 * (1.0 - r2) <= 0.975 * 0.975 * r2 * (1.0 - r3)) {
        if (P.alpha_rule == BMD_ALPHA_BONFERRONI) {
            z = -norm_quantile(P.alpha0 / 3.0);
        } else {
            TvnConst<double> c;
            c.init(r2, r3, max(kPanelsSetup, tvn_panels<double>(r2, r3)), gl);
            const PanelNode nd = panel_node(gl, lane);
            auto F = [&](double x) { return (1.0 - tvn_wave(x, x, x, c, nd)) - P.alpha0; };
            z = falling_root(F, -norm_quantile(P.alpha0), -norm_quantile(P.alpha0 / 3.0), 4e-16);
        }
    }
    if (lane == 0) {
        r_out[g] = r2;
        z1_out[g] = z;
        z2_out[g] = z;
        z3_out[g] = z;
    }
}

// Launch order of the designs.  The sweep runs every lane of a wavefront
// with the wavefront's largest panel count, and along a row of the grid the
// count falls from dozens of panels (q_2 just above q_1) to three, so index
// order wastes most of the work.  Existing designs are sorted by their panel
// counts, largest first, ties in index order, and designs that do not exist
// go last.  The FP32 and FP64 counts both fall as the smaller conditional
// scale grows, so each step along that scale raises one of them or both:
// their sum (offset to start at 0) orders the designs by both at once.
constexpr int kOrderBins = (64 - 3) + (128 - 8) + 2;   // sums 0..181, then "does not exist"

__device__ __forceinline__ int nested3_key(const DevProblem& P, const double* z, int64_t g) {
    const double zg = z[g];
    if (zg != zg) return kOrderBins - 1;
    double q1, q2;
    nested3_q(P, g, &q1, &q2);
    return kOrderBins - 2 - ((tvn_panels<float>(1.0 - q1, 1.0 - q2) - 3) + (tvn_panels<double>(1.0 - q1, 1.0 - q2) - 8));
}

// The stable counting sort of nested_order.hpp (one workgroup of 16 wavefronts).
__global__ __launch_bounds__(1024) void k_order_nested3(DevProblem P, const double* __restrict__ z,
                                                        int32_t* __restrict__ order) {
    order_by_key<kOrderBins>(P.G, [&](int64_t g) { return nested3_key(P, z, g); }, order);
}

template <typename T>
struct Nested3Args {
    DevProblem P;
    const double* z;        // [G] the common critical value (NaN: no design)
    const int32_t* order;   // [G] launch order (k_order_nested3)
    const T* b0;
    const T* b1;
    const T* tau;           // [M] true cutoff quantile
    int64_t M;
    int64_t slice_len;
    double* partials;       // [n_slices][2][G]: sums, then sums of squares (VAR only)
    const double* gl;
};

// One thread per design in the launch order above: tile blockIdx.y of
// kEvalBlock designs, the draws of slice blockIdx.x.  The panel count is the
// wavefront's largest (every lane runs the same node count), the Phi_3
// constants are the lane's own.  Wavefronts whose designs all do not exist
// write NaN sums and leave.  Workgroups are dispatched in linear order, x
// fastest, and go to the XCDs round-robin: with the slices along x every XCD
// gets every tile equally often, and the costliest tiles (the order's first)
// start first, so the last workgroups to run are the cheapest.
template <typename T, bool VAR>
__global__ __launch_bounds__(kEvalBlock) void k_eval_nested3(Nested3Args<T> a) {
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
    double q1, q2;
    nested3_q(a.P, g, &q1, &q2);
    // lanes without a design compute with a harmless stand-in, then write NaN
    const bool exists = zd == zd;
    if (!exists) {
        q1 = 0.3;
        q2 = 0.6;
    }
    const double r2 = 1.0 - q1, r3 = 1.0 - q2;
    TvnConst<T, false> c;
    c.init(r2, r3, wave_max_i32(tvn_panels<T>(r2, r3)), a.gl);
    const T z = static_cast<T>(exists ? zd : 2.0);
    const T s1 = static_cast<T>(a.P.sqrtI), s2 = static_cast<T>(sqrt(r2 * a.P.info)),
            s3 = static_cast<T>(sqrt(r3 * a.P.info));
    const T ir2 = static_cast<T>(1.0 / r2), ir3 = static_cast<T>(1.0 / r3);
    const T tq1 = static_cast<T>(q1), tq2 = static_cast<T>(q2);
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(a.M, kb + a.slice_len);
    double sum1 = 0.0, sum2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const T b0 = a.b0[k], b1 = a.b1[k], tau = a.tau[k];
        const T h1 = z - s1 * (b0 + b1 * (T(1) - tau));
        const T h2 = z - s2 * (b0 + b1 * (T(1) - fmax(tq1, tau)) * ir2);
        const T h3 = z - s3 * (b0 + b1 * (T(1) - fmax(tq2, tau)) * ir3);
        const double v = static_cast<double>(T(1) - tvn(h1, h2, h3, c));
        sum1 += v;
        if constexpr (VAR) sum2 = fma(v, v, sum2);
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(slice) * 2 * G;
        out[g] = exists ? sum1 : zd;
        if constexpr (VAR) out[G + g] = exists ? sum2 : zd;
    }
}

template <typename T>
hipError_t launch_typed(const bmd_problem* p, const DrawArrays<T>& D, double* partials, int n_slices,
                        int64_t slice_len, bool var, hipStream_t s) {
    Nested3Args<T> a{};
    a.P = p->P;
    a.z = p->d_z3;
    a.order = p->d_order;
    a.b0 = D.b0;
    a.b1 = D.b1;
    a.tau = D.tauT;
    a.M = D.M;
    a.slice_len = slice_len;
    a.partials = partials;
    a.gl = p->d_gl;
    const void* k = var ? reinterpret_cast<const void*>(k_eval_nested3<T, true>)
                        : reinterpret_cast<const void*>(k_eval_nested3<T, false>);
    void* args[] = {&a};
    const int64_t tiles = (p->P.G + kEvalBlock - 1) / kEvalBlock;
    if (tiles > kNested3MaxTiles) return hipErrorInvalidConfiguration;   // creation keeps G within this
    return hipLaunchKernel(k, dim3(static_cast<unsigned>(n_slices), static_cast<unsigned>(tiles)),
                           dim3(kEvalBlock), args, 0, s);
}

}  // namespace

hipError_t launch_nested3_precompute(const bmd_problem* p, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_nested3_precompute, dim3(static_cast<unsigned>(G)), dim3(64), 0, s, p->P,
                       p->d_gl, p->d_r, p->d_z1, p->d_z2, p->d_z3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_nested3, dim3(1), dim3(1024), 0, s, p->P, p->d_z3, p->d_order);
    return hipGetLastError();
}

int nested3_blocks_per_cu(int prec) {
    const void* k = prec == BMD_FP64 ? reinterpret_cast<const void*>(k_eval_nested3<double, false>)
                                     : reinterpret_cast<const void*>(k_eval_nested3<float, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kEvalBlock, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_eval_nested3(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                               int n_slices, int64_t slice_len, bool want_var, hipStream_t s) {
    if (prec == BMD_FP64) return launch_typed<double>(p, draws_fp64(p, M, ws), partials, n_slices, slice_len, want_var, s);
    return launch_typed<float>(p, draws_fp32(p, M, ws), partials, n_slices, slice_len, want_var, s);
}

}  // namespace bmd
