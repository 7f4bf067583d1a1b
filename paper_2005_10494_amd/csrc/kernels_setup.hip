// Per-design and per-draw setup kernels: grid coordinates, subgroup fractions,
// critical values (Formula 2), axis tables, and the prior draws of Formula 5.
#include <cstring>

#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {
namespace {

// Decode a row-major grid index (axis 0 slowest).
// Coordinate of grid index i on axis j: the subgroup-fraction axis of the
// alpha design space, else a cutoff quantile (or the alpha_1 axis).
__device__ __forceinline__ double axis_coord(const DevProblem& P, int j, int i) {
    if (P.design_space == BMD_DESIGN_ALPHA && P.d == 2 && j == 0) return grid_coord(P.r_lo, P.r_hi, i, P.m[0]);
    return grid_coord(P.q_lo, P.q_hi, i, P.m[j]);
}

__device__ __forceinline__ void decode(const DevProblem& P, int64_t g, int* idx) {
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        if (j < P.d) {
            const int64_t s = P.stride[j];
            idx[j] = static_cast<int>(g / s);
            g -= static_cast<int64_t>(idx[j]) * s;
        }
    }
}

// Equicorrelated orthant probability P(X_j > v_j, j < d) through the one-factor
// representation, integrated over the common factor with a Gauss-Hermite rule.
__device__ double orthant_gh(const DevProblem& P, const double* v, const double* __restrict__ gh,
                             int K) {
    const double* x = gh;
    const double* w = gh + K;
    double acc = 0.0;
    for (int m = 0; m < K; ++m) {
        double prod = w[m];
        const double t = P.sr * x[m];
        for (int j = 0; j < P.d; ++j) prod *= norm_cdf((t - v[j]) / P.sq);
        acc += prod;
    }
    return acc;
}

// Phi_2 with the largest Gauss-Legendre rule (setup-time accuracy, FP64).
__device__ double bvn_setup(double h, double k, double rho, const double* __restrict__ gl) {
    const int n = 24;
    const double* x = gl + gl_offset(n);
    const double* w = x + n;
    const double th = asin(rho);
    const double hk = h * k, hs = 0.5 * (h * h + k * k);
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        const double s = sin(0.5 * th * (1.0 + x[i]));
        const double a = 1.0 / ((1.0 - s) * (1.0 + s));
        acc += w[i] * exp(a * (s * hk - hs));
    }
    return norm_cdf(h) * norm_cdf(k) + th * 0.079577471545947667884 * acc;
}

// Common critical value with family-wise error alpha0 at null correlation
// rho (Formula 2 for two tests): F(z) = 2 Phi(-z) - Phi_2(-z, -z; rho) - alpha0
// is decreasing; safeguarded Newton inside [z(alpha0), z(alpha0/2)] with
// F'(z) = -2 phi(z) Phi(z sqrt((1 - rho)/(1 + rho))).
__device__ double zstar(double rho, double alpha0, const double* __restrict__ gl) {
    double lo = -norm_quantile(alpha0), hi = -norm_quantile(0.5 * alpha0);
    double z = 0.5 * (lo + hi);
    const double c = sqrt((1.0 - rho) / (1.0 + rho));
    for (int it = 0; it < 60; ++it) {
        const double F = 2.0 * norm_cdf(-z) - bvn_setup(-z, -z, rho, gl) - alpha0;
        if (F > 0.0) lo = z; else hi = z;
        const double dF = -2.0 * norm_pdf(z) * norm_cdf(z * c);
        double zn = z - F / dF;
        if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
        const double step = fabs(zn - z);
        z = zn;
        if (step <= 4e-16 * z || hi - lo <= 4e-16 * z) break;
    }
    return z;
}

// Second critical value on the FWER boundary given the first (Formula 2 for
// two nested tests): FWER(z2) = Phi(-z1) + Phi(-z2) - Phi_2(-z1, -z2; rho) =
// alpha0, which falls in z2 with derivative -phi(z2) Phi((z1 - rho z2) /
// sqrt(1 - rho^2)).  Newton steps inside the bracket [level alpha0 for the
// second test alone, level alpha0 - alpha_1 (the union bound)], bisection when
// a step leaves it.  Needs alpha_1 = Phi(-z1) < alpha0.
__device__ double z2_on_fwer(double z1, double rho, double alpha0, const double* __restrict__ gl) {
    const double a1 = norm_cdf(-z1);
    double lo = -norm_quantile(alpha0), hi = -norm_quantile(alpha0 - a1);
    double z = 0.5 * (lo + hi);
    const double c = 1.0 / sqrt((1.0 - rho) * (1.0 + rho));
    for (int it = 0; it < 60; ++it) {
        const double F = a1 + norm_cdf(-z) - bvn_setup(-z1, -z, rho, gl) - alpha0;
        if (F > 0.0) lo = z; else hi = z;
        const double dF = -norm_pdf(z) * norm_cdf((z1 - rho * z) * c);
        double zn = z - F / dF;
        if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
        const double step = fabs(zn - z);
        z = zn;
        if (step <= 4e-16 * fabs(z) || hi - lo <= 4e-16 * fabs(z)) break;
    }
    return z;
}

__global__ __launch_bounds__(128) void k_design_precompute(DevProblem P, const double* __restrict__ ghp, int Kp,
                                    const double* __restrict__ gl, double* __restrict__ r_out,
                                    double* __restrict__ z1_out, double* __restrict__ z2_out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= P.G) return;
    int idx[kMaxDim];
    decode(P, g, idx);
    if (P.design_space == BMD_DESIGN_ALPHA) {
        // (r_2, alpha_1) or alpha_1 at r_2 = r_lo; alpha_2 on the FWER boundary
        const double r = P.d == 2 ? axis_coord(P, 0, idx[0]) : P.r_lo;
        const double z1 = -norm_quantile(axis_coord(P, P.d - 1, idx[P.d - 1]));
        r_out[g] = r;
        z1_out[g] = z1;
        z2_out[g] = z2_on_fwer(z1, sqrt(r), P.alpha0, gl);
        return;
    }
    double c[kMaxDim];
    double r;
    if (P.d == 1) {
        r = 1.0 - grid_coord(P.q_lo, P.q_hi, idx[0], P.m[0]);
    } else {
        for (int j = 0; j < P.d; ++j) c[j] = norm_quantile(grid_coord(P.q_lo, P.q_hi, idx[j], P.m[j]));
        r = orthant_gh(P, c, ghp, Kp);
    }
    r_out[g] = r;
    if (P.alpha_rule == BMD_ALPHA_FWER_EQUAL) {
        const double z = zstar(sqrt(r), P.alpha0, gl);
        z1_out[g] = z;
        z2_out[g] = z;
    } else if (P.alpha_rule == BMD_ALPHA_SPLIT) {
        z1_out[g] = P.zf1;
        z2_out[g] = z2_on_fwer(P.zf1, sqrt(r), P.alpha0, gl);
    } else {
        z1_out[g] = P.zf1;
        z2_out[g] = P.zf2;
    }
}

// Critical values of one level split for every design: z1 given, z2 on the
// design's FWER boundary (its r from the precompute).
__global__ __launch_bounds__(128) void k_levels_z(int64_t G, double z1, double alpha0, const double* __restrict__ r,
                                                  const double* __restrict__ gl, double* __restrict__ z1_out,
                                                  double* __restrict__ z2_out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    z1_out[g] = z1;
    z2_out[g] = z2_on_fwer(z1, sqrt(r[g]), alpha0, gl);
}

// Golden-section search of the first level per design (the level split of
// Sec. 2.4 searched, second level on the design's FWER boundary), one call
// between consecutive sweeps.  st holds [8][G]: bracket ends a, b, interior
// points x1 < x2, their estimates f1, f2, the best estimate seen and its
// level; side[g] names the point the last sweep evaluated (1: x1, 2: x2,
// 3: a_lo, 4: a_hi).  Phase 0 sets the bracket and probes x1; phase 1 records
// f(x1) and probes x2; every later phase records the probe and keeps the best,
// then (when `probe`) either drops the part beyond the lower interior point
// (ties keep the left part) and probes the new point (end = 0), or probes the
// range's end a_lo (end = 1) or a_hi (end = 2).  A probe writes the design's
// z1 and z2.
__global__ __launch_bounds__(128) void k_levels_golden(int64_t G, int phase, bool probe, int end, double a_lo,
                                                       double a_hi,
                                                       double alpha0, const double* __restrict__ r,
                                                       const double* __restrict__ mean, const double* __restrict__ gl,
                                                       double* __restrict__ st, int32_t* __restrict__ side,
                                                       double* __restrict__ z1_out, double* __restrict__ z2_out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    constexpr double gr = 0.61803398874989484820;   // (sqrt 5 - 1) / 2
    double* A = st;
    double* B = st + G;
    double* X1 = st + 2 * G;
    double* X2 = st + 3 * G;
    double* F1 = st + 4 * G;
    double* F2 = st + 5 * G;
    double* best = st + 6 * G;
    double* best_x = st + 7 * G;
    double next = 0.0;
    if (phase == 0) {
        A[g] = a_lo;
        B[g] = a_hi;
        X1[g] = a_hi - gr * (a_hi - a_lo);
        X2[g] = a_lo + gr * (a_hi - a_lo);
        side[g] = 1;
        next = X1[g];
    } else {
        const double f = mean[g];
        const int sd = side[g];
        const double x = sd == 1 ? X1[g] : sd == 2 ? X2[g] : sd == 3 ? a_lo : a_hi;
        if (sd == 1) F1[g] = f;
        if (sd == 2) F2[g] = f;
        if (phase == 1) {
            best[g] = f;
            best_x[g] = x;
            side[g] = 2;
            next = X2[g];
        } else {
            if (f > best[g]) {
                best[g] = f;
                best_x[g] = x;
            }
            if (probe && end != 0) {
                side[g] = 2 + end;
                next = end == 1 ? a_lo : a_hi;
            } else if (probe) {
                if (F1[g] >= F2[g]) {   // the maximum lies in [a, x2]
                    B[g] = X2[g];
                    X2[g] = X1[g];
                    F2[g] = F1[g];
                    X1[g] = B[g] - gr * (B[g] - A[g]);
                    side[g] = 1;
                    next = X1[g];
                } else {                // in [x1, b]
                    A[g] = X1[g];
                    X1[g] = X2[g];
                    F1[g] = F2[g];
                    X2[g] = A[g] + gr * (B[g] - A[g]);
                    side[g] = 2;
                    next = X2[g];
                }
            }
        }
    }
    if (probe) {
        const double z1 = -norm_quantile(next);
        z1_out[g] = z1;
        z2_out[g] = z2_on_fwer(z1, sqrt(r[g]), alpha0, gl);
    }
}

// Derivative-driven search of the first level per design (the level split of
// Sec. 2.4, second level on the design's FWER boundary; the smoothness of
// Appendix A.3 makes the shared-draw estimate a smooth function of alpha_1
// with a derivative the sweep returns): a root of the derivative inside
// [a_lo, a_hi] by the Illinois variant of false position, one call between
// consecutive derivative sweeps.  st holds [9][G]: bracket ends lo, hi,
// derivatives there glo, ghi, the probed level x, the best estimate seen and
// its level, the side kept last (+1 lo, -1 hi, 0 none) and a done flag.
// Phase 0 probes a_lo, phase 1 records it and probes a_hi, phase 2 records
// it and decides: a derivative <= 0 at a_lo or >= 0 at a_hi puts the maximum
// at that end (done), otherwise false position starts; every later phase
// records the probe, keeps the best and moves one end.  A probe writes the
// design's z1 and z2; a finished design probes its best level again.
__global__ __launch_bounds__(128) void k_levels_newton(int64_t G, int phase, double a_lo, double a_hi, double tol,
                                                       double alpha0, const double* __restrict__ r,
                                                       const double* __restrict__ mean,
                                                       const double* __restrict__ dmean,
                                                       const double* __restrict__ gl, double* __restrict__ st,
                                                       double* __restrict__ z1_out, double* __restrict__ z2_out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double* LO = st;
    double* HI = st + G;
    double* GLO = st + 2 * G;
    double* GHI = st + 3 * G;
    double* X = st + 4 * G;
    double* best = st + 5 * G;
    double* best_x = st + 6 * G;
    double* kept = st + 7 * G;
    double* done = st + 8 * G;
    double next = 0.0;
    if (phase == 0) {
        LO[g] = a_lo;
        HI[g] = a_hi;
        kept[g] = 0.0;
        done[g] = 0.0;
        next = a_lo;
    } else {
        const double f = mean[g], d = dmean[g], x = X[g];
        if (phase == 1 || f > best[g]) {
            best[g] = f;
            best_x[g] = x;
        }
        if (phase == 1) {
            GLO[g] = d;
            next = a_hi;
        } else if (phase == 2) {
            GHI[g] = d;
            if (GLO[g] <= 0.0 || GHI[g] >= 0.0) done[g] = 1.0;   // the maximum sits at an end
        } else if (done[g] == 0.0) {
            // the root lies where the derivative changes sign
            if (d > 0.0) {
                LO[g] = x;
                GLO[g] = d;
                if (kept[g] == -1.0) GHI[g] *= 0.5;
                kept[g] = -1.0;
            } else {
                HI[g] = x;
                GHI[g] = d;
                if (kept[g] == 1.0) GLO[g] *= 0.5;
                kept[g] = 1.0;
            }
            if (d == 0.0 || HI[g] - LO[g] <= tol) done[g] = 1.0;
        }
        if (phase >= 2) {
            if (done[g] != 0.0) {
                next = best_x[g];
            } else {
                next = (LO[g] * GHI[g] - HI[g] * GLO[g]) / (GHI[g] - GLO[g]);
                if (!(next > LO[g] && next < HI[g])) next = 0.5 * (LO[g] + HI[g]);
            }
        }
    }
    X[g] = next;
    const double z1 = -norm_quantile(next);
    z1_out[g] = z1;
    z2_out[g] = z2_on_fwer(z1, sqrt(r[g]), alpha0, gl);
}

// Running maximum over levels: level k's means against the best so far
// (k = 0 initialises); strict improvement only, so ties keep the lower k.
__global__ void k_levels_best(int64_t G, int k, const double* __restrict__ mean, double* __restrict__ best,
                              int32_t* __restrict__ best_k) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const double m = mean[g];
    if (k == 0 || m > best[g]) {
        best[g] = m;
        if (best_k) best_k[g] = k;
    }
}

// A[(j*K + m)*mmax + i] = w_m^[j==0] Phi((sqrt(rho) x_m - c_{j,i}) / sqrt(1-rho)).
template <typename T>
__global__ void k_axis_tables(DevProblem P, const double* __restrict__ gh, int K, T* __restrict__ A) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = static_cast<int64_t>(P.d) * K * P.mmax;
    if (t >= total) return;
    const int i = static_cast<int>(t % P.mmax);
    const int m = static_cast<int>((t / P.mmax) % K);
    const int j = static_cast<int>(t / (static_cast<int64_t>(P.mmax) * K));
    double v = 0.0;
    if (i < P.m[j]) {
        const double c = norm_quantile(grid_coord(P.q_lo, P.q_hi, i, P.m[j]));
        v = norm_cdf((P.sr * gh[m] - c) / P.sq);
        if (j == 0) v *= gh[K + m];
    }
    A[t] = static_cast<T>(v);
}

// Number of grid indices i in [0, m) with q_i <= tau (the grid is nondecreasing).
__device__ __forceinline__ int32_t count_le(const DevProblem& P, int j, double tau) {
    int lo = 0, hi = P.m[j];   // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (grid_coord(P.q_lo, P.q_hi, mid, P.m[j]) <= tau) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Prior draw k (Formula 5's Delta^(k)) into slot kk of the per-draw arrays.
template <typename T>
__device__ __forceinline__ void draw_one(const DevProblem& P, const double* __restrict__ gh, int K, uint64_t k,
                                         int64_t kk, int64_t M, const DrawArrays<T>& D) {
    double u[8];
    draw_uniforms<8>(k, P.scenario, P.key0, P.key1, P.n_uniform, u);
    if (P.effect == BMD_EFFECT_STEP) {
        const double b0 = P.mu_b0 + P.sd_b0 * norm_quantile(u[0]);
        const double b1 = P.mu_b1 + P.sd_b1 * norm_quantile(u[1]);
        double t[kMaxDim];
        // two cutoffs on one biomarker: one true cutoff per draw
        const int nbio = (P.design_space == BMD_DESIGN_NESTED3 || P.design_space == BMD_DESIGN_NESTED4) ? 1 : P.d;
        for (int j = 0; j < nbio; ++j) {
            const double tau = affine_uniform(P.tau_lo, P.tau_hi, u[2 + j]);
            t[j] = norm_quantile(tau);
            D.tau[j * M + kk] = tau;
            if (P.G > 0) D.thr[kk * P.d + j] = count_le(P, j, tau);
        }
        double PR;
        if (nbio == 1) {
            PR = 1.0 - D.tau[kk];
        } else {
            PR = 0.0;
            T* B = D.B + static_cast<int64_t>(kk) * P.d * K;
            for (int m = 0; m < K; ++m) {
                double prod = gh[K + m];
                const double s = P.sr * gh[m];
                for (int j = 0; j < P.d; ++j) {
                    const double v = norm_cdf((s - t[j]) / P.sq);
                    B[m * P.d + j] = static_cast<T>(j == 0 ? gh[K + m] * v : v);
                    prod *= v;
                }
                PR += prod;
            }
        }
        D.b0[kk] = static_cast<T>(b0);
        D.b1[kk] = static_cast<T>(b1);
        D.PR[kk] = static_cast<T>(PR);
        D.mu1[kk] = static_cast<T>(P.sqrtI * (b0 + b1 * PR));
        D.tauT[kk] = static_cast<T>(D.tau[kk]);
        D.q4[4 * kk + 0] = D.b0[kk];
        D.q4[4 * kk + 1] = D.b1[kk];
        D.q4[4 * kk + 2] = D.mu1[kk];
        D.q4[4 * kk + 3] = T(0);
    } else {
        const double e1 = norm_quantile(u[0]);
        const double e2 = norm_quantile(u[1]);
        D.e1[kk] = static_cast<T>(e1);
        D.e2[kk] = static_cast<T>(e2);
        if (P.n_uniform >= 3) D.e3[kk] = static_cast<T>(norm_quantile(u[2]));
        if (P.n_uniform >= 4) D.e4[kk] = static_cast<T>(norm_quantile(u[3]));
        D.mu1[kk] = static_cast<T>(P.sqrtI * (P.th1 + P.sg1 * e1));
    }
}

// One prior draw per thread.
template <typename T>
__global__ __launch_bounds__(128) void k_draws(DevProblem P, const double* __restrict__ gh, int K, uint64_t k0, int64_t M,
                        DrawArrays<T> D) {
    const int64_t kk = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (kk >= M) return;
    draw_one<T>(P, gh, K, k0 + static_cast<uint64_t>(kk), kk, M, D);
}

// Draws of many problems in one launch: thread t takes draw t - first[s] of the
// last job s with first[s] <= t (jobs in increasing order of first).
template <typename T>
__global__ __launch_bounds__(128) void k_draws_batch(const DrawJob<T>* __restrict__ jobs, int n_jobs, int64_t total) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first <= t) lo = mid; else hi = mid - 1;
    }
    const DrawJob<T>& j = jobs[lo];
    const int64_t kk = t - j.first;
    draw_one<T>(j.P, j.gh, j.K, static_cast<uint64_t>(kk), kk, j.D.M, j.D);
}

__global__ __launch_bounds__(128) void k_inspect_draws(DevProblem P, const double* __restrict__ gh, int K, uint64_t k0,
                                int64_t n, double* __restrict__ u_out, double* __restrict__ f_out) {
    const int64_t kk = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (kk >= n) return;
    double u[8];
    for (int i = 0; i < 8; ++i) u[i] = 0.0;
    draw_uniforms<8>(k0 + static_cast<uint64_t>(kk), P.scenario, P.key0, P.key1, P.n_uniform, u);
    double* f = f_out + kk * BMD_DRAW_FIELDS;
    for (int i = 0; i < BMD_DRAW_FIELDS; ++i) f[i] = 0.0;
    for (int i = 0; i < 8; ++i) u_out[kk * 8 + i] = u[i];
    if (P.effect == BMD_EFFECT_STEP) {
        f[0] = P.mu_b0 + P.sd_b0 * norm_quantile(u[0]);
        f[1] = P.mu_b1 + P.sd_b1 * norm_quantile(u[1]);
        double t[kMaxDim];
        const int nbio = (P.design_space == BMD_DESIGN_NESTED3 || P.design_space == BMD_DESIGN_NESTED4) ? 1 : P.d;
        for (int j = 0; j < nbio; ++j) {
            const double tau = affine_uniform(P.tau_lo, P.tau_hi, u[2 + j]);
            t[j] = norm_quantile(tau);
            f[5 + j] = tau;
            f[11 + j] = t[j];
        }
        f[2] = nbio == 1 ? 1.0 - f[5] : orthant_gh(P, t, gh, K);
    } else {
        f[3] = norm_quantile(u[0]);
        f[4] = norm_quantile(u[1]);
        if (P.n_uniform >= 3) f[5] = norm_quantile(u[2]);
        if (P.n_uniform >= 4) f[6] = norm_quantile(u[3]);
    }
}

__global__ __launch_bounds__(128) void k_inspect_designs(DevProblem P, int64_t g0, int64_t n, const double* __restrict__ r,
                                  const double* __restrict__ z1, const double* __restrict__ z2,
                                  const double* __restrict__ z3, const double* __restrict__ z4,
                                  double* __restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t g = g0 + t;
    int idx[kMaxDim];
    decode(P, g, idx);
    double* f = out + t * BMD_DESIGN_FIELDS;
    for (int i = 0; i < BMD_DESIGN_FIELDS; ++i) f[i] = 0.0;
    for (int j = 0; j < P.d; ++j) {
        f[j] = axis_coord(P, j, idx[j]);
        f[6 + j] = P.design_space == BMD_DESIGN_CUTOFFS ? norm_quantile(f[j]) : 0.0;
    }
    if (P.design_space == BMD_DESIGN_ALPHA3) {
        f[6] = P.r_hi;
        f[7] = z3[g];
    } else if (P.design_space == BMD_DESIGN_NESTED3) {
        f[6] = 1.0 - f[1];   // r_3
        f[7] = z3[g];
    } else if (P.design_space == BMD_DESIGN_NESTED4) {
        f[6] = 1.0 - f[1];   // r_3
        f[7] = z3[g];
        f[8] = 1.0 - f[2];   // r_4
        f[9] = z4[g];
    } else if (P.design_space == BMD_DESIGN_ALPHA4) {
        f[6] = P.r_hi;
        f[7] = z3[g];
        f[8] = P.r_4;
        f[9] = z4[g];
    }
    f[12] = r[g];
    f[13] = sqrt(r[g]);
    f[14] = z1[g];
    f[15] = z2[g];
}

inline unsigned blocks_for(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

}  // namespace

hipError_t launch_levels_z(const bmd_problem* p, double z1, hipStream_t s) {
    hipLaunchKernelGGL(k_levels_z, dim3(blocks_for(p->P.G, 128)), dim3(128), 0, s, p->P.G, z1, p->P.alpha0, p->d_r,
                       p->d_gl, p->d_z1, p->d_z2);
    return hipGetLastError();
}

hipError_t launch_levels_golden(const bmd_problem* p, int phase, bool probe, int end, double a_lo, double a_hi,
                                const double* mean, double* st, int32_t* side, hipStream_t s) {
    hipLaunchKernelGGL(k_levels_golden, dim3(blocks_for(p->P.G, 128)), dim3(128), 0, s, p->P.G, phase, probe, end,
                       a_lo, a_hi, p->P.alpha0, p->d_r, mean, p->d_gl, st, side, p->d_z1, p->d_z2);
    return hipGetLastError();
}

hipError_t launch_levels_newton(const bmd_problem* p, int phase, double a_lo, double a_hi, double tol,
                                const double* mean, const double* dmean, double* st, hipStream_t s) {
    hipLaunchKernelGGL(k_levels_newton, dim3(blocks_for(p->P.G, 128)), dim3(128), 0, s, p->P.G, phase, a_lo, a_hi,
                       tol, p->P.alpha0, p->d_r, mean, dmean, p->d_gl, st, p->d_z1, p->d_z2);
    return hipGetLastError();
}

hipError_t launch_levels_best(const bmd_problem* p, int k, const double* mean, double* best, int32_t* best_k,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_levels_best, dim3(blocks_for(p->P.G, 256)), dim3(256), 0, s, p->P.G, k, mean, best, best_k);
    return hipGetLastError();
}

// Design order of the nested-population sweeps: the designs whose last
// critical value exists (not NaN) first, then the others, each in index order,
// so that the sweep's wavefronts fill with designs that have a last level and
// the rest form whole wavefronts that leave at once.  One workgroup: a count,
// then a scan per tile of 1,024 designs.
__global__ __launch_bounds__(1024) void k_order_feasible(int64_t G, const double* __restrict__ z_last,
                                                         int32_t* __restrict__ order) {
    __shared__ int scan[1024];
    __shared__ int64_t total;
    const int t = threadIdx.x;
    if (t == 0) total = 0;
    __syncthreads();
    int64_t mine = 0;
    for (int64_t g = t; g < G; g += 1024) mine += z_last[g] == z_last[g];
    atomicAdd(reinterpret_cast<unsigned long long*>(&total), static_cast<unsigned long long>(mine));
    __syncthreads();
    const int64_t nf = total;
    int64_t base_f = 0, base_n = 0;
    for (int64_t g0 = 0; g0 < G; g0 += 1024) {
        const int64_t g = g0 + t;
        const int ok = g < G && z_last[g] == z_last[g];
        scan[t] = ok;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan of the flags
            const int v = t >= off ? scan[t - off] : 0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        const int incl = scan[t];
        const int tile_f = scan[1023];
        if (g < G) {
            const int64_t before_f = incl - ok;                 // feasible designs before g in this tile
            const int64_t before_n = static_cast<int64_t>(t) - before_f;
            order[ok ? base_f + before_f : nf + base_n + before_n] = static_cast<int32_t>(g);
        }
        base_f += tile_f;
        base_n += min<int64_t>(1024, G - g0) - tile_f;
        __syncthreads();
    }
}

hipError_t launch_design_precompute(const bmd_problem* p, hipStream_t s) {
    if (p->P.G == 0) return hipSuccess;
    if (p->P.design_space == BMD_DESIGN_NESTED3) return launch_nested3_precompute(p, s);   // its own order
    if (p->P.design_space == BMD_DESIGN_NESTED4) return launch_nested4_precompute(p, s);
    if (p->P.design_space == BMD_DESIGN_ALPHA3 || p->P.design_space == BMD_DESIGN_ALPHA4) {
        const bool four = p->P.design_space == BMD_DESIGN_ALPHA4;
        hipError_t e = four ? launch_four_precompute(p, s) : launch_three_precompute(p, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_order_feasible, dim3(1), dim3(1024), 0, s, p->P.G, four ? p->d_z4 : p->d_z3,
                           p->d_order);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_design_precompute, dim3(blocks_for(p->P.G, 128)), dim3(128), 0, s, p->P,
                       p->d_ghp, kPrecomputeGH, p->d_gl, p->d_r, p->d_z1, p->d_z2);
    return hipGetLastError();
}

hipError_t launch_axis_tables(const bmd_problem* p, int prec, hipStream_t s) {
    if (p->P.G == 0) return hipSuccess;
    const PrecTables& t = p->tab[prec];
    const int64_t total = static_cast<int64_t>(p->P.d) * t.K * p->P.mmax;
    if (prec == BMD_FP64)
        hipLaunchKernelGGL(k_axis_tables<double>, dim3(blocks_for(total, 256)), dim3(256), 0, s, p->P,
                           t.gh, t.K, static_cast<double*>(t.A));
    else
        hipLaunchKernelGGL(k_axis_tables<float>, dim3(blocks_for(total, 256)), dim3(256), 0, s, p->P,
                           t.gh, t.K, static_cast<float*>(t.A));
    return hipGetLastError();
}

template <typename T>
static DrawArrays<T> carve(const bmd_problem* p, int prec, int64_t M, void* ws) {
    DrawArrays<T> D;
    const int d = p->P.d, K = p->tab[prec].K;
    char* c = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* r = c;
        c += (bytes + 255) / 256 * 256;
        return r;
    };
    D.b0 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.b1 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.mu1 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.PR = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.tauT = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.e1 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.e2 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.e3 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.e4 = reinterpret_cast<T*>(take(sizeof(T) * M));
    D.thr = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * d * M));
    D.q4 = reinterpret_cast<T*>(take(sizeof(T) * 4 * M));
    D.tau = reinterpret_cast<double*>(take(sizeof(double) * d * M));
    D.B = reinterpret_cast<T*>(take(sizeof(T) * (d >= 2 ? static_cast<size_t>(M) * d * K : 1)));
    D.M = M;
    D.K = K;
    return D;
}

size_t draw_workspace_bytes(const bmd_problem* p, int prec, int64_t M) {
    const size_t T = prec == BMD_FP64 ? 8 : 4;
    const int d = p->P.d, K = p->tab[prec].K;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return 9 * al(T * M) + al(4 * d * M) + al(4 * T * M) + al(8 * d * M) +
           al(T * (d >= 2 ? static_cast<size_t>(M) * d * K : 1));
}

DrawArrays<double> draws_fp64(const bmd_problem* p, int64_t M, const void* ws) {
    return carve<double>(p, BMD_FP64, M, const_cast<void*>(ws));
}
DrawArrays<float> draws_fp32(const bmd_problem* p, int64_t M, const void* ws) {
    return carve<float>(p, BMD_FP32_COMP, M, const_cast<void*>(ws));
}

hipError_t launch_draws(const bmd_problem* p, int prec, uint64_t k0, int64_t M, void* ws, hipStream_t s) {
    const PrecTables& t = p->tab[prec];
    if (prec == BMD_FP64)
        hipLaunchKernelGGL(k_draws<double>, dim3(blocks_for(M, 128)), dim3(128), 0, s, p->P, t.gh, t.K, k0, M,
                           carve<double>(p, prec, M, ws));
    else
        hipLaunchKernelGGL(k_draws<float>, dim3(blocks_for(M, 128)), dim3(128), 0, s, p->P, t.gh, t.K, k0, M,
                           carve<float>(p, prec, M, ws));
    return hipGetLastError();
}

DrawArrays<double> draws_fp64_at(const bmd_problem* p, int64_t M, void* ws) { return carve<double>(p, BMD_FP64, M, ws); }
DrawArrays<float> draws_fp32_at(const bmd_problem* p, int64_t M, void* ws) {
    return carve<float>(p, BMD_FP32_COMP, M, ws);
}

size_t draw_job_bytes(int prec) { return prec == BMD_FP64 ? sizeof(DrawJob<double>) : sizeof(DrawJob<float>); }

void fill_draw_job(int prec, void* dst, const bmd_problem* p, void* draws_ws, int64_t M, int64_t first) {
    const PrecTables& t = p->tab[prec];
    if (prec == BMD_FP64) {
        DrawJob<double> j{p->P, t.gh, t.K, first, carve<double>(p, prec, M, draws_ws)};
        std::memcpy(dst, &j, sizeof j);
    } else {
        DrawJob<float> j{p->P, t.gh, t.K, first, carve<float>(p, prec, M, draws_ws)};
        std::memcpy(dst, &j, sizeof j);
    }
}

hipError_t launch_draws_batch(int prec, const void* jobs, int n_jobs, int64_t total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (prec == BMD_FP64)
        hipLaunchKernelGGL(k_draws_batch<double>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                           static_cast<const DrawJob<double>*>(jobs), n_jobs, total);
    else
        hipLaunchKernelGGL(k_draws_batch<float>, dim3(blocks_for(total, 128)), dim3(128), 0, s,
                           static_cast<const DrawJob<float>*>(jobs), n_jobs, total);
    return hipGetLastError();
}

hipError_t launch_inspect_draws(const bmd_problem* p, uint64_t k0, int64_t n, double* u, double* fields,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_inspect_draws, dim3(blocks_for(n, 128)), dim3(128), 0, s, p->P, p->d_ghp,
                       kPrecomputeGH, k0, n, u, fields);
    return hipGetLastError();
}

hipError_t launch_inspect_designs(const bmd_problem* p, int64_t g0, int64_t n, double* fields, hipStream_t s) {
    hipLaunchKernelGGL(k_inspect_designs, dim3(blocks_for(n, 128)), dim3(128), 0, s, p->P, g0, n, p->d_r,
                       p->d_z1, p->d_z2, p->d_z3, p->d_z4, fields);
    return hipGetLastError();
}

}  // namespace bmd
