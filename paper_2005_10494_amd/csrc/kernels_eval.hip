// Grid sweep of the expected-power estimate (Formula 5): one thread per design,
// draw slices across workgroups, FP64 per-design sums.
//
// Per (design g, draw k) the summand is 1 - Phi_2(z1 - mu1_k, z2 - mu2_gk; sqrt r_g):
//   step prior:  mu1 = sqrt(I) (b0 + b1 P(R)),  mu2 = sqrt(r I) (b0 + b1 O / r),
//                O = P(x_j > max(c_j, t_j) all j)  (responders inside the subgroup)
//   paper prior: mu1 = sqrt(I) Delta_1,  mu2 = sqrt(r I) Delta_2  (Formula 10)
// The integrand is evaluated in T (double or float); sums are always FP64.
#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {
namespace {

template <typename T>
struct EvalArgs {
    DevProblem P;
    const double* r;
    const double* z1;
    const double* z2;
    const T* A;          // axis tables [d][K][mmax]
    DrawArrays<T> D;
    const double* gl;    // packed GL table (FP64 nodes)
    const T* glw;        // packed GL table in T (weights read from here)
    int64_t slice_len;
    double* partials;    // [n_slices][2][G]
};

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

template <typename T>
__device__ __forceinline__ T logistic(T x) {
    return T(1) / (T(1) + exp(-x));
}

// Responder-in-subgroup fraction O for draw k (d >= 2, grid design idx).
template <typename T, int D>
__device__ __forceinline__ T overlap_grid(const EvalArgs<T>& a, const int* idx, const double* q, T rT,
                                          int64_t k) {
    const int64_t M = a.D.M;
    const int K = a.D.K;
    const int mmax = a.P.mmax;
    const T* Bk = a.D.B + k * D * K;
    if (a.P.width > 0.0) {
        T s[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            s[j] = logistic(static_cast<T>((q[j] - a.D.tau[j * M + k]) / a.P.width));
        T acc = T(0);
        for (int m = 0; m < K; ++m) {
            T prod = T(1);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const T av = a.A[(static_cast<int64_t>(j) * K + m) * mmax + idx[j]];
                const T bv = Bk[j * K + m];
                prod *= s[j] * av + (T(1) - s[j]) * bv;
            }
            acc += prod;
        }
        return acc;
    }
    bool fl[D];
    bool all = true, none = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        fl[j] = idx[j] >= a.D.thr[j * M + k];
        all = all && fl[j];
        none = none && !fl[j];
    }
    if (all) return rT;
    if (none) return a.D.PR[k];
    const T* src[D];
    int64_t step[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        src[j] = fl[j] ? a.A + static_cast<int64_t>(j) * K * mmax + idx[j] : Bk + j * K;
        step[j] = fl[j] ? mmax : 1;
    }
    T acc = T(0);
    for (int m = 0; m < K; ++m) {
        T prod = src[0][m * step[0]];
#pragma unroll
        for (int j = 1; j < D; ++j) prod *= src[j][m * step[j]];
        acc += prod;
    }
    return acc;
}

template <typename T, int D, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_eval_direct(EvalArgs<T> a) {
    const int64_t G = a.P.G;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kEvalBlock + threadIdx.x;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;   // idle lanes shadow the last design

    int idx[D];
    double q[D];
    {
        int64_t rem = gg;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            idx[j] = static_cast<int>(rem / a.P.stride[j]);
            rem -= static_cast<int64_t>(idx[j]) * a.P.stride[j];
            q[j] = grid_coord(a.P.q_lo, a.P.q_hi, idx[j], a.P.m[j]);
        }
    }
    const double r = a.r[gg];
    const double rho = sqrt(r);
    const int n_lane = sizeof(T) == 8 ? bvn_nodes_fp64(rho) : bvn_nodes_fp32(rho);
    const int n = wave_max(n_lane);
    BvnConst<T, NMAX> bc;
    bc.init(rho, n, a.gl);
    const T* w = a.glw + gl_offset(n) + n;

    const double srI_d = sqrt(r * a.P.info);
    const T z1 = static_cast<T>(a.z1[gg]);
    const T z2 = static_cast<T>(a.z2[gg]);
    const T srI = static_cast<T>(srI_d);
    const T invr = static_cast<T>(1.0 / r);
    const T rT = static_cast<T>(r);
    const T omq = static_cast<T>(1.0 - q[0]);
    // paper prior: mu2 = c0 + c1 e1 + c2 e2
    T c0 = T(0), c1 = T(0), c2 = T(0);
    if (a.P.effect == BMD_EFFECT_PAPER_GAUSS) {
        const double th2 = -log1p(-(a.P.paper_a - a.P.paper_b * r));
        const double sg2 = 1.0 / sqrt(a.P.paper_events * r / 4.0);
        c0 = static_cast<T>(srI_d * th2);
        c1 = static_cast<T>(srI_d * sg2 * sqrt(r));
        c2 = static_cast<T>(srI_d * sg2 * sqrt(1.0 - r));
    }

    const int64_t M = a.D.M;
    const int64_t kb = static_cast<int64_t>(blockIdx.y) * a.slice_len;
    const int64_t ke = min(M, kb + a.slice_len);
    const bool step_prior = a.P.effect == BMD_EFFECT_STEP;
    const int zinf = a.P.zinf;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const T mu1 = a.D.mu1[k];
        T mu2;
        if (step_prior) {
            T O;
            if constexpr (D == 1) {
                if (a.P.width > 0.0) {
                    const double tau = a.D.tau[k];
                    const T s = logistic(static_cast<T>((q[0] - tau) / a.P.width));
                    O = T(1) - (s * static_cast<T>(q[0]) + (T(1) - s) * a.D.tauT[k]);
                } else {
                    O = idx[0] >= a.D.thr[k] ? omq : T(1) - a.D.tauT[k];
                }
            } else {
                O = overlap_grid<T, D>(a, idx, q, rT, k);
            }
            mu2 = srI * (a.D.b0[k] + a.D.b1[k] * O * invr);
        } else {
            mu2 = c0 + c1 * a.D.e1[k] + c2 * a.D.e2[k];
        }
        const T h = z1 - mu1, kq = z2 - mu2;
        T p;
        if (zinf == 0) p = bvn_cdf<NMAX>(h, kq, bc, w, n);
        else if (zinf == 1) p = norm_cdf(kq);
        else if (zinf == 2) p = norm_cdf(h);
        else p = T(1);
        const double v = static_cast<double>(T(1) - p);
        s1 += v;
        s2 += v * v;
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(blockIdx.y) * 2 * G;
        out[g] = s1;
        out[G + g] = s2;
    }
}

__global__ void k_finalize(int64_t G, int64_t M, int n_slices, const double* __restrict__ part,
                           double* __restrict__ mean, double* __restrict__ var) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double s1 = 0.0, s2 = 0.0;
    for (int s = 0; s < n_slices; ++s) {
        s1 += part[static_cast<int64_t>(s) * 2 * G + g];
        s2 += part[static_cast<int64_t>(s) * 2 * G + G + g];
    }
    const double Md = static_cast<double>(M);
    mean[g] = s1 / Md;
    if (var) var[g] = M > 1 ? fmax(0.0, (s2 - s1 * s1 / Md) / (Md - 1.0)) : 0.0;
}

template <typename T, int NMAX>
hipError_t launch_typed(const bmd_problem* p, int prec, const EvalArgs<T>& a, int n_slices, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((p->P.G + kEvalBlock - 1) / kEvalBlock), static_cast<unsigned>(n_slices));
    switch (p->P.d) {
        case 1: hipLaunchKernelGGL((k_eval_direct<T, 1, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_eval_direct<T, 2, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_eval_direct<T, 3, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_eval_direct<T, 4, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_eval_direct<T, 5, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_eval_direct<T, 6, NMAX>), grid, dim3(kEvalBlock), 0, s, a); break;
    }
    (void)prec;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval_grid(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, hipStream_t s) {
    if (prec == BMD_FP64) {
        EvalArgs<double> a{p->P, p->d_r, p->d_z1, p->d_z2, static_cast<const double*>(p->tab[prec].A),
                           draws_fp64(p, M, ws), p->d_gl, static_cast<const double*>(p->tab[prec].glw),
                           slice_len, partials};
        return launch_typed<double, 24>(p, prec, a, n_slices, s);
    }
    EvalArgs<float> a{p->P, p->d_r, p->d_z1, p->d_z2, static_cast<const float*>(p->tab[prec].A),
                      draws_fp32(p, M, ws), p->d_gl, static_cast<const float*>(p->tab[prec].glw),
                      slice_len, partials};
    return launch_typed<float, 12>(p, prec, a, n_slices, s);
}

hipError_t launch_finalize(const bmd_problem* p, int64_t M, const double* partials, int n_slices, double* mean,
                           double* var, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((G + 255) / 256)), dim3(256), 0, s, G, M, n_slices,
                       partials, mean, var);
    return hipGetLastError();
}

}  // namespace bmd
