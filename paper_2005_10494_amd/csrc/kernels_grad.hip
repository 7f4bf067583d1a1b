// Objective and gradient at continuous design points (the differentiation
// form): d obj / d q_j and d obj / d (mu_b0, mu_b1), averaged over the prior
// draws, which the draw kernel writes to HBM in passes and the gradient kernel
// stages chunk by chunk in LDS.
//
// Per (point, draw) the summand is f = 1 - Phi_2(h, k; rho) with
//   h = z1 - sqrt(I) (b0 + b1 P(R)),  k = z2 - sqrt(r I) (b0 + b1 O / r),  rho = sqrt(r),
// and its adjoint is propagated through
//   dPhi_2/dh = phi(h) Phi((k - rho h)/s),  dPhi_2/dk = phi(k) Phi((h - rho k)/s),
//   dPhi_2/drho = phi_2(h, k; rho),  s = sqrt(1 - rho^2)   (Plackett),
// the overlap O (logistic or exact cutoff indicator, leave-one-out products
// over the Gauss-Hermite nodes), the subgroup fraction r(q) and the equal-FWER
// critical value z*(r) (implicit derivative of Formula 2).
#include <algorithm>
#include <cstdlib>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "draw_chunk.hpp"

namespace bmd {
namespace {

constexpr int kGradBlock = 128;   // points per workgroup
constexpr int kPointFields = 32;

// Per-point record (FP64):
//  0 r, 1 z1, 2 z2, 3 dz/drho, 4 valid, 5..10 dr/dq_j, 11..16 q_j, 17..22 c_j

__device__ double orthant_factor_gh(const DevProblem& P, const double* c, const double* __restrict__ gh,
                                    int K, int deriv_axis) {
    const double* x = gh;
    const double* w = gh + K;
    double acc = 0.0;
    for (int m = 0; m < K; ++m) {
        const double t = P.sr * x[m];
        double prod = w[m];
        for (int j = 0; j < P.d; ++j) {
            const double a = (t - c[j]) / P.sq;
            prod *= (j == deriv_axis) ? norm_pdf(a) : norm_cdf(a);
        }
        acc += prod;
    }
    return acc;
}

__device__ double bvn_setup24(double h, double k, double rho, const double* __restrict__ gl) {
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

__device__ double zstar_pt(double rho, double alpha0, const double* __restrict__ gl) {
    double lo = -norm_quantile(alpha0), hi = -norm_quantile(0.5 * alpha0);
    double z = 0.5 * (lo + hi);
    const double c = sqrt((1.0 - rho) / (1.0 + rho));
    for (int it = 0; it < 60; ++it) {
        const double F = 2.0 * norm_cdf(-z) - bvn_setup24(-z, -z, rho, gl) - alpha0;
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

// One thread per point: design quantities, their q-derivatives, and the
// per-node tables A_j[m] = Phi(a_jm), dA_j[m] = d A_j[m] / d q_j
// (a_jm = (sqrt(rho_b) x_m - c_j)/sqrt(1 - rho_b); weights folded into j = 0).
template <typename T>
__global__ __launch_bounds__(128) void k_grad_points(DevProblem P, const double* __restrict__ q_in, int64_t B,
                              const double* __restrict__ ghp, int Kp, const double* __restrict__ gh, int K,
                              const double* __restrict__ gl, double* __restrict__ info, T* __restrict__ A,
                              T* __restrict__ dA) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double* f = info + b * kPointFields;
    const int d = P.d;
    double q[kMaxDim], c[kMaxDim];
    bool valid = true;
    for (int j = 0; j < d; ++j) {
        q[j] = q_in[b * d + j];
        // grid endpoints may round a few ulp past q_lo / q_hi
        valid = valid && (q[j] >= P.q_lo - 1e-12 && q[j] <= P.q_hi + 1e-12);
        if (!valid) q[j] = P.q_lo;
        c[j] = norm_quantile(q[j]);
    }
    double r, dr[kMaxDim];
    if (d == 1) {
        r = 1.0 - q[0];
        dr[0] = -1.0;
    } else {
        r = orthant_factor_gh(P, c, ghp, Kp, -1);
        for (int j = 0; j < d; ++j)
            dr[j] = -orthant_factor_gh(P, c, ghp, Kp, j) / P.sq / norm_pdf(c[j]);
    }
    const double rho = sqrt(r);
    double z1, z2, dzdrho = 0.0;
    if (P.alpha_rule == BMD_ALPHA_FWER_EQUAL) {
        z1 = z2 = zstar_pt(rho, P.alpha0, gl);
        // Formula 2 held fixed: dz*/drho = -phi_2(z,z;rho) / (2 phi(z) Phi(z sqrt((1-rho)/(1+rho))))
        const double om = (1.0 - rho) * (1.0 + rho);
        const double dens = exp(-z1 * z1 / (1.0 + rho)) / (2.0 * M_PI * sqrt(om));
        dzdrho = -dens / (2.0 * norm_pdf(z1) * norm_cdf(z1 * sqrt((1.0 - rho) / (1.0 + rho))));
    } else {
        z1 = P.zf1;
        z2 = P.zf2;
    }
    f[0] = r;
    f[1] = z1;
    f[2] = z2;
    f[3] = dzdrho;
    f[4] = valid ? 1.0 : 0.0;
    for (int j = 0; j < kMaxDim; ++j) {
        f[5 + j] = j < d ? dr[j] : 0.0;
        f[11 + j] = j < d ? q[j] : 0.0;
        f[17 + j] = j < d ? c[j] : 0.0;
    }
    if (d >= 2) {
        for (int j = 0; j < d; ++j) {
            const double dcdq = 1.0 / norm_pdf(c[j]);
            for (int m = 0; m < K; ++m) {
                const double a = (P.sr * gh[m] - c[j]) / P.sq;
                const double wf = j == 0 ? gh[K + m] : 1.0;
                A[(static_cast<int64_t>(j) * K + m) * B + b] = static_cast<T>(wf * norm_cdf(a));
                dA[(static_cast<int64_t>(j) * K + m) * B + b] = static_cast<T>(-wf * norm_pdf(a) / P.sq * dcdq);
            }
        }
    }
}

// Logistic 1/(1 + e^-x); FP32 with the hardware exp2 and reciprocal.
__device__ __forceinline__ double lgst(double x) { return 1.0 / (1.0 + exp(-x)); }
__device__ __forceinline__ float lgst(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634074f * x));
}
// e^x; FP32 with the hardware exp2.
__device__ __forceinline__ double expT(double x) { return exp(x); }
__device__ __forceinline__ float expT(float x) { return __builtin_amdgcn_exp2f(1.4426950408889634074f * x); }

struct GradArgs {
    DevProblem P;
    int64_t B;
    int64_t M;
    int K;
    int chunk;             // draws staged per chunk
    const double* info;
    const void* A;
    const void* dA;
    const double* gl;
    const void* glw;
    int64_t slice_len;
    int slice0;            // first draw slice of this launch (a pass over draws)
    int64_t draw_k0;       // first draw held by the draw arrays of this pass
    double* partials;      // [n_slices][d+3][B]
    int lanes;             // threads per point (a power of two <= 64): each takes every lanes-th draw pass
};

// Copy draws k0 .. k0+nk-1 of a pass (local indices) from the draw arrays into
// the LDS chunk; every thread of the block calls it.  Ends with the chunk
// visible to the whole block.
template <typename T, int D>
__device__ void stage_chunk(const DrawArrays<T>& G, int K, const ChunkView<T>& c, int64_t k0, int nk) {
    __syncthreads();   // previous chunk fully consumed
    for (int e = threadIdx.x; e < nk; e += blockDim.x) {
        c.b0[e] = G.b0[k0 + e];
        c.b1[e] = G.b1[k0 + e];
        c.PR[e] = G.PR[k0 + e];
        c.mu1[e] = G.mu1[k0 + e];
#pragma unroll
        for (int j = 0; j < D; ++j) c.tau[e * kMaxDim + j] = G.tau[j * G.M + k0 + e];
    }
    if constexpr (D >= 2) {
        const T* src = G.B + k0 * D * K;   // B rows of consecutive draws are contiguous
        if constexpr (sizeof(T) == 8) {
            // FP64: eight loads in flight before their LDS writes, then the
            // tail one by one (the FP64 refinement's gradient call 5.2 -> 4.1
            // ms; the FP32 kernel, short of registers, was slower with it)
            const int total = nk * D * K, bd = blockDim.x;
            int e = threadIdx.x;
            for (; e + 7 * bd < total; e += 8 * bd) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = src[e + u * bd];
#pragma unroll
                for (int u = 0; u < 8; ++u) c.Bt[e + u * bd] = v[u];
            }
            for (; e < total; e += bd) c.Bt[e] = src[e];
        } else {
            for (int e = threadIdx.x; e < nk * D * K; e += blockDim.x) c.Bt[e] = src[e];
        }
    }
    __syncthreads();
}

// R draws per pass over the point's node tables.  SPLIT (few points): `lanes`
// consecutive threads share a point; thread `sub` of a point takes the draw
// passes sub, sub + lanes, ... of every chunk, and the point's sums are added
// across those lanes (a fixed butterfly order) before they are written.  (A
// separate instantiation: the runtime stride costs the one-lane kernel 17
// VGPRs and a wavefront per SIMD.)
template <typename T, int D, int NMAX, int R, bool SPLIT>
__global__ __launch_bounds__(kGradBlock) void k_grad(GradArgs a, DrawArrays<T> Dr) {
    extern __shared__ __align__(16) char lds[];
    const ChunkView<T> ch = carve_chunk<T>(lds, a.chunk, a.K);
    const DevProblem& P = a.P;
    const int K = a.K;
    const int64_t Bn = a.B;
    const int L = SPLIT ? a.lanes : 1;
    const int sub = static_cast<int>(threadIdx.x) & (L - 1);
    const int64_t b = (static_cast<int64_t>(blockIdx.x) * kGradBlock + threadIdx.x) / L;
    const bool active = b < Bn;
    const int64_t bb = active ? b : Bn - 1;
    const double* f = a.info + bb * kPointFields;
    const T* A = static_cast<const T*>(a.A);
    const T* dA = static_cast<const T*>(a.dA);

    const double r = f[0];
    const double rho = sqrt(r);
    int n = sizeof(T) == 8 ? bvn_nodes_fp64(rho) : bvn_nodes_fp32(rho);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n = max(n, __shfl_xor(n, off));
    n = __builtin_amdgcn_readfirstlane(n);
    BvnConst<T, NMAX> bc;
    bc.init(rho, n, a.gl);
    const T* wgl = static_cast<const T*>(a.glw) + gl_offset(n) + n;

    const T sI = static_cast<T>(P.sqrtI);
    const T srI = static_cast<T>(sqrt(r * P.info));
    const T invr = static_cast<T>(1.0 / r);
    const T rhoT = static_cast<T>(rho);
    const T isig = static_cast<T>(1.0 / sqrt((1.0 - rho) * (1.0 + rho)));
    const T z1 = static_cast<T>(f[1]), z2 = static_cast<T>(f[2]);
    const double sqr = sqrt(r);
    T da[D], dz[D], uu[D], ww[D];
    double qd[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double drj = f[5 + j];
        const double drho = drj / (2.0 * rho);
        da[j] = static_cast<T>(drho);
        dz[j] = static_cast<T>(f[3] * drho);
        uu[j] = static_cast<T>(P.sqrtI * drj / (2.0 * sqr));
        ww[j] = static_cast<T>(P.sqrtI * drj / (2.0 * r * sqr));
        qd[j] = f[11 + j];
    }
    const T vv = static_cast<T>(P.sqrtI / sqr);
    const bool logistic = P.width > 0.0;
    const double iw64 = logistic ? 1.0 / P.width : 0.0;
    const T iw = static_cast<T>(iw64);

    double s_obj = 0.0, s_mu0 = 0.0, s_mu1 = 0.0, s_q[D];
#pragma unroll
    for (int j = 0; j < D; ++j) s_q[j] = 0.0;

    const int slice = a.slice0 + static_cast<int>(blockIdx.y);
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(a.M, kb + a.slice_len);
    for (int64_t k0 = kb; k0 < ke; k0 += a.chunk) {
        const int nk = static_cast<int>(min<int64_t>(a.chunk, ke - k0));
        stage_chunk<T, D>(Dr, K, ch, k0 - a.draw_k0, nk);
        for (int i0 = sub * R; i0 < nk; i0 += R * L) {
            T O[R], dO[R][D], s[R][D], sp[R][D];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = min(i0 + rr, nk - 1);
                O[rr] = T(0);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double dq = qd[j] - ch.tau[i * kMaxDim + j];
                    if (logistic) {
                        s[rr][j] = lgst(static_cast<T>(dq * iw64));
                        sp[rr][j] = s[rr][j] * (T(1) - s[rr][j]) * iw;
                    } else {
                        s[rr][j] = dq > 0.0 ? T(1) : T(0);
                        sp[rr][j] = T(0);
                    }
                    dO[rr][j] = T(0);
                }
            }
            if constexpr (D == 1) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int i = min(i0 + rr, nk - 1);
                    const T tau = static_cast<T>(ch.tau[i * kMaxDim]);
                    const T q0 = static_cast<T>(qd[0]);
                    if (logistic) {
                        O[rr] = T(1) - (s[rr][0] * q0 + (T(1) - s[rr][0]) * tau);
                        dO[rr][0] = -(s[rr][0] + sp[rr][0] * static_cast<T>(qd[0] - ch.tau[i * kMaxDim]));
                    } else {
                        O[rr] = s[rr][0] > T(0) ? T(1) - q0 : T(1) - tau;
                        dO[rr][0] = s[rr][0] > T(0) ? T(-1) : T(0);
                    }
                }
            } else {
                for (int m = 0; m < K; ++m) {
                    T av[D], dav[D];
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        const int64_t o = (static_cast<int64_t>(j) * K + m) * Bn + bb;
                        av[j] = A[o];
                        dav[j] = dA[o];
                    }
#pragma unroll
                    for (int rr = 0; rr < R; ++rr) {
                        const int i = min(i0 + rr, nk - 1);
                        const T* Bi = ch.Bt + (static_cast<size_t>(i) * K + m) * D;
                        // mix_j = s_j a_j + (1 - s_j) b_j = b_j + s_j (a_j - b_j);
                        // d mix_j / d q_j = s'_j (a_j - b_j) + s_j a'_j
                        T dif[D], mix[D], pre[D + 1];
                        pre[0] = T(1);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            const T bv = Bi[j];
                            dif[j] = av[j] - bv;
                            mix[j] = fma(s[rr][j], dif[j], bv);
                            pre[j + 1] = pre[j] * mix[j];
                        }
                        O[rr] += pre[D];
                        T suf = T(1);
#pragma unroll
                        for (int j = D - 1; j >= 0; --j) {
                            const T dmix = fma(sp[rr][j], dif[j], s[rr][j] * dav[j]);
                            dO[rr][j] = fma(dmix, pre[j] * suf, dO[rr][j]);
                            suf *= mix[j];
                        }
                    }
                }
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                if (i0 + rr >= nk) break;
                const int i = i0 + rr;
                const T b0 = ch.b0[i], b1 = ch.b1[i], PR = ch.PR[i], mu1 = ch.mu1[i];
                const T mu2 = srI * (b0 + b1 * O[rr] * invr);
                const T h = z1 - mu1, kq = z2 - mu2;
                T p, ph, pk, pr;
                if (P.zinf == 0) {
                    p = bvn_cdf<NMAX>(h, kq, bc, wgl, n);
                    ph = norm_pdf(h) * norm_cdf((kq - rhoT * h) * isig);
                    pk = norm_pdf(kq) * norm_cdf((h - rhoT * kq) * isig);
                    const T e = (h * h - T(2) * rhoT * h * kq + kq * kq) * isig * isig;
                    pr = expT(-T(0.5) * e) * isig * T(0.15915494309189533577);
                } else if (P.zinf == 2) {
                    p = norm_cdf(h); ph = norm_pdf(h); pk = T(0); pr = T(0);
                } else if (P.zinf == 1) {
                    p = norm_cdf(kq); ph = T(0); pk = norm_pdf(kq); pr = T(0);
                } else {
                    p = T(1); ph = T(0); pk = T(0); pr = T(0);
                }
                s_obj += static_cast<double>(T(1) - p);
                s_mu0 += static_cast<double>(ph * sI + pk * srI);
                s_mu1 += static_cast<double>(ph * sI * PR + pk * srI * O[rr] * invr);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const T dmu2 = b0 * uu[j] + b1 * (vv * dO[rr][j] - O[rr] * ww[j]);
                    const T dp = (ph + pk) * dz[j] - pk * dmu2 + pr * da[j];
                    s_q[j] -= static_cast<double>(dp);
                }
            }
        }
    }
    for (int off = 1; off < L; off <<= 1) {   // the point's lanes are consecutive within one wavefront
        s_obj += __shfl_xor(s_obj, off);
        s_mu0 += __shfl_xor(s_mu0, off);
        s_mu1 += __shfl_xor(s_mu1, off);
#pragma unroll
        for (int j = 0; j < D; ++j) s_q[j] += __shfl_xor(s_q[j], off);
    }
    if (active && sub == 0) {
        double* out = a.partials + static_cast<int64_t>(slice) * (D + 3) * Bn;
        out[b] = s_obj;
#pragma unroll
        for (int j = 0; j < D; ++j) out[(1 + j) * Bn + b] = s_q[j];
        out[(1 + D) * Bn + b] = s_mu0;
        out[(2 + D) * Bn + b] = s_mu1;
    }
}

__global__ void k_grad_finalize(int d, int64_t B, int64_t M, int n_slices, const double* __restrict__ part,
                                const double* __restrict__ info, double* __restrict__ obj,
                                double* __restrict__ gq, double* __restrict__ gmu) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const bool valid = info[b * kPointFields + 4] != 0.0;
    const double Md = static_cast<double>(M);
    for (int c = 0; c < d + 3; ++c) {
        double s = 0.0;
        for (int sl = 0; sl < n_slices; ++sl) s += part[(static_cast<int64_t>(sl) * (d + 3) + c) * B + b];
        const double v = valid ? s / Md : NAN;
        if (c == 0) obj[b] = v;
        else if (c <= d) { if (gq) gq[b * d + (c - 1)] = v; }
        else if (gmu) gmu[b * 2 + (c - 1 - d)] = v;
    }
}

// The same reduction with one workgroup per (point, component): for few points
// and many slices, where one thread per point would walk thousands of slices.
// Thread t adds slices t, t + 256, ... in order, then a fixed-order tree.
__global__ __launch_bounds__(256) void k_grad_finalize_wide(int d, int64_t B, int64_t M, int n_slices,
                                                            const double* __restrict__ part,
                                                            const double* __restrict__ info, double* __restrict__ obj,
                                                            double* __restrict__ gq, double* __restrict__ gmu) {
    __shared__ double red[256];
    const int64_t b = blockIdx.x / (d + 3);
    const int c = static_cast<int>(blockIdx.x % (d + 3));
    double s = 0.0;
    for (int sl = threadIdx.x; sl < n_slices; sl += 256) s += part[(static_cast<int64_t>(sl) * (d + 3) + c) * B + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const bool valid = info[b * kPointFields + 4] != 0.0;
    const double v = valid ? red[0] / static_cast<double>(M) : NAN;
    if (c == 0) obj[b] = v;
    else if (c <= d) { if (gq) gq[b * d + (c - 1)] = v; }
    else if (gmu) gmu[b * 2 + (c - 1 - d)] = v;
}

template <typename T, int NMAX, int R, bool SPLIT>
const void* grad_kernel(int d) {
    switch (d) {
        case 1: return reinterpret_cast<const void*>(k_grad<T, 1, NMAX, 1, SPLIT>);
        case 2: return reinterpret_cast<const void*>(k_grad<T, 2, NMAX, R, SPLIT>);
        case 3: return reinterpret_cast<const void*>(k_grad<T, 3, NMAX, R, SPLIT>);
        case 4: return reinterpret_cast<const void*>(k_grad<T, 4, NMAX, R, SPLIT>);
        case 5: return reinterpret_cast<const void*>(k_grad<T, 5, NMAX, R, SPLIT>);
        default: return reinterpret_cast<const void*>(k_grad<T, 6, NMAX, R, SPLIT>);
    }
}

template <typename T, int NMAX, int R>
hipError_t launch_grad_typed(const GradArgs& ga, const DrawArrays<T>& Dr, int d, int n_slices, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((ga.B * ga.lanes + kGradBlock - 1) / kGradBlock),
                    static_cast<unsigned>(n_slices));
    const size_t lds = chunk_bytes<T>(ga.chunk, d, ga.K);
    const void* k = ga.lanes > 1 ? grad_kernel<T, NMAX, R, true>(d) : grad_kernel<T, NMAX, R, false>(d);
    void* args[] = {const_cast<GradArgs*>(&ga), const_cast<DrawArrays<T>*>(&Dr)};
    return hipLaunchKernel(k, grid, dim3(kGradBlock), args, lds, s);
}

}  // namespace

// Draws held in HBM per pass: whole slices, at most kGradDrawBudget bytes
// (BMD_GRAD_BUDGET, in bytes, overrides it; small values force many passes).
int64_t grad_pass_draws(const bmd_problem* p, int prec, int64_t M, int64_t slice_len) {
    size_t budget = kGradDrawBudget;
    if (const char* env = std::getenv("BMD_GRAD_BUDGET")) {
        const long long v = std::atoll(env);
        if (v > 0) budget = static_cast<size_t>(v);
    }
    const double per = static_cast<double>(draw_workspace_bytes(p, prec, 1 << 20)) / (1 << 20);
    int64_t slices = static_cast<int64_t>(static_cast<double>(budget) / (per * slice_len));
    slices = std::max<int64_t>(1, slices);
    return std::min<int64_t>(M, slices * slice_len);
}

size_t grad_workspace_bytes(const bmd_problem* p, int prec, int64_t B, int n_slices, int64_t M, int64_t slice_len) {
    const size_t T = prec == BMD_FP64 ? 8 : 4;
    const int d = p->P.d, K = p->tab[prec].K;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al(sizeof(double) * kPointFields * B) + 2 * al(T * d * K * B) +
           al(sizeof(double) * (d + 3) * B * n_slices) +
           al(draw_workspace_bytes(p, prec, grad_pass_draws(p, prec, M, slice_len)));
}

int grad_blocks_per_cu(const bmd_problem* p, int prec) {
    const int d = p->P.d, K = p->tab[prec].K;
    const int C = grad_chunk(prec, d, K);
    const void* f = prec == BMD_FP64 ? grad_kernel<double, 24, 1, false>(d) : grad_kernel<float, 12, 2, false>(d);
    const size_t lds = prec == BMD_FP64 ? chunk_bytes<double>(C, d, K) : chunk_bytes<float>(C, d, K);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kGradBlock, lds) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

// Threads per point: one when the points fill a workgroup, else the power of
// two (at most a wavefront) that lets the few points fill one.
int grad_lanes(int64_t B) {
    int L = 1;
    while (L < 64 && B * L < kGradBlock) L *= 2;
    return L;
}

// Draws per LDS chunk: as many as fit in 48 KB, at most 32.
int grad_chunk(int prec, int d, int K) {
    int C = 32;
    while (C > 1 && (prec == BMD_FP64 ? chunk_bytes<double>(C, d, K) : chunk_bytes<float>(C, d, K)) > 48 * 1024)
        C /= 2;
    return C;
}

hipError_t launch_grad(const bmd_problem* p, int prec, const double* d_q, int64_t B, int64_t M, void* ws,
                       int n_slices, int64_t slice_len, double* obj, double* gq, double* gmu, hipStream_t s) {
    const int d = p->P.d, K = p->tab[prec].K;
    const size_t T = prec == BMD_FP64 ? 8 : 4;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char* c = static_cast<char*>(ws);
    double* info = reinterpret_cast<double*>(c);
    c += al(sizeof(double) * kPointFields * B);
    void* A = c;
    c += al(T * d * K * B);
    void* dA = c;
    c += al(T * d * K * B);
    double* part = reinterpret_cast<double*>(c);
    c += al(sizeof(double) * (d + 3) * B * n_slices);
    void* dws = c;
    const unsigned pb = static_cast<unsigned>((B + 127) / 128);
    if (prec == BMD_FP64)
        hipLaunchKernelGGL(k_grad_points<double>, dim3(pb), dim3(128), 0, s, p->P, d_q, B, p->d_ghp, kPrecomputeGH,
                           p->tab[prec].gh, K, p->d_gl, info, static_cast<double*>(A), static_cast<double*>(dA));
    else
        hipLaunchKernelGGL(k_grad_points<float>, dim3(pb), dim3(128), 0, s, p->P, d_q, B, p->d_ghp, kPrecomputeGH,
                           p->tab[prec].gh, K, p->d_gl, info, static_cast<float*>(A), static_cast<float*>(dA));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // Passes over the draws: generate a pass into HBM, then the slices it holds.
    const int64_t pass = grad_pass_draws(p, prec, M, slice_len);
    for (int64_t k0 = 0; k0 < M; k0 += pass) {
        const int64_t np = std::min<int64_t>(pass, M - k0);
        e = launch_draws(p, prec, static_cast<uint64_t>(k0), np, dws, s);
        if (e != hipSuccess) return e;
        const int slice0 = static_cast<int>(k0 / slice_len);
        const int ns = static_cast<int>((np + slice_len - 1) / slice_len);
        GradArgs ga{p->P, B, M, K, grad_chunk(prec, d, K), info, A, dA, p->d_gl, p->tab[prec].glw,
                    slice_len, slice0, k0, part, grad_lanes(B)};
        e = prec == BMD_FP64 ? launch_grad_typed<double, 24, 1>(ga, draws_fp64_at(p, np, dws), d, ns, s)
                             : launch_grad_typed<float, 12, 2>(ga, draws_fp32_at(p, np, dws), d, ns, s);
        if (e != hipSuccess) return e;
    }
    if (n_slices > 256 && B * (d + 3) <= (int64_t(1) << 20))
        hipLaunchKernelGGL(k_grad_finalize_wide, dim3(static_cast<unsigned>(B * (d + 3))), dim3(256), 0, s, d, B, M,
                           n_slices, part, info, obj, gq, gmu);
    else
        hipLaunchKernelGGL(k_grad_finalize, dim3(pb), dim3(128), 0, s, d, B, M, n_slices, part, info, obj, gq, gmu);
    return hipGetLastError();
}

}  // namespace bmd
