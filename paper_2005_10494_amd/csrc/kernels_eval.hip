// Grid sweep of the expected-power estimate (Formula 5): one thread per design,
// draw slices across workgroups, FP64 per-design sums reduced in fixed order.
// The summand itself is in eval_core.hpp; T is the integrand type.
#include <type_traits>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "eval_core.hpp"

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

template <typename T, int D, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_eval_direct(EvalArgs<T> a) {
    const int64_t G = a.P.G;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kEvalBlock + threadIdx.x;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;   // idle lanes shadow the last design
    DesignState<T, D, NMAX> s;
    s.init(a.P, gg, a.r, a.z1, a.z2, a.gl, a.glw);
    const GlobalDraws<T> src{a.D, D};
    const int64_t M = a.D.M;
    const int64_t kb = static_cast<int64_t>(blockIdx.y) * a.slice_len;
    const int64_t ke = min(M, kb + a.slice_len);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        const double v = static_cast<double>(summand<T, D, NMAX>(a.P, s, src, k, a.A, a.D.K));
        s1 += v;
        s2 += v * v;
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(blockIdx.y) * 2 * G;
        out[g] = s1;
        out[G + g] = s2;
    }
}

typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mf_f4 mf_step(float a, float b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf_d4 mf_step(double a, double b, mf_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Tile geometry of the matrix-core sweep: designs g = p * Sn + l with prefix
// index p (axes < split) and suffix index l (axes >= split); a workgroup owns a
// 16 x 16 tile of (p, l) and a slice of draws.
struct MfmaGeom {
    int split;
    int64_t Pn, Sn;       // prefix and suffix counts
    int64_t tiles_l;      // tiles along the suffix index
    int chunk;            // draws staged per LDS chunk
};

// Sweep for grid designs with d >= 2, step prior, exact cutoff indicator.
// Phase A (matrix cores): for each draw of the chunk,
//   O[p][l] = sum_m Pre[p][m] Suf[l][m],
//   Pre[p][m] = prod_{j < split} v_j(p)[m],  Suf[l][m] = prod_{j >= split} v_j(l)[m],
//   v_j[m] = A_j[i_j][m] if the design's cutoff on axis j lies above the drawn one
//            (i_j >= thr_j(k)), else the draw's B_j[m]  (Gauss-Hermite weights in axis 0),
// i.e. the one-factor quadrature of P(x_j > max(c_j, t_j) all j) for all 256
// designs at once; each wavefront takes every fourth draw.
// Phase B (vector units): one design per thread, the bivariate normal part.
template <typename T, int D, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_eval_mfma(EvalArgs<T> a, MfmaGeom geo) {
    using acc_t = typename std::conditional<sizeof(T) == 8, mf_d4, mf_f4>::type;
    extern __shared__ __align__(16) char lds[];
    const int K = a.D.K;
    const int CH = geo.chunk;
    const int Kp = (K + 3) / 4 * 4;
    T* sO = reinterpret_cast<T*>(lds);                       // [CH][256]
    T* sB = sO + static_cast<size_t>(CH) * kEvalBlock;        // [CH][D][Kp]
    T* sb0 = sB + static_cast<size_t>(CH) * D * Kp;          // [CH]
    T* sb1 = sb0 + CH;
    T* smu1 = sb1 + CH;
    int* sthr = reinterpret_cast<int*>(smu1 + CH);            // [CH][D]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t p0 = (tile / geo.tiles_l) * 16, l0 = (tile % geo.tiles_l) * 16;
    const int64_t G = a.P.G;
    const int64_t M = a.D.M;
    const int mmax = a.P.mmax;

    // phase B design: row tid/16, column tid%16 of the tile
    const int64_t pB = p0 + tid / 16, lB = l0 + tid % 16;
    const bool validB = pB < geo.Pn && lB < geo.Sn;
    const int64_t g = validB ? pB * geo.Sn + lB : G - 1;
    DesignState<T, D, NMAX> st;
    st.init(a.P, g, a.r, a.z1, a.z2, a.gl, a.glw);

    // phase A operands: lane supplies row (p0 + lane%16) of Pre and column
    // (l0 + lane%16) of Suf at node m0 + lane/16
    const int r16 = lane & 15, kq = lane >> 4;
    const int64_t pA = p0 + r16, lA = l0 + r16;
    const bool rowA = pA < geo.Pn, colA = lA < geo.Sn;
    int iA[D];
    {
        int64_t rem = (rowA ? pA : 0) * geo.Sn + (colA ? lA : 0);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            iA[j] = static_cast<int>(rem / a.P.stride[j]);
            rem -= static_cast<int64_t>(iA[j]) * a.P.stride[j];
        }
    }

    const int64_t kb = static_cast<int64_t>(blockIdx.y) * a.slice_len;
    const int64_t ke = min(M, kb + a.slice_len);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k0 = kb; k0 < ke; k0 += CH) {
        const int nk = static_cast<int>(min<int64_t>(CH, ke - k0));
        __syncthreads();
        // stage the chunk's draws
        for (int e = tid; e < nk * D * Kp; e += kEvalBlock) {
            const int i = e / (D * Kp), rem = e % (D * Kp), j = rem / Kp, m = rem % Kp;
            sB[e] = m < K ? a.D.B[(k0 + i) * D * K + j * K + m] : T(0);
        }
        for (int e = tid; e < nk; e += kEvalBlock) {
            sb0[e] = a.D.b0[k0 + e];
            sb1[e] = a.D.b1[k0 + e];
            smu1[e] = a.D.mu1[k0 + e];
        }
        for (int e = tid; e < nk * D; e += kEvalBlock) {
            const int i = e / D, j = e % D;
            sthr[e] = a.D.thr[j * M + k0 + i];
        }
        __syncthreads();
        // phase A: overlaps of the tile, one draw per wavefront at a time
        for (int i = wave; i < nk; i += kEvalBlock / 64) {
            bool fl[D];
#pragma unroll
            for (int j = 0; j < D; ++j) fl[j] = iA[j] >= sthr[i * D + j];
            const T* Bi = sB + static_cast<size_t>(i) * D * Kp;
            acc_t c = {0, 0, 0, 0};
            for (int m0 = 0; m0 < Kp; m0 += 4) {
                const int m = m0 + kq;
                T pre = T(1), suf = T(1);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const T av = m < K ? a.A[(static_cast<int64_t>(j) * K + m) * mmax + iA[j]] : T(0);
                    const T v = fl[j] ? av : Bi[j * Kp + m];
                    if (j < geo.split) pre *= v; else suf *= v;
                }
                c = mf_step(rowA ? pre : T(0), colA ? suf : T(0), c);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                sO[static_cast<size_t>(i) * kEvalBlock + mfma16_row<T>(kq, v) * 16 + r16] = c[v];
        }
        __syncthreads();
        // phase B: bivariate normal part for this thread's design
        for (int i = 0; i < nk; ++i) {
            const T O = sO[static_cast<size_t>(i) * kEvalBlock + tid];
            const T mu2 = st.srI * (sb0[i] + sb1[i] * O * st.invr);
            const T h = st.z1 - smu1[i], kq2 = st.z2 - mu2;
            T p;
            if (a.P.zinf == 0) p = bvn_cdf<NMAX>(h, kq2, st.bc, st.w, st.n);
            else if (a.P.zinf == 1) p = norm_cdf(kq2);
            else if (a.P.zinf == 2) p = norm_cdf(h);
            else p = T(1);
            const double v = static_cast<double>(T(1) - p);
            s1 += v;
            s2 += v * v;
        }
    }
    if (validB) {
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

template <typename T>
size_t mfma_lds_bytes(int chunk, int d, int K) {
    const int Kp = (K + 3) / 4 * 4;
    return sizeof(T) * static_cast<size_t>(chunk) * (kEvalBlock + static_cast<size_t>(d) * Kp + 3) +
           sizeof(int) * static_cast<size_t>(chunk) * d;
}

// Prefix/suffix split with the least tile padding (ties: the later split).
MfmaGeom mfma_geometry(const bmd_problem* p, int prec) {
    MfmaGeom geo{};
    const int d = p->P.d;
    double best = 1e300;
    for (int s = 1; s < d; ++s) {
        int64_t P = 1, S = 1;
        for (int j = 0; j < s; ++j) P *= p->P.m[j];
        for (int j = s; j < d; ++j) S *= p->P.m[j];
        const double padded = static_cast<double>((P + 15) / 16 * 16) * static_cast<double>((S + 15) / 16 * 16);
        if (padded <= best) {
            best = padded;
            geo.split = s;
            geo.Pn = P;
            geo.Sn = S;
        }
    }
    geo.tiles_l = (geo.Sn + 15) / 16;
    const int K = p->tab[prec].K;
    int ch = 32;
    const size_t cap = 48 * 1024;
    while (ch > 4 && (prec == BMD_FP64 ? mfma_lds_bytes<double>(ch, d, K) : mfma_lds_bytes<float>(ch, d, K)) > cap)
        ch /= 2;
    geo.chunk = ch;
    return geo;
}

template <typename T, int NMAX>
hipError_t launch_typed(const bmd_problem* p, int prec, const EvalArgs<T>& a, int n_slices, hipStream_t s) {
    const int d = p->P.d;
    if (use_mfma_sweep(p)) {
        const MfmaGeom geo = mfma_geometry(p, prec);
        const int64_t tiles = ((geo.Pn + 15) / 16) * geo.tiles_l;
        const dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(n_slices));
        const size_t lds = mfma_lds_bytes<T>(geo.chunk, d, a.D.K);
        switch (d) {
            case 2: hipLaunchKernelGGL((k_eval_mfma<T, 2, NMAX>), grid, dim3(kEvalBlock), lds, s, a, geo); break;
            case 3: hipLaunchKernelGGL((k_eval_mfma<T, 3, NMAX>), grid, dim3(kEvalBlock), lds, s, a, geo); break;
            case 4: hipLaunchKernelGGL((k_eval_mfma<T, 4, NMAX>), grid, dim3(kEvalBlock), lds, s, a, geo); break;
            case 5: hipLaunchKernelGGL((k_eval_mfma<T, 5, NMAX>), grid, dim3(kEvalBlock), lds, s, a, geo); break;
            default: hipLaunchKernelGGL((k_eval_mfma<T, 6, NMAX>), grid, dim3(kEvalBlock), lds, s, a, geo); break;
        }
        return hipGetLastError();
    }
    const dim3 grid(static_cast<unsigned>((p->P.G + kEvalBlock - 1) / kEvalBlock), static_cast<unsigned>(n_slices));
    switch (d) {
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

// The matrix-core sweep covers grid problems with at least two biomarkers,
// the step prior and the exact cutoff indicator; the rest use the direct one.
bool use_mfma_sweep(const bmd_problem* p) {
    return p->grid && p->P.d >= 2 && p->P.effect == BMD_EFFECT_STEP && p->P.width == 0.0 && !p->force_direct;
}

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
