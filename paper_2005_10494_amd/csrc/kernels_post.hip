// Smoothing of the estimated surface and its argmax (Sec. 2.3: borrow strength
// from neighbouring designs, then take the best point).  Smoothing runs on the
// matrix cores (FP64 16x16x4 or FP32 16x16x4 MFMA).
//
// The product-Gaussian Nadaraya-Watson smoother factorises: with row-normalised
// one-axis matrices W_j[i][h] = exp(-((q_i - q_h)/b_j)^2/2) / sum_h' (...),
// S = W_0 x_0 W_1 x_1 ... f, applied one axis at a time.
#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {
namespace {

typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// One 16x16x4 matrix-core step: C += A (16x4) B (4x16); operand and result
// layout as described at mfma16_row.
__device__ __forceinline__ mfma_d4 mfma_step(double a, double b, mfma_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma_f4 mfma_step(float a, float b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One separable smoothing pass as a GEMM on the matrix cores:
//   out(i, c) = sum_h W[i][h] in(h, c),  i, h < m,  c < C,
// where the columns c run over every (outer, inner) pair of the axis, the
// element (h, c) of the surface sitting at (c / inner) m inner + h inner +
// c % inner.  One wavefront owns CT tiles of 16 columns and the NI row blocks
// of 16 starting at block blockIdx.y * NI; with one group of row blocks per
// column tile each surface value is loaded once per pass.  W (m x m) stays in
// the caches.
// T is the arithmetic type (FP64, or FP32 converting the FP64 surface on load
// and accumulating in FP32).
template <typename T, int NI, int CT>
__global__ __launch_bounds__(64) void k_smooth_mfma(const T* __restrict__ W, int m, const double* __restrict__ in,
                                                    double* __restrict__ out, int64_t C, int64_t inner) {
    using acc_t = typename std::conditional<sizeof(T) == 8, mfma_d4, mfma_f4>::type;
    const int lane = threadIdx.x;
    const int r = lane & 15, kq = lane >> 4;
    bool valid[CT];
    int64_t base[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int64_t c = (static_cast<int64_t>(blockIdx.x) * CT + t) * 16 + r;
        valid[t] = c < C;
        base[t] = valid[t] ? (c / inner) * m * inner + c % inner : 0;
    }
    const int nblk = (m + 15) / 16;
    {
        const int b0 = blockIdx.y * NI;
        acc_t acc[CT][NI];
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int ib = 0; ib < NI; ++ib) acc[t][ib] = acc_t{0, 0, 0, 0};
        for (int h0 = 0; h0 < m; h0 += 4) {
            const int h = h0 + kq;
            T b[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) b[t] = (h < m && valid[t]) ? static_cast<T>(in[base[t] + h * inner]) : T(0);
#pragma unroll
            for (int ib = 0; ib < NI; ++ib) {
                if (b0 + ib < nblk) {   // wave-uniform
                    const int i = (b0 + ib) * 16 + r;
                    const T a = (i < m && h < m) ? W[static_cast<int64_t>(i) * m + h] : T(0);
#pragma unroll
                    for (int t = 0; t < CT; ++t) acc[t][ib] = mfma_step(a, b[t], acc[t][ib]);
                }
            }
        }
#pragma unroll
        for (int ib = 0; ib < NI; ++ib) {
            if (b0 + ib < nblk) {
#pragma unroll
                for (int t = 0; t < CT; ++t) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int io = (b0 + ib) * 16 + mfma16_row<T>(kq, v);
                        if (io < m && valid[t]) out[base[t] + io * inner] = static_cast<double>(acc[t][ib][v]);
                    }
                }
            }
        }
    }
}

// The pass along the last axis (inner = 1) with a short axis: the 16 CT
// columns of a wavefront are consecutive rows of m values, one contiguous
// block, which the lanes copy to LDS (row-padded to m + 1) with coalesced
// loads; the matrix cores take their B operands from there, and the results
// go back through the same LDS block to coalesced stores.  (Read straight
// from the surface, each load of the 16 columns touches 16 rows m values
// apart.)  Same products in the same order as k_smooth_mfma, so the results
// are identical.
constexpr int kRowsMaxM = 64;

template <typename T, int NI, int CT>
__global__ __launch_bounds__(64) void k_smooth_rows(const T* __restrict__ W, int m, const double* __restrict__ in,
                                                    double* __restrict__ out, int64_t C) {
    using acc_t = typename std::conditional<sizeof(T) == 8, mfma_d4, mfma_f4>::type;
    extern __shared__ __align__(16) char smem[];
    T* tile = reinterpret_cast<T*>(smem);   // [16 CT][m + 1]
    const int lane = threadIdx.x;
    const int r = lane & 15, kq = lane >> 4;
    const int ld = m + 1;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * 16 * CT;
    const int ncol = static_cast<int>(min<int64_t>(16 * CT, C - c0));
    const int n_el = ncol * m, n_all = 16 * CT * m;
    const double* src = in + c0 * m;
    const int q64 = 64 / m, r64 = 64 - (64 / m) * m;
    {
        int col = lane / m, h = lane - (lane / m) * m;
        for (int e = lane; e < n_all; e += 64) {
            tile[col * ld + h] = e < n_el ? static_cast<T>(src[e]) : T(0);
            col += q64;
            h += r64;
            if (h >= m) {
                h -= m;
                ++col;
            }
        }
    }
    __syncthreads();
    const int nblk = (m + 15) / 16;
    const int b0 = blockIdx.y * NI;
    acc_t acc[CT][NI];
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int ib = 0; ib < NI; ++ib) acc[t][ib] = acc_t{0, 0, 0, 0};
    for (int h0 = 0; h0 < m; h0 += 4) {
        const int h = h0 + kq;
        T bv[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) bv[t] = h < m ? tile[(t * 16 + r) * ld + h] : T(0);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib) {
            if (b0 + ib < nblk) {   // wave-uniform
                const int i = (b0 + ib) * 16 + r;
                const T a = (i < m && h < m) ? W[static_cast<int64_t>(i) * m + h] : T(0);
#pragma unroll
                for (int t = 0; t < CT; ++t) acc[t][ib] = mfma_step(a, bv[t], acc[t][ib]);
            }
        }
    }
    __syncthreads();   // every B operand is read before the block is overwritten
#pragma unroll
    for (int ib = 0; ib < NI; ++ib) {
        if (b0 + ib < nblk) {
#pragma unroll
            for (int t = 0; t < CT; ++t) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int io = (b0 + ib) * 16 + mfma16_row<T>(kq, v);
                    if (io < m) tile[(t * 16 + r) * ld + io] = acc[t][ib][v];
                }
            }
        }
    }
    __syncthreads();
    double* dst = out + c0 * m;
    {
        int col = lane / m, h = lane - (lane / m) * m;
        for (int e = lane; e < n_el; e += 64) {
            dst[e] = static_cast<double>(tile[col * ld + h]);
            col += q64;
            h += r64;
            if (h >= m) {
                h -= m;
                ++col;
            }
        }
    }
}

template <typename T, int CT, int NI>
void launch_smooth_rows(const T* W, int m, const double* in, double* out, int64_t C, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((C + 16 * CT - 1) / (16 * CT)), 1);
    const size_t lds = sizeof(T) * 16 * CT * static_cast<size_t>(m + 1);
    hipLaunchKernelGGL((k_smooth_rows<T, NI, CT>), grid, dim3(64), lds, s, W, m, in, out, C);
}

template <typename T, int CT, int NI>
void launch_smooth_group(const T* W, int m, const double* in, double* out, int64_t C, int64_t inner, hipStream_t s) {
    const int nblk = (m + 15) / 16;
    const dim3 grid(static_cast<unsigned>((C + 16 * CT - 1) / (16 * CT)), static_cast<unsigned>((nblk + NI - 1) / NI));
    hipLaunchKernelGGL((k_smooth_mfma<T, NI, CT>), grid, dim3(64), 0, s, W, m, in, out, C, inner);
}

// Surfaces with many columns (at least 4,096 tiles of 16): two column tiles
// per wavefront and all row blocks in one group, each value read once
// (measured in FP32 on the 24^5 surface: 3.0 TB/s with one row block per
// wavefront and columns along the inner index only, 3.3 with one tile and
// all row blocks, 3.8 with two tiles, 3.3 with four).  Fewer columns: one tile
// and one row block per wavefront, so that small grids still spread over the
// compute units (a 97 x 97 grid has 97 columns per pass).
template <typename T>
void launch_smooth_pass(const T* W, int m, const double* in, double* out, int64_t C, int64_t inner, hipStream_t s) {
    const int nblk = (m + 15) / 16;
    if ((C + 15) / 16 < 4096)
        launch_smooth_group<T, 1, 1>(W, m, in, out, C, inner, s);
    else if (inner == 1 && m <= kRowsMaxM)   // all row blocks in one wavefront (nblk <= 4)
        nblk <= 1   ? launch_smooth_rows<T, 2, 1>(W, m, in, out, C, s)
        : nblk <= 2 ? launch_smooth_rows<T, 2, 2>(W, m, in, out, C, s)
                    : launch_smooth_rows<T, 2, 4>(W, m, in, out, C, s);
    else if (nblk <= 1)
        launch_smooth_group<T, 2, 1>(W, m, in, out, C, inner, s);
    else if (nblk <= 2)
        launch_smooth_group<T, 2, 2>(W, m, in, out, C, inner, s);
    else if (nblk <= 4)
        launch_smooth_group<T, 2, 4>(W, m, in, out, C, inner, s);
    else if (nblk <= 8)
        launch_smooth_group<T, 2, 8>(W, m, in, out, C, inner, s);
    else
        launch_smooth_group<T, 2, 16>(W, m, in, out, C, inner, s);
}

__device__ __forceinline__ bool better(double va, int64_t ia, double vb, int64_t ib) {
    return va > vb || (va == vb && ia < ib);
}

__device__ __forceinline__ void wave_best(double& v, int64_t& i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(v, off);
        const int64_t oi = __shfl_down(i, off);
        if (better(ov, oi, v, i)) { v = ov; i = oi; }
    }
}

__device__ void block_best(double& v, int64_t& i) {
    __shared__ double sv[16];
    __shared__ int64_t si[16];
    wave_best(v, i);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sv[wid] = v; si[wid] = i; }
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    if (wid == 0) {
        v = lane < nw ? sv[lane] : -DBL_MAX;
        i = lane < nw ? si[lane] : INT64_MAX;
        wave_best(v, i);
    }
}

// Stage 1: per-block best of a grid-strided range; NaN counts as -inf.
__global__ void k_argmax_part(const double* __restrict__ x, int64_t n, double* __restrict__ pv,
                              int64_t* __restrict__ pi) {
    double v = -DBL_MAX;
    int64_t i = INT64_MAX;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double xv = x[t];
        if (!(xv != xv) && better(xv, t, v, i)) { v = xv; i = t; }
    }
    block_best(v, i);
    if (threadIdx.x == 0) { pv[blockIdx.x] = v; pi[blockIdx.x] = i; }
}

// Stage 2: one block over the partial results; result in pv[0], pi[0].
__global__ void k_argmax_final(int n_part, double* __restrict__ pv, int64_t* __restrict__ pi) {
    double v = -DBL_MAX;
    int64_t i = INT64_MAX;
    for (int t = threadIdx.x; t < n_part; t += blockDim.x)
        if (better(pv[t], pi[t], v, i)) { v = pv[t]; i = pi[t]; }
    block_best(v, i);
    __syncthreads();
    if (threadIdx.x == 0) { pv[0] = v; pi[0] = i; }
}

// Surfaces where some designs have no value (NaN): the smoother over the
// designs that have one is the ratio of the smoothed zero-filled surface and
// the smoothed indicator of those designs (the row normalisation cancels).
__global__ void k_mask_split(int64_t G, const double* __restrict__ in, double* __restrict__ f0,
                             double* __restrict__ v) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const double x = in[g];
    const bool ok = !(x != x);
    f0[g] = ok ? x : 0.0;
    v[g] = ok ? 1.0 : 0.0;
}

// Designs without a value stay NaN; every other one has a positive indicator
// sum (its own weight).
__global__ void k_mask_ratio(int64_t G, const double* __restrict__ in, const double* __restrict__ den,
                             double* __restrict__ out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const double x = in[g];
    out[g] = x != x ? x : out[g] / den[g];
}

}  // namespace

// ---------------------------------------------------------------------------
// The smoothed surface at a continuous design q (the fitted surface of Sec.
// 2.3 between grid points) with its first and second derivatives in q:
//   S(q) = N(q) / D(q),  N = sum_h K(q, q_h) f_h,  D = sum_h K(q, q_h),
//   K = prod_j k_j,  k_j = exp(-t_j^2 / 2),  t_j = (q_j - x_j,h) / b_j,
// over the grid designs whose value is not NaN.  With u_j = -t_j / b_j,
// dK/dq_j = K u_j and d2K/dq_j dq_l = K (u_j u_l - [j = l] / b_j^2); the
// kernels reduce sum K f (1, u_j, u_j u_l) and sum K (1, u_j, u_j u_l) and
// the host adds the diagonal terms.  FP64 throughout.
// ---------------------------------------------------------------------------

constexpr int kLocalBlocks = 1024;

// Accumulators per side: 1 + D + D (D + 1) / 2.
template <int D>
constexpr int local_acc() {
    return 1 + D + D * (D + 1) / 2;
}

struct LocalArgs {
    DevProblem P;
    const double* in;
    double q[kMaxDim];
    double lo[kMaxDim], hi[kMaxDim];   // axis ranges of the grid
    double bw[kMaxDim];                // bandwidths
    double* partials;                  // [kLocalBlocks][2 * local_acc]
};

template <int D>
__global__ __launch_bounds__(256) void k_smooth_local(LocalArgs a) {
    constexpr int NA = local_acc<D>();
    __shared__ double red[256];
    double accf[NA], accw[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) accf[i] = accw[i] = 0.0;
    const int64_t G = a.P.G;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < G;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double v = a.in[g];
        if (v != v) continue;   // NaN designs carry no weight
        double w = 1.0, u[D];
        int64_t rem = g;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int idx = static_cast<int>(rem / a.P.stride[j]);
            rem -= static_cast<int64_t>(idx) * a.P.stride[j];
            const double t = (a.q[j] - grid_coord(a.lo[j], a.hi[j], idx, a.P.m[j])) / a.bw[j];
            w *= exp(-0.5 * t * t);
            u[j] = -t / a.bw[j];
        }
        const double wv = w * v;
        accf[0] += wv;
        accw[0] += w;
        int k = 1 + D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            accf[1 + j] = fma(wv, u[j], accf[1 + j]);
            accw[1 + j] = fma(w, u[j], accw[1 + j]);
#pragma unroll
            for (int l = j; l < D; ++l, ++k) {
                const double uu = u[j] * u[l];
                accf[k] = fma(wv, uu, accf[k]);
                accw[k] = fma(w, uu, accw[k]);
            }
        }
    }
    // block sums in a fixed tree order, one accumulator at a time
    double* out = a.partials + static_cast<int64_t>(blockIdx.x) * 2 * NA;
#pragma unroll
    for (int i = 0; i < 2 * NA; ++i) {
        red[threadIdx.x] = i < NA ? accf[i] : accw[i - NA];
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[i] = red[0];
        __syncthreads();
    }
}

// Sums of the block partials in block order: out[i] = sum_b partials[b][i].
__global__ __launch_bounds__(64) void k_smooth_local_final(const double* __restrict__ partials, int n_blocks,
                                                           int n_acc, double* __restrict__ out) {
    const int i = threadIdx.x;
    if (i >= n_acc) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += partials[static_cast<int64_t>(b) * n_acc + i];
    out[i] = s;
}

hipError_t launch_smooth_masked(const bmd_problem* p, int prec, const double* in, double* out, double* ws,
                                hipStream_t s) {
    const int64_t G = p->P.G;
    double* tmp = ws;
    double* f0 = ws + G;
    double* v = ws + 2 * G;
    double* den = ws + 3 * G;
    const dim3 grid(static_cast<unsigned>((G + 255) / 256));
    hipLaunchKernelGGL(k_mask_split, grid, dim3(256), 0, s, G, in, f0, v);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_smooth(p, prec, f0, out, tmp, s);
    if (e == hipSuccess) e = launch_smooth(p, prec, v, den, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mask_ratio, grid, dim3(256), 0, s, G, in, den, out);
    return hipGetLastError();
}

hipError_t launch_smooth(const bmd_problem* p, int prec, const double* in, double* out, double* tmp,
                         hipStream_t s) {
    const int d = p->P.d;
    const int64_t G = p->P.G;
    const double* src = in;
    for (int j = 0; j < d; ++j) {
        double* dst = ((d - 1 - j) % 2 == 0) ? out : tmp;
        const int m = p->P.m[j];
        const int64_t inner = p->P.stride[j];
        const int64_t C = G / m;   // columns: every (outer, inner) pair of axis j
        if (prec == BMD_FP64)
            launch_smooth_pass<double>(p->d_W + p->w_off[j], m, src, dst, C, inner, s);
        else
            launch_smooth_pass<float>(p->d_Wf + p->w_off[j], m, src, dst, C, inner, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        src = dst;
    }
    return hipSuccess;
}

size_t smooth_local_bytes() { return sizeof(double) * (static_cast<size_t>(kLocalBlocks) + 1) * 2 * local_acc<kMaxDim>(); }

hipError_t launch_smooth_local(const bmd_problem* p, const double* in, const double* q, const double* lo,
                               const double* hi, double* ws, double* out, hipStream_t s) {
    LocalArgs a{};
    a.P = p->P;
    a.in = in;
    for (int j = 0; j < p->P.d; ++j) {
        a.q[j] = q[j];
        a.lo[j] = lo[j];
        a.hi[j] = hi[j];
        a.bw[j] = p->desc.bandwidth[j];
    }
    a.partials = ws;
    const int64_t G = p->P.G;
    const int blocks = static_cast<int>(std::min<int64_t>(kLocalBlocks, (G + 255) / 256));
    int na = 0;
    switch (p->P.d) {
        case 1: hipLaunchKernelGGL(k_smooth_local<1>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<1>(); break;
        case 2: hipLaunchKernelGGL(k_smooth_local<2>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<2>(); break;
        case 3: hipLaunchKernelGGL(k_smooth_local<3>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<3>(); break;
        case 4: hipLaunchKernelGGL(k_smooth_local<4>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<4>(); break;
        case 5: hipLaunchKernelGGL(k_smooth_local<5>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<5>(); break;
        default: hipLaunchKernelGGL(k_smooth_local<6>, dim3(blocks), dim3(256), 0, s, a); na = local_acc<6>(); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_local_final, dim3(1), dim3(64), 0, s, ws, blocks, 2 * na, out);
    return hipGetLastError();
}

hipError_t launch_argmax(const bmd_problem* p, const double* v, int64_t n, double* part_v, int64_t* part_i,
                         int n_part, hipStream_t s) {
    (void)p;
    hipLaunchKernelGGL(k_argmax_part, dim3(n_part), dim3(256), 0, s, v, n, part_v, part_i);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, s, n_part, part_v, part_i);
    return hipGetLastError();
}

}  // namespace bmd
