// Smoothing of the estimated surface and its argmax (Sec. 2.3: borrow strength
// from neighbouring designs, then take the best point).
//
// The product-Gaussian Nadaraya-Watson smoother factorises: with row-normalised
// one-axis matrices W_j[i][h] = exp(-((q_i - q_h)/b_j)^2/2) / sum_h' (...),
// S = W_0 x_0 W_1 x_1 ... f, applied one axis at a time.
#include <cfloat>

#include "bmd_internal.hpp"
#include "device_math.hpp"

namespace bmd {
namespace {

template <typename T>
__global__ void k_smooth_axis(int64_t G, int m, int64_t inner, const T* __restrict__ W,
                              const double* __restrict__ in, double* __restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= G) return;
    const int64_t s = t % inner;
    const int64_t oi = t / inner;
    const int i = static_cast<int>(oi % m);
    const int64_t o = oi / m;
    const double* src = in + o * m * inner + s;
    const T* Wi = W + static_cast<int64_t>(i) * m;
    T acc = T(0);
    for (int h = 0; h < m; ++h) acc += Wi[h] * static_cast<T>(src[static_cast<int64_t>(h) * inner]);
    out[t] = static_cast<double>(acc);
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

}  // namespace

hipError_t launch_smooth(const bmd_problem* p, int prec, const double* in, double* out, double* tmp,
                         hipStream_t s) {
    const int d = p->P.d;
    const int64_t G = p->P.G;
    const double* src = in;
    for (int j = 0; j < d; ++j) {
        double* dst = ((d - 1 - j) % 2 == 0) ? out : tmp;
        const unsigned blocks = static_cast<unsigned>((G + 255) / 256);
        if (prec == BMD_FP64)
            hipLaunchKernelGGL(k_smooth_axis<double>, dim3(blocks), dim3(256), 0, s, G, p->P.m[j], p->P.stride[j],
                               p->d_W + p->w_off[j], src, dst);
        else
            hipLaunchKernelGGL(k_smooth_axis<float>, dim3(blocks), dim3(256), 0, s, G, p->P.m[j], p->P.stride[j],
                               p->d_Wf + p->w_off[j], src, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        src = dst;
    }
    return hipSuccess;
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
