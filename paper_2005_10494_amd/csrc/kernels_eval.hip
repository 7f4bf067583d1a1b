// Grid sweep of the expected-power estimate (Formula 5): one thread per design,
// draw slices across workgroups, FP64 per-design sums reduced in fixed order.
// The summand itself is in eval_core.hpp; T is the integrand type.
#include <type_traits>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "eval_core.hpp"
#include "sweep_body.hpp"

namespace bmd {
namespace {

// VAR: also the per-design sums of squares (only when a variance is asked for).
template <typename T, int D, int NMAX, bool VAR>
__global__ __launch_bounds__(kEvalBlock) void k_eval_direct(EvalArgs<T> a) {
    direct_body<T, D, NMAX, VAR ? kSquares : kSums>(a, blockIdx.x, blockIdx.y);
}

// Tile of workgroup (x, y): the tiles of one draw slice lie along x, so every
// XCD works on the slice whose draws its L2 holds.  Workgroups go to the XCDs
// round-robin by linear index, and a row of tiles whose length is a multiple
// of 8 would give XCD j the tiles x = j mod 8 in every slice; the tiles' costs
// differ with their designs' node counts, which follow the grid axes, so the
// tile is rotated by the slice index and each XCD gets every tile class.
__device__ __forceinline__ unsigned sweep_tile() { return (blockIdx.x + blockIdx.y) % gridDim.x; }

// FP32 with up to three biomarkers: at most 96 VGPRs, so that five wavefronts
// share each SIMD (more axes would spill the node coefficients).
template <typename T, int D, int NMAX, bool VAR>
__global__ __launch_bounds__(kEvalBlock, sizeof(T) == 4 && D <= 3 ? 5 : 1) void k_eval_mfma(EvalArgs<T> a, MfmaGeom geo) {
    extern __shared__ __align__(16) char lds[];
    mfma_tile_body<T, D, NMAX, VAR ? kSquares : kSums>(a, geo, sweep_tile(), blockIdx.y, lds);
}

// The same sweeps with the summands' derivatives in alpha_1 as second sums.
template <typename T, int D, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_eval_direct_da(EvalArgs<T> a) {
    direct_body<T, D, NMAX, kDAlpha>(a, blockIdx.x, blockIdx.y);
}
template <typename T, int D, int NMAX>
__global__ __launch_bounds__(kEvalBlock) void k_eval_mfma_da(EvalArgs<T> a, MfmaGeom geo) {
    extern __shared__ __align__(16) char lds[];
    mfma_tile_body<T, D, NMAX, kDAlpha>(a, geo, sweep_tile(), blockIdx.y, lds);
}

// mean = sums / M in slice order; second: nothing (mode 0), the sample
// variance from the sums of squares (1), the second sums / M (2).
__global__ void k_finalize(int64_t G, int64_t M, int n_slices, const double* __restrict__ part,
                           double* __restrict__ mean, double* __restrict__ second, int mode) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double s1 = 0.0, s2 = 0.0;
    for (int s = 0; s < n_slices; ++s) s1 += part[static_cast<int64_t>(s) * 2 * G + g];
    const double Md = static_cast<double>(M);
    mean[g] = s1 / Md;
    if (mode != 0) {
        for (int s = 0; s < n_slices; ++s) s2 += part[static_cast<int64_t>(s) * 2 * G + G + g];
        second[g] = mode == 2 ? s2 / Md : M > 1 ? fmax(0.0, (s2 - s1 * s1 / Md) / (Md - 1.0)) : 0.0;
    }
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
    // Largest chunk of at most 32 draws that keeps every wavefront pass of
    // phase A full (a multiple of 8 in FP32: two draws per pass, four
    // wavefronts; of 4 in FP64) within the LDS share of the resident
    // workgroups: five per compute unit for FP32 with up to three biomarkers
    // (32 KB each of 160 KB), else four (40 KB); FP64 holds two (its
    // registers allow no more), 64 KB each.
    const int step = prec == BMD_FP64 ? 4 : 8;
    const size_t cap = prec == BMD_FP64 ? 64 * 1024 : d <= 3 ? 32 * 1024 : 40 * 1024;
    int ch = 32;
    while (ch > step && (prec == BMD_FP64 ? mfma_lds_bytes<double>(ch, d, K) : mfma_lds_bytes<float>(ch, d, K)) > cap)
        ch -= step;
    geo.chunk = ch;
    return geo;
}

// The sweep kernel for biomarker count d.
template <typename T, int NMAX>
const void* sweep_kernel_da(int d, bool mf) {
    if (mf) {
        switch (d) {
            case 2: return reinterpret_cast<const void*>(k_eval_mfma_da<T, 2, NMAX>);
            case 3: return reinterpret_cast<const void*>(k_eval_mfma_da<T, 3, NMAX>);
            case 4: return reinterpret_cast<const void*>(k_eval_mfma_da<T, 4, NMAX>);
            case 5: return reinterpret_cast<const void*>(k_eval_mfma_da<T, 5, NMAX>);
            default: return reinterpret_cast<const void*>(k_eval_mfma_da<T, 6, NMAX>);
        }
    }
    switch (d) {
        case 1: return reinterpret_cast<const void*>(k_eval_direct_da<T, 1, NMAX>);
        case 2: return reinterpret_cast<const void*>(k_eval_direct_da<T, 2, NMAX>);
        case 3: return reinterpret_cast<const void*>(k_eval_direct_da<T, 3, NMAX>);
        case 4: return reinterpret_cast<const void*>(k_eval_direct_da<T, 4, NMAX>);
        case 5: return reinterpret_cast<const void*>(k_eval_direct_da<T, 5, NMAX>);
        default: return reinterpret_cast<const void*>(k_eval_direct_da<T, 6, NMAX>);
    }
}

template <typename T, int NMAX, bool VAR>
const void* sweep_kernel(int d, bool mf) {
    if (mf) {
        switch (d) {
            case 2: return reinterpret_cast<const void*>(k_eval_mfma<T, 2, NMAX, VAR>);
            case 3: return reinterpret_cast<const void*>(k_eval_mfma<T, 3, NMAX, VAR>);
            case 4: return reinterpret_cast<const void*>(k_eval_mfma<T, 4, NMAX, VAR>);
            case 5: return reinterpret_cast<const void*>(k_eval_mfma<T, 5, NMAX, VAR>);
            default: return reinterpret_cast<const void*>(k_eval_mfma<T, 6, NMAX, VAR>);
        }
    }
    switch (d) {
        case 1: return reinterpret_cast<const void*>(k_eval_direct<T, 1, NMAX, VAR>);
        case 2: return reinterpret_cast<const void*>(k_eval_direct<T, 2, NMAX, VAR>);
        case 3: return reinterpret_cast<const void*>(k_eval_direct<T, 3, NMAX, VAR>);
        case 4: return reinterpret_cast<const void*>(k_eval_direct<T, 4, NMAX, VAR>);
        case 5: return reinterpret_cast<const void*>(k_eval_direct<T, 5, NMAX, VAR>);
        default: return reinterpret_cast<const void*>(k_eval_direct<T, 6, NMAX, VAR>);
    }
}

template <typename T, int NMAX>
hipError_t launch_typed(const bmd_problem* p, int prec, const EvalArgs<T>& a, int n_slices, int mode,
                        hipStream_t s) {
    const int d = p->P.d;
    const bool mf = use_mfma_sweep(p);
    const void* k = mode == kDAlpha    ? sweep_kernel_da<T, NMAX>(d, mf)
                    : mode == kSquares ? sweep_kernel<T, NMAX, true>(d, mf)
                                       : sweep_kernel<T, NMAX, false>(d, mf);
    if (mf) {
        MfmaGeom geo = mfma_geometry(p, prec);
        const int64_t tiles = ((geo.Pn + 15) / 16) * geo.tiles_l;
        const size_t lds = mfma_lds_bytes<T>(geo.chunk, d, a.D.K);
        void* args[] = {const_cast<EvalArgs<T>*>(&a), &geo};
        return hipLaunchKernel(k, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(n_slices)),
                               dim3(kEvalBlock), args, lds, s);
    }
    void* args[] = {const_cast<EvalArgs<T>*>(&a)};
    return hipLaunchKernel(k, dim3(static_cast<unsigned>((p->P.G + kEvalBlock - 1) / kEvalBlock),
                                   static_cast<unsigned>(n_slices)),
                           dim3(kEvalBlock), args, 0, s);
}

// Resident workgroups per compute unit of the sweep kernel eval_grid launches
// (the variant without sums of squares).
template <typename T, int NMAX>
int resident_typed(const bmd_problem* p, int prec) {
    const bool mf = use_mfma_sweep(p);
    size_t lds = 0;
    if (mf) {
        const MfmaGeom geo = mfma_geometry(p, prec);
        lds = mfma_lds_bytes<T>(geo.chunk, p->P.d, p->tab[prec].K);
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_kernel<T, NMAX, false>(p->P.d, mf), kEvalBlock,
                                                     lds) != hipSuccess ||
        nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

}  // namespace

// The matrix-core sweep covers grid problems with at least two biomarkers,
// the step prior and the exact cutoff indicator; the rest use the direct one.
bool use_mfma_sweep(const bmd_problem* p) {
    return p->grid && p->P.design_space == BMD_DESIGN_CUTOFFS && p->P.d >= 2 && p->P.effect == BMD_EFFECT_STEP &&
           p->P.width == 0.0 && !p->force_direct;
}

MfmaGeom sweep_geometry(const bmd_problem* p, int prec) { return mfma_geometry(p, prec); }

int64_t sweep_tiles(const bmd_problem* p, int prec) {
    if (use_mfma_sweep(p)) {
        const MfmaGeom geo = mfma_geometry(p, prec);
        return ((geo.Pn + 15) / 16) * geo.tiles_l;
    }
    return (p->P.G + kEvalBlock - 1) / kEvalBlock;
}

int sweep_blocks_per_cu(const bmd_problem* p, int prec) {
    if (p->P.design_space == BMD_DESIGN_ALPHA3) return three_blocks_per_cu(prec);
    if (p->P.design_space == BMD_DESIGN_NESTED3) return nested3_blocks_per_cu(prec);
    if (p->P.design_space == BMD_DESIGN_NESTED4) return nested4_blocks_per_cu(prec);
    if (p->P.design_space == BMD_DESIGN_ALPHA4) return four_blocks_per_cu(prec);
    return prec == BMD_FP64 ? resident_typed<double, 24>(p, prec) : resident_typed<float, 12>(p, prec);
}

int sweep_chunk(const bmd_problem* p, int prec) {
    return use_mfma_sweep(p) ? mfma_geometry(p, prec).chunk : 1;
}

int64_t sweep_staged_bytes_per_draw(const bmd_problem* p, int prec) {
    if (!use_mfma_sweep(p)) return 0;
    const int64_t T = prec == BMD_FP64 ? 8 : 4, d = p->P.d, K = p->tab[prec].K;
    return d * K * T + 4 * T + 4 * d;
}

hipError_t launch_eval_grid(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, bool want_var, hipStream_t s) {
    if (p->P.design_space == BMD_DESIGN_ALPHA3)
        return launch_eval_three(p, prec, M, ws, partials, n_slices, slice_len, want_var, s);
    if (p->P.design_space == BMD_DESIGN_NESTED3)
        return launch_eval_nested3(p, prec, M, ws, partials, n_slices, slice_len, want_var, s);
    if (p->P.design_space == BMD_DESIGN_NESTED4)
        return launch_eval_nested4(p, prec, M, ws, partials, n_slices, slice_len, want_var, s);
    if (p->P.design_space == BMD_DESIGN_ALPHA4)
        return launch_eval_four(p, prec, M, ws, partials, n_slices, slice_len, want_var, s);
    return launch_eval_mode(p, prec, M, ws, partials, n_slices, slice_len, want_var ? kSquares : kSums, s);
}

hipError_t launch_eval_grid_dalpha(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                                   int n_slices, int64_t slice_len, hipStream_t s) {
    return launch_eval_mode(p, prec, M, ws, partials, n_slices, slice_len, kDAlpha, s);
}

hipError_t launch_eval_mode(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, int mode, hipStream_t s) {
    if (prec == BMD_FP64) {
        EvalArgs<double> a{p->P, p->d_r, p->d_z1, p->d_z2, static_cast<const double*>(p->tab[prec].A),
                           draws_fp64(p, M, ws), p->d_gl, static_cast<const double*>(p->tab[prec].glw),
                           slice_len, partials};
        return launch_typed<double, 24>(p, prec, a, n_slices, mode, s);
    }
    EvalArgs<float> a{p->P, p->d_r, p->d_z1, p->d_z2, static_cast<const float*>(p->tab[prec].A),
                      draws_fp32(p, M, ws), p->d_gl, static_cast<const float*>(p->tab[prec].glw),
                      slice_len, partials};
    return launch_typed<float, 12>(p, prec, a, n_slices, mode, s);
}

hipError_t launch_finalize(const bmd_problem* p, int64_t M, const double* partials, int n_slices, double* mean,
                           double* var, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((G + 255) / 256)), dim3(256), 0, s, G, M, n_slices,
                       partials, mean, var, var ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_finalize_dalpha(const bmd_problem* p, int64_t M, const double* partials, int n_slices, double* mean,
                                  double* dmean, hipStream_t s) {
    const int64_t G = p->P.G;
    hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((G + 255) / 256)), dim3(256), 0, s, G, M, n_slices,
                       partials, mean, dmean, 2);
    return hipGetLastError();
}

}  // namespace bmd
