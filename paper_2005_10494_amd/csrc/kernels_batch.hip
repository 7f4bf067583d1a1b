// Many independent grid problems (Sec. 3's families of design problems) in
// one captured graph: a draw launch for every problem's prior draws, then one
// sweep launch per (precision, biomarker count, kernel kind) over a work list
// of (problem, design tile, draw slice) items, then a fixed-order finalize.
//
// Each item runs the same tile body as the one-problem sweep (sweep_body.hpp),
// so a batch computes exactly the one-problem sums per slice.
#include <algorithm>
#include <climits>
#include <cstring>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "sweep_body.hpp"

namespace bmd {

namespace {

// One problem of a batch, as the sweep bodies read it.  The host packs the
// records at stride sizeof(BatchRecord<T>) and the kernel indexes them the
// same way; 16-byte alignment keeps every record on a 16-byte boundary for
// the kernel's wide scalar loads.
template <typename T>
struct alignas(16) BatchRecord {
    EvalArgs<T> a;
    MfmaGeom geo;
    int scenario;      // index of the problem in the batch (left / t_done slot)
};
static_assert(sizeof(BatchRecord<float>) % 16 == 0 && sizeof(BatchRecord<double>) % 16 == 0,
              "record stride must equal its aligned size");

// One work item per workgroup: item blockIdx.x of the list, which is sorted
// costliest first, so the hardware dispatcher hands the long items out first
// and back-fills the short ones (the balance a persistent queue would give,
// without a work loop: with one, the compiler hoists the tile's per-thread
// addressing out of the loop and keeps it live across items, costing about 70
// VGPRs and half the occupancy).  The records come in as their own __restrict__
// argument, read-only for the launch, so their wave-uniform fields are fetched
// with scalar loads.  The last item of a problem stamps its completion time.
// Register bounds of the FP32 matrix-core items, chosen per launch by the
// batch autotuner from two variants: W = 0 keeps five wavefronts per SIMD up
// to three biomarkers and four beyond (at six, two node coefficients of the
// 10- and 12-node rules are reloaded from scratch; the other rules never touch
// them); W = 1 allows one wavefront fewer and so more registers.
template <int D, bool MF, int W>
constexpr int batch_waves() {
    return MF ? (D <= 3 ? 5 : 4) - W : 1;
}
template <typename T, int D, int NMAX, bool MF, int W>
__global__ __launch_bounds__(kEvalBlock, (sizeof(T) == 4 ? batch_waves<D, MF, W>() : 1)) void k_batch(BatchPhase ph, const BatchRecord<T>* __restrict__ recs) {
    extern __shared__ __align__(16) char lds[];
    if (threadIdx.x == 0) atomicMin(ph.t_start, static_cast<unsigned long long>(wall_clock64()));
    const int4 it = ph.items[blockIdx.x];
    const int rec = __builtin_amdgcn_readfirstlane(it.x);
    const int tile = __builtin_amdgcn_readfirstlane(it.y);
    const int slice = __builtin_amdgcn_readfirstlane(it.z);
    const BatchRecord<T>& R = recs[rec];
    if constexpr (MF)
        mfma_tile_body<T, D, NMAX, kSums>(R.a, R.geo, tile, slice, lds);
    else
        direct_body<T, D, NMAX, kSums>(R.a, tile, slice);
    __syncthreads();   // every thread's partial sums are written
    if (threadIdx.x == 0) {
        __threadfence();
        const int sc = R.scenario;
        if (atomicSub(&ph.left[sc], 1) == 1) ph.t_done[sc] = static_cast<unsigned long long>(wall_clock64());
    }
}

__global__ void k_batch_reset(int* left, unsigned long long* t_done, const int* items, int first, int n,
                              unsigned long long* t_start) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        left[first + t] = items[t];
        t_done[first + t] = 0;
    }
    if (t == 0 && t_start) *t_start = ULLONG_MAX;
}

// mean[g] = (sum over slices, in slice order) / M for every design of every job.
__global__ void k_batch_finalize(const BatchFinal* __restrict__ jobs, int n_jobs, int64_t total) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int lo = 0, hi = n_jobs - 1;   // last job with first <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first <= t) lo = mid; else hi = mid - 1;
    }
    const BatchFinal& J = jobs[lo];
    const int64_t g = t - J.first;
    double s = 0.0;
    for (int sl = 0; sl < J.n_slices; ++sl) s += J.partials[static_cast<int64_t>(sl) * 2 * J.G + g];
    J.mean[g] = s / static_cast<double>(J.M);
}

template <typename T, int NMAX, bool MF, int W>
const void* batch_kernel(int d) {
    switch (d) {
        case 1: return MF ? nullptr : reinterpret_cast<const void*>(k_batch<T, 1, NMAX, false, 0>);
        case 2: return reinterpret_cast<const void*>(k_batch<T, 2, NMAX, MF, W>);
        case 3: return reinterpret_cast<const void*>(k_batch<T, 3, NMAX, MF, W>);
        case 4: return reinterpret_cast<const void*>(k_batch<T, 4, NMAX, MF, W>);
        case 5: return reinterpret_cast<const void*>(k_batch<T, 5, NMAX, MF, W>);
        default: return reinterpret_cast<const void*>(k_batch<T, 6, NMAX, MF, W>);
    }
}

// Launch-bound variants: two for the FP32 matrix-core items, one otherwise.
const void* phase_kernel(const bmd_problem* p, int prec, int variant) {
    const bool mf = use_mfma_sweep(p);
    if (prec == BMD_FP64) return mf ? batch_kernel<double, 24, true, 0>(p->P.d) : batch_kernel<double, 24, false, 0>(p->P.d);
    if (!mf) return batch_kernel<float, 12, false, 0>(p->P.d);
    return variant == 1 ? batch_kernel<float, 12, true, 1>(p->P.d) : batch_kernel<float, 12, true, 0>(p->P.d);
}

}  // namespace

size_t batch_record_bytes(int prec) {
    return prec == BMD_FP64 ? sizeof(BatchRecord<double>) : sizeof(BatchRecord<float>);
}

int batch_variants(const bmd_problem* p, int prec) { return prec == BMD_FP32_COMP && use_mfma_sweep(p) ? 2 : 1; }

int batch_variant_waves(const bmd_problem* p, int prec, int variant) {
    if (prec != BMD_FP32_COMP || !use_mfma_sweep(p)) return 0;   // no launch bound
    return (p->P.d <= 3 ? 5 : 4) - variant;
}

void batch_fill_record(int prec, void* dst, const bmd_problem* p, void* draws_ws, int64_t M, int64_t slice_len,
                       double* partials, int scenario, int chunk) {
    MfmaGeom geo = use_mfma_sweep(p) ? sweep_geometry(p, prec) : MfmaGeom{};
    if (use_mfma_sweep(p) && chunk > 0) geo.chunk = chunk;
    if (prec == BMD_FP64) {
        BatchRecord<double> r{EvalArgs<double>{p->P, p->d_r, p->d_z1, p->d_z2,
                                               static_cast<const double*>(p->tab[prec].A), draws_fp64_at(p, M, draws_ws),
                                               p->d_gl, static_cast<const double*>(p->tab[prec].glw), slice_len, partials},
                              geo, scenario};
        std::memcpy(dst, &r, sizeof r);
    } else {
        BatchRecord<float> r{EvalArgs<float>{p->P, p->d_r, p->d_z1, p->d_z2,
                                             static_cast<const float*>(p->tab[prec].A), draws_fp32_at(p, M, draws_ws),
                                             p->d_gl, static_cast<const float*>(p->tab[prec].glw), slice_len, partials},
                             geo, scenario};
        std::memcpy(dst, &r, sizeof r);
    }
}

size_t batch_phase_lds(const bmd_problem* p, int prec, int chunk) {
    if (!use_mfma_sweep(p)) return 0;
    const int ch = chunk > 0 ? chunk : sweep_geometry(p, prec).chunk;
    return prec == BMD_FP64 ? mfma_lds_bytes<double>(ch, p->P.d, p->tab[prec].K)
                            : mfma_lds_bytes<float>(ch, p->P.d, p->tab[prec].K);
}

int batch_phase_blocks_per_cu(const bmd_problem* p, int prec, size_t lds, int variant) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, phase_kernel(p, prec, variant), kEvalBlock, lds) !=
            hipSuccess ||
        nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t launch_batch_phase(const bmd_problem* p, int prec, const BatchPhase& ph, size_t lds, int variant,
                              hipStream_t s) {
    if (ph.n_items <= 0) return hipSuccess;
    const void* recs = ph.sc;
    void* args[] = {const_cast<BatchPhase*>(&ph), const_cast<void**>(&recs)};
    return hipLaunchKernel(phase_kernel(p, prec, variant), dim3(static_cast<unsigned>(ph.n_items)), dim3(kEvalBlock),
                           args, lds, s);
}

hipError_t launch_batch_reset(int* left, unsigned long long* t_done, const int* items, int first, int n,
                              unsigned long long* t_start, hipStream_t s) {
    const int m = std::max(n, 1);
    hipLaunchKernelGGL(k_batch_reset, dim3((m + 255) / 256), dim3(256), 0, s, left, t_done, items, first, n, t_start);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchFinal* jobs, int n_jobs, int64_t total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_finalize, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, jobs,
                       n_jobs, total);
    return hipGetLastError();
}

}  // namespace bmd
