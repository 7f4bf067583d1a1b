// Internal declarations shared by the HIP translation units of libbmd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "bmd.h"

namespace bmd {

constexpr int kMaxDim = BMD_MAX_DIM;
constexpr int kMaxGH = 128;          // Gauss-Hermite nodes, upper bound
constexpr int kPrecomputeGH = 128;   // nodes for the per-design subgroup fraction r
constexpr int kGLTable = 200;        // packed Gauss-Legendre rules n = 4..24
constexpr int kEvalBlock = 256;      // designs per workgroup in the eval kernels
constexpr int kSweepRounds = 8;      // rounds of resident workgroups a grid sweep is sliced into
// Staged draw bytes (node tables, drift quads, thresholds) of one matrix-core
// sweep slice, at most: the resident workgroups of a slice start at different
// times and each walks the whole slice, so one slice is the window of draws
// the L2 of an XCD (4 MB) has to hold while the tiles re-read it.
constexpr int64_t kSliceBytes = 2 << 20;
constexpr size_t kBatchBudget = size_t(96) << 30;   // draw bytes one batch group may hold
constexpr size_t kGradDrawBudget = size_t(4) << 30; // draw bytes one gradient pass may hold

// Problem constants passed by value to every kernel.
struct DevProblem {
    int d;
    int64_t G;                 // grid size (0 for continuous problems)
    int32_t m[kMaxDim];
    int64_t stride[kMaxDim];   // stride[j] = prod_{l>j} m_l
    int mmax;
    double q_lo, q_hi;
    int design_space;          // bmd_design_space
    double r_lo, r_hi;         // alpha design space: subgroup-fraction axis (d = 2) or r_2 = r_lo
    double r_4;                // four nested populations: r_4 (r_2 = r_lo, r_3 = r_hi)
    double rho_b, sr, sq;      // sqrt(rho_b), sqrt(1 - rho_b)
    double info, sqrtI;
    double alpha0;
    int alpha_rule;
    double zf1, zf2;           // critical values for the non-FWER rules (may be +inf)
    int zinf;                  // bit 0: z1 = +inf, bit 1: z2 = +inf (fixed rule only)
    int effect;
    double mu_b0, sd_b0, mu_b1, sd_b1, tau_lo, tau_hi;
    double paper_a, paper_b, paper_events;
    double th1, sg1;           // paper prior: theta_1 and sigma_1 of the full population
    double width;              // logistic indicator width (0 = exact)
    uint32_t key0, key1, scenario;
    int n_uniform;             // uniforms per draw
};

// Per-draw arrays, produced by the draw kernel and read by the eval kernels.
template <typename T>
struct DrawArrays {
    T* b0;      // [M]
    T* b1;      // [M]
    T* mu1;     // [M]  sqrt(I) * Delta_1
    T* PR;      // [M]  responder fraction
    T* tauT;    // [M]  tau_0 (one-biomarker closed form)
    T* e1;      // [M]  paper prior normals
    T* e2;      // [M]
    T* e3;      // [M]  third normal (three and four nested populations)
    T* e4;      // [M]  fourth normal (four nested populations)
    int32_t* thr;   // [M][d] first grid index whose cutoff quantile exceeds tau_j
    T* q4;      // [M][4] (b0, b1, mu1, 0): one 4-vector per draw for the matrix-core sweep
    double* tau;    // [d][M]
    T* B;       // [M][K][d] Phi((sqrt(rho) x_m - t_j)/sqrt(1-rho)), GH weight folded into j = 0
    int64_t M;
    int K;
};

// One problem's share of a batched draw launch.
template <typename T>
struct DrawJob {
    DevProblem P;
    const double* gh;       // FP64 Gauss-Hermite rule x[K], w[K]
    int K;
    int64_t first;          // first flattened draw index of this job
    DrawArrays<T> D;        // D.M = this job's draws
};

// The work list of one sweep launch of a batch (one workgroup per item).
struct BatchPhase {
    const void* sc;               // device array of per-scenario sweep records (type per precision)
    const int4* items;            // (record, tile, slice, 0), costliest first
    int n_items;
    int* left;                    // [n_scenarios] items not yet finished
    unsigned long long* t_start;  // earliest start stamp of the whole batch
    unsigned long long* t_done;   // [n_scenarios] completion stamp
};

// One problem's finalize record: mean over its draw slices.
struct BatchFinal {
    int64_t first;                // first flattened design index
    int64_t G, M;
    int n_slices;
    const double* partials;       // [n_slices][2][G]
    double* mean;                 // [G]
};

// Device constants owned by a problem, per integrand precision.
struct PrecTables {
    int K = 0;                  // Gauss-Hermite nodes
    double* gh = nullptr;       // [2K] nodes then weights (FP64)
    void* A = nullptr;          // [d][K][mmax] axis tables in T (weights folded into axis 0)
    void* glw = nullptr;        // packed GL weights in T
};

struct TpsFit;   // thin-plate spline fit of a problem's surface (kernels_tps.hip)

}  // namespace bmd

// Opaque handle of the C ABI.
struct bmd_problem {
    bmd_problem_desc desc;
    bmd::DevProblem P;
    bool grid = false;
    int device = 0;
    int n_cu = 0;                    // compute units of the device
    int sweep_bpc[2] = {0, 0};       // resident sweep workgroups per CU, per precision (0: not yet queried)
    bmd::PrecTables tab[2];          // [BMD_FP64], [BMD_FP32_COMP]
    double* d_gl = nullptr;          // packed GL table (x and w, FP64)
    double* d_ghp = nullptr;         // [2*kPrecomputeGH] GH rule for r
    double* d_r = nullptr;           // [G]
    double* d_z1 = nullptr;          // [G]
    double* d_z2 = nullptr;          // [G]
    double* d_z3 = nullptr;          // [G] third critical value (three and four nested populations)
    double* d_z4 = nullptr;          // [G] fourth critical value (four nested populations)
    int32_t* d_order = nullptr;      // [G] nested populations: designs with a last level first, then the rest
    double* d_W = nullptr;           // smoothing matrices, FP64, sum_j m_j^2
    float* d_Wf = nullptr;           // same in FP32
    int64_t w_off[bmd::kMaxDim] = {0, 0, 0, 0, 0, 0};
    void* d_ws = nullptr;            // workspace
    size_t ws_cap = 0;
    void* d_ws2 = nullptr;           // second workspace (smoothing ping-pong, argmax partials)
    size_t ws2_cap = 0;
    std::vector<double> gh_host[2];  // host copies of the eval GH rules
    bool force_direct = false;      // BMD_SWEEP=direct: use the direct sweep everywhere
    int64_t slice_bytes = bmd::kSliceBytes;   // staged draw bytes per matrix-core sweep slice (0: no limit)
    bool profiling = false;
    hipEvent_t ev[10] = {};          // begin/end pairs per profiled phase
    bool ev_used[5] = {false, false, false, false, false};
    bmd::TpsFit* tps = nullptr;      // the last bmd_smooth_tps fit (centres and coefficients on the device)
};

namespace bmd {

// Host quadrature rules (quad_nodes.cpp).
void gauss_hermite_prob(int n, double* x, double* w);   // int f(z) phi(z) dz
void gauss_legendre(int n, double* x, double* w);       // int_{-1}^{1} f(x) dx
void gl_table(double* out);                             // packed n = 4,6,8,10,12,16,20,24

// Launchers (return hipSuccess or the first HIP error).
hipError_t launch_design_precompute(const bmd_problem* p, hipStream_t s);
// Level splits (rule BMD_ALPHA_SPLIT for every design at first-level critical
// value z1) and the running maximum over levels.
hipError_t launch_levels_z(const bmd_problem* p, double z1, hipStream_t s);
hipError_t launch_levels_best(const bmd_problem* p, int k, const double* mean, double* best, int32_t* best_k,
                              hipStream_t s);
// Three nested populations (kernels_three.hip): critical values of every
// design, and the grid sweep (direct, one thread per design).
hipError_t launch_three_precompute(const bmd_problem* p, hipStream_t s);
// Two cutoffs on one biomarker (kernels_nested3.hip): critical values and
// the sweep's launch order of every design, and the grid sweep.
constexpr int64_t kNested3MaxTiles = 65535;   // sweep tiles of kEvalBlock designs (grid y dimension)
hipError_t launch_nested3_precompute(const bmd_problem* p, hipStream_t s);
// Thin-plate spline of a grid surface (kernels_tps.hip): fit on the designs
// with a value and, when d_out is given, the fitted surface at every design
// (NaN where d_in is NaN); the fit replaces p->tps on success.  code: kTpsOk,
// kTpsCount (n outside [d + 2, kTpsMaxPoints]), kTpsSingular (the designs do
// not determine the spline), kTpsNoMem, kTpsHip (err).  Synchronises s.
constexpr int64_t kTpsMaxPoints = 16384;
enum { kTpsOk = 0, kTpsCount = 1, kTpsSingular = 2, kTpsNoMem = 3, kTpsHip = 4 };
struct TpsFitResult {
    int code;
    int64_t n;
    hipError_t err;
};
TpsFitResult tps_fit_grid(bmd_problem* p, const double* d_in, double lam, double* d_out, hipStream_t s);
// Value, gradient and Hessian (rows j <= l) of the fit in unit-box coordinates
// u: h_out [1 + d + d (d + 1) / 2]; d_scratch holds 16 doubles.  Synchronises s.
hipError_t tps_at_unit(const bmd_problem* p, const double* u, double* d_scratch, double* h_out, hipStream_t s);
void tps_release(bmd_problem* p);
int tps_dims(const bmd_problem* p);   // 0 without a fit
int nested3_blocks_per_cu(int prec);
// Three cutoffs on one biomarker (kernels_nested4.hip): the same for
// (q_1, q_2, q_3) grids of four nested populations.
hipError_t launch_nested4_precompute(const bmd_problem* p, hipStream_t s);
int nested4_blocks_per_cu(int prec);
hipError_t launch_eval_nested4(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                               int n_slices, int64_t slice_len, bool want_var, hipStream_t s);
hipError_t launch_eval_nested3(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                               int n_slices, int64_t slice_len, bool want_var, hipStream_t s);
int three_blocks_per_cu(int prec);
hipError_t launch_eval_three(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                             int n_slices, int64_t slice_len, bool want_var, hipStream_t s);
// Four nested populations (kernels_four.hip): the same for (alpha_1, alpha_2,
// alpha_3) grids with the fourth level on the FWER boundary.
hipError_t launch_four_precompute(const bmd_problem* p, hipStream_t s);
int four_blocks_per_cu(int prec);
hipError_t launch_eval_four(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, bool want_var, hipStream_t s);
hipError_t launch_axis_tables(const bmd_problem* p, int prec, hipStream_t s);
hipError_t launch_draws(const bmd_problem* p, int prec, uint64_t k0, int64_t M, void* ws,
                        hipStream_t s);
size_t draw_workspace_bytes(const bmd_problem* p, int prec, int64_t M);
DrawArrays<double> draws_fp64(const bmd_problem* p, int64_t M, const void* ws);
DrawArrays<float> draws_fp32(const bmd_problem* p, int64_t M, const void* ws);
bool use_mfma_sweep(const bmd_problem* p);
// Workgroups along the design axis of the sweep launch, resident workgroups
// per compute unit for it, and its draw chunk (1 for the direct sweep).
int64_t sweep_tiles(const bmd_problem* p, int prec);
int sweep_blocks_per_cu(const bmd_problem* p, int prec);
int sweep_chunk(const bmd_problem* p, int prec);
// The two-layer sampling estimator (kernels_twolayer.hip): inner draws
// [n][N2] FP64 in `inner`, block counts [G][A][B] in `blocks`, outer draws
// k = 0..N1-1 already in `outer` (FP64); writes mean[G] and, if var is not
// NULL, the unbiased variance estimate var[G].
size_t two_layer_inner_bytes(int n, int64_t N2);
hipError_t launch_two_layer(const bmd_problem* p, int prec, int n, int64_t N1, int64_t N2, int A, int B,
                            const DrawArrays<double>& outer, double* inner, uint32_t* blocks, double* mean,
                            double* var, hipStream_t s);
// Bytes of one draw that a matrix-core sweep tile stages (0 for the direct sweep).
int64_t sweep_staged_bytes_per_draw(const bmd_problem* p, int prec);
struct MfmaGeom;
MfmaGeom sweep_geometry(const bmd_problem* p, int prec);
// want_var: also write the sums of squares (the second half of each slice).
hipError_t launch_eval_grid(const bmd_problem* p, int prec, int64_t M, const void* ws,
                            double* partials, int n_slices, int64_t slice_len, bool want_var, hipStream_t s);
hipError_t launch_finalize(const bmd_problem* p, int64_t M, const double* partials, int n_slices,
                           double* mean, double* var, hipStream_t s);
// Sweep and finalize with the summands' derivatives in alpha_1 (cutoff designs,
// rules BMD_ALPHA_SPLIT and BMD_ALPHA_FIXED): dmean = d mean / d alpha_1.
hipError_t launch_eval_mode(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                            int n_slices, int64_t slice_len, int mode, hipStream_t s);
hipError_t launch_eval_grid_dalpha(const bmd_problem* p, int prec, int64_t M, const void* ws, double* partials,
                                   int n_slices, int64_t slice_len, hipStream_t s);
hipError_t launch_finalize_dalpha(const bmd_problem* p, int64_t M, const double* partials, int n_slices,
                                  double* mean, double* dmean, hipStream_t s);
hipError_t launch_smooth(const bmd_problem* p, int prec, const double* in, double* out,
                         double* tmp, hipStream_t s);
hipError_t launch_argmax(const bmd_problem* p, const double* v, int64_t n, double* part_v,
                         int64_t* part_i, int n_part, hipStream_t s);
// The smoothed surface's numerator and denominator sums with their first and
// second derivatives at the continuous design q (axis ranges lo, hi): out gets
// 2 (1 + d + d (d + 1) / 2) FP64 values (kernels_post.hip); ws holds
// smooth_local_bytes().
size_t smooth_local_bytes();
hipError_t launch_smooth_local(const bmd_problem* p, const double* in, const double* q, const double* lo,
                               const double* hi, double* ws, double* out, hipStream_t s);
size_t grad_workspace_bytes(const bmd_problem* p, int prec, int64_t B, int n_slices, int64_t M, int64_t slice_len);
int grad_chunk(int prec, int d, int K);
int grad_blocks_per_cu(const bmd_problem* p, int prec);   // resident gradient workgroups per CU
int grad_lanes(int64_t B);   // threads per point of the gradient kernel (few points share their draws)
hipError_t launch_grad(const bmd_problem* p, int prec, const double* d_q, int64_t B, int64_t M, void* ws,
                       int n_slices, int64_t slice_len, double* obj, double* gq, double* gmu, hipStream_t s);
// Batched form.  Sweep records are filled on the host (batch_record_bytes, the
// record size and the stride the kernel indexes them with, each written by
// batch_fill_record for scenario `scenario` of the batch);
// one sweep launch per (precision, d, kernel kind), one workgroup per item.
DrawArrays<double> draws_fp64_at(const bmd_problem* p, int64_t M, void* ws);
DrawArrays<float> draws_fp32_at(const bmd_problem* p, int64_t M, void* ws);
hipError_t launch_draws_batch(int prec, const void* jobs, int n_jobs, int64_t total, hipStream_t s);
// chunk: draws per LDS chunk of the matrix-core items (0 = the one-problem
// sweep's); variant: launch-bound variant (batch_variants of them, see
// batch_variant_waves: waves per SIMD the bound keeps, 0 = none).
size_t batch_record_bytes(int prec);
void batch_fill_record(int prec, void* dst, const bmd_problem* p, void* draws_ws, int64_t M, int64_t slice_len,
                       double* partials, int scenario, int chunk);
size_t batch_phase_lds(const bmd_problem* p, int prec, int chunk);
int batch_variants(const bmd_problem* p, int prec);
int batch_variant_waves(const bmd_problem* p, int prec, int variant);
int batch_phase_blocks_per_cu(const bmd_problem* p, int prec, size_t lds, int variant);
hipError_t launch_batch_phase(const bmd_problem* p, int prec, const BatchPhase& ph, size_t lds, int variant,
                              hipStream_t s);
// Set left[first .. first+n) from items and clear their completion stamps;
// t_start (if non-NULL) restarts the clock.
hipError_t launch_batch_reset(int* left, unsigned long long* t_done, const int* items, int first, int n,
                              unsigned long long* t_start, hipStream_t s);
size_t draw_job_bytes(int prec);
void fill_draw_job(int prec, void* dst, const bmd_problem* p, void* draws_ws, int64_t M, int64_t first);
hipError_t launch_batch_finalize(const BatchFinal* jobs, int n_jobs, int64_t total, hipStream_t s);
hipError_t launch_inspect_draws(const bmd_problem* p, uint64_t k0, int64_t n, double* u,
                                double* fields, hipStream_t s);
hipError_t launch_inspect_designs(const bmd_problem* p, int64_t g0, int64_t n, double* fields,
                                  hipStream_t s);

}  // namespace bmd
