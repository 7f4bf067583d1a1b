/*
 * bmd.h - C ABI of the MI355X (gfx950) hot path for optimal biomarker-cutoff
 * trial designs, after Lu, Zhou, Xing & Zhang, "The Optimal Design of Clinical
 * Trials with Potential Biomarker Effects, A Novel Computational Approach"
 * (arXiv 2005.10494).
 *
 * The method (Sec. 2): the expected power of a trial that tests the full
 * population and a biomarker-defined subgroup (Formula 4) is estimated by an
 * outer Monte Carlo average over prior draws of the effects (Formula 5), at
 * every point of a grid of candidate designs; the noisy surface is smoothed
 * (Sec. 2.3) and its maximiser is the design (Sec. 2.4).  Here a design is a
 * vector of biomarker cutoff quantiles q (one per biomarker), the subgroup is
 * S = {x_j > Phi^-1(q_j) for all j}, its population fraction r plays the role
 * of the paper's r_2 (Sec. 2.1), the two Z-statistics have null correlation
 * sqrt(r) (Formula 1, Appendix A.1), and Phi_Sigma is a bivariate normal CDF
 * evaluated in closed quadrature form rather than by the paper's inner
 * sampling layer (Formula 6).
 *
 * Conventions for every entry point:
 *   - Status codes are returned; nothing throws across the ABI.  On failure
 *     bmd_last_error() describes the cause (thread-local, valid until the next
 *     call from the same thread).  Outputs are then unspecified and the
 *     problem stays usable.
 *   - Arguments are validated on the host before any launch.
 *   - Pointers named d_* are device pointers (HBM of the current device),
 *     h_* are host pointers.  The caller owns every output buffer; the problem
 *     owns its device constants and workspace.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on the stream unless stated otherwise.
 *   - A problem is used from one host thread at a time; calls on one problem
 *     must not overlap on different streams.
 */
#ifndef BMD_H
#define BMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMD_ABI_VERSION 3
#define BMD_MAX_DIM 6
/* Size of the fixed device scratch of bmd_eval_grid_noalloc (128 MiB). */
#define BMD_NOALLOC_SCRATCH_BYTES (128ull << 20)

typedef struct bmd_problem bmd_problem;

typedef enum {
    BMD_OK = 0,
    BMD_EINVAL = -1,   /* invalid argument (NULL pointer, bad enum, non-finite) */
    BMD_ERANGE = -2,   /* argument outside the supported range                 */
    BMD_ENOMEM = -3,   /* device or host allocation failed                     */
    BMD_EDEVICE = -4,  /* a HIP call or kernel launch failed                   */
    BMD_ENOTSUP = -5,  /* combination not supported by this entry point        */
    BMD_ESTATE = -6    /* call not valid for this problem (e.g. grid vs points)*/
} bmd_status;

typedef enum {
    BMD_FP64 = 0,       /* integrand, sums and smoothing in FP64                */
    BMD_FP32_COMP = 1   /* FP32 integrand, FP64 per-design sums, FP32 smoothing */
} bmd_precision;

/* Critical values of the two tests (Formula 2 and its alternatives, Sec. 1). */
typedef enum {
    BMD_ALPHA_FWER_EQUAL = 0,  /* z1 = z2 = z*, 1 - Phi_2(z*, z*; sqrt r) = alpha0 */
    BMD_ALPHA_BONFERRONI = 1,  /* z1 = z2 = Phi^-1(1 - alpha0/2)                   */
    BMD_ALPHA_FIXED = 2,       /* z_i = Phi^-1(1 - alpha_fixed[i]); 0 = test off   */
    BMD_ALPHA_SPLIT = 3        /* z1 = Phi^-1(1 - alpha_fixed[0]), alpha_fixed[0] in
                                  (0, alpha0); z2 per design on the FWER boundary:
                                  1 - Phi_2(z1, z2; sqrt r) = alpha0               */
} bmd_alpha_rule;

/* Prior f(Delta) of Formula 4. */
typedef enum {
    /* Baseline effect b0 ~ N(mu_b0, sd_b0^2), extra effect b1 ~ N(mu_b1, sd_b1^2)
     * in responders R = {x_j > Phi^-1(tau_j) all j}, true cutoff quantiles
     * tau_j ~ U(tau_lo, tau_hi) iid.  Population-average effects:
     * Delta_1 = b0 + b1 P(R), Delta_2 = b0 + b1 P(R and S) / r. */
    BMD_EFFECT_STEP = 0,
    /* Formula 10 on the two nested populations: Delta ~ N(theta, Sigma_p) with
     * theta_i = -log(1 - (paper_a - paper_b r_i)), sigma_i = 1/sqrt(E r_i / 4),
     * corr(Delta_1, Delta_2) = sqrt(r), r_1 = 1, r_2 = r, E = paper_events. */
    BMD_EFFECT_PAPER_GAUSS = 1
} bmd_effect_model;

/* What a grid design is. */
typedef enum {
    /* d biomarker cutoff quantiles (the paper's r-design through cutoffs). */
    BMD_DESIGN_CUTOFFS = 0,
    /* The paper's own design variables for n = 2 nested populations (Sec. 2.2,
     * Sec. 3): the first test's level alpha_1 on the last axis, over [q_lo,
     * q_hi] inside (0, alpha0), with alpha_2 on the FWER boundary of Formula 2
     * (alpha_rule must be BMD_ALPHA_FWER_EQUAL, which then means FWER =
     * alpha0); with d = 2, axis 0 is the subgroup fraction r_2 over [r_lo,
     * r_hi]; with d = 1, r_2 = r_lo.  Formula 10 prior only
     * (BMD_EFFECT_PAPER_GAUSS); rho_b, gh_nodes and indicator_width are unused. */
    BMD_DESIGN_ALPHA = 1,
    /* n = 3 nested populations 1 > r_2 > r_3 (Sec. 2.2, Appendix A.1, Sec. 3
     * condition (c)): d = 2, axis 0 the first test's level alpha_1 and axis 1
     * the second's alpha_2, both over [q_lo, q_hi] inside (0, alpha0); the
     * third critical value lies on the FWER boundary 1 - Phi_3(z1, z2, z3) =
     * alpha0 of the null correlations sqrt(r_2), sqrt(r_3), sqrt(r_3/r_2).
     * r_lo holds r_2 and r_hi holds r_3, 0 < r_3 < r_2 <= 0.9, with partial
     * correlation sqrt(r_3 (1 - r_2) / (r_2 (1 - r_3))) <= 0.975.  A design
     * whose first two levels already spend alpha0 has no third level: its
     * estimate is NaN.  Formula 10 prior with three normals per draw
     * (BMD_EFFECT_PAPER_GAUSS); alpha_rule must be BMD_ALPHA_FWER_EQUAL.
     * Grid sweeps only (no batch, gradient or level-split calls). */
    BMD_DESIGN_ALPHA3 = 2,
    /* n = 4 nested populations 1 > r_2 > r_3 > r_4 (Sec. 2.2 with n = 4, the
     * designs with three candidate thresholds of Sec. 3): d = 3, axes alpha_1,
     * alpha_2, alpha_3 over [q_lo, q_hi] inside (0, alpha0); the fourth critical
     * value lies on the FWER boundary 1 - Phi_4(z1, .., z4) = alpha0 of the null
     * correlations sqrt(r_j / r_i).  r_lo holds r_2, r_hi holds r_3 and r_4 the
     * fourth fraction, 0 < r_4 < r_3 <= 0.95 r_2, r_2 <= 0.9, the partial
     * correlation of the third on the second population given the first at
     * most 0.975 (as for three populations) and that of the third and fourth
     * given the second, sqrt(r_4 (r_2 - r_3) / (r_3 (r_2 - r_4))), at most
     * 0.975.  Designs whose first three levels already spend alpha0 have no
     * fourth level and a NaN estimate.  Formula 10 prior with four normals per
     * draw; alpha_rule BMD_ALPHA_FWER_EQUAL; grid sweeps only. */
    BMD_DESIGN_ALPHA4 = 3,
    /* n = 3 nested populations cut from one biomarker by two cutoffs (Sec.
     * 2.2 with n = 3, in the cutoff design space): d = 2, axis 0 the first
     * cutoff quantile q_1 and axis 1 the second q_2, both over [q_lo, q_hi]
     * with 0.1 <= q_lo and q_hi < 1; the tests are the full population,
     * {x > Phi^-1(q_1)} (fraction r_2 = 1 - q_1) and {x > Phi^-1(q_2)}
     * (r_3 = 1 - q_2), with the null correlations sqrt(r_j / r_i) of Appendix
     * A.1.  Designs with q_1 >= q_2, or whose partial correlation
     * sqrt(r_3 (1 - r_2) / (r_2 (1 - r_3))) exceeds 0.975, do not exist: their
     * estimate is NaN.  Step prior with one true cutoff tau per draw
     * (BMD_EFFECT_STEP; the responders inside population i are a fraction
     * 1 - max(q_i, tau) of all patients); alpha_rule BMD_ALPHA_FWER_EQUAL (one
     * critical value z* with 1 - Phi_3(z*, z*, z*) = alpha0) or
     * BMD_ALPHA_BONFERRONI (Phi^-1(1 - alpha0 / 3)); indicator_width 0; at
     * most 16,776,960 designs (ERANGE); grid sweeps, smoothing (over the
     * designs that exist) and argmax only. */
    BMD_DESIGN_NESTED3 = 4,
    /* n = 4 nested populations cut from one biomarker by three cutoffs: d = 3,
     * axes q_1, q_2, q_3 over [q_lo, q_hi] with 0.1 <= q_lo and q_hi < 1; the
     * tests are the full population and {x > Phi^-1(q_i)} (r_{i+1} = 1 - q_i).
     * Designs outside q_1 < q_2 < q_3, with a partial correlation of the third
     * statistic on the second (given the first) or of the fourth and third
     * (given the second) above 0.975, or with r_3 > 0.95 r_2 do not exist (NaN).
     * Step prior with one true cutoff, as BMD_DESIGN_NESTED3; alpha_rule
     * BMD_ALPHA_FWER_EQUAL (one z* with 1 - Phi_4(z*, .., z*) = alpha0) or
     * BMD_ALPHA_BONFERRONI (Phi^-1(1 - alpha0 / 4)); indicator_width 0; at most
     * 16,776,960 designs; grid sweeps, smoothing (over the designs that exist)
     * and argmax only. */
    BMD_DESIGN_NESTED4 = 5
} bmd_design_space;

/* Problem descriptor (copied by bmd_create_problem). */
typedef struct {
    int32_t d;                 /* number of biomarkers / cutoff axes, 1..6          */
    int32_t m[BMD_MAX_DIM];    /* grid points per axis (>= 2 for j < d); all zero =>
                                  continuous-design problem (bmd_grad_design only)  */
    double q_lo, q_hi;         /* cutoff-quantile range, 0 < q_lo < q_hi < 1; grid
                                  q_j,i = q_lo + ((q_hi - q_lo) i) / (m_j - 1)       */
    double rho_b;              /* biomarker equicorrelation, 0 <= rho_b <= 0.5      */
    double info;               /* information units I (paper I_3), > 0              */
    double alpha0;             /* family-wise error rate, 0 < alpha0 < 0.5          */
    int32_t alpha_rule;        /* bmd_alpha_rule                                    */
    double alpha_fixed[2];     /* levels for BMD_ALPHA_FIXED, each in [0, 0.5)      */
    int32_t effect;            /* bmd_effect_model                                  */
    double mu_b0, sd_b0;       /* step prior, sd >= 0 (0 = point mass)              */
    double mu_b1, sd_b1;
    double tau_lo, tau_hi;     /* 0 < tau_lo <= tau_hi < 1                          */
    double paper_a, paper_b;   /* Formula 10 effect D0(r) = a - b r, D0 < 1         */
    double paper_events;       /* E in sigma_i = 1/sqrt(E r_i / 4), > 0             */
    double indicator_width;    /* 0: exact cutoff indicator; w > 0: logistic mix
                                  1/(1 + exp(-(q_j - tau_j)/w)) of the two cutoffs  */
    double bandwidth[BMD_MAX_DIM]; /* smoothing kernel sd per axis (quantile units) */
    int32_t gh_nodes;          /* Gauss-Hermite nodes for orthant probabilities:
                                  0 = chosen per precision from rho_b and d (a
                                  multiple of 4 up to 128), else a multiple of 4
                                  in [4, 128] (the kernels take nodes in fours)    */
    uint64_t seed;             /* Philox4x32-10 key (lo, hi words)                  */
    uint32_t scenario_id;      /* third Philox counter word                         */
    int32_t design_space;      /* bmd_design_space (0 = cutoffs)                    */
    double r_lo, r_hi;         /* BMD_DESIGN_ALPHA: subgroup-fraction axis (d = 2),
                                  0 < r_lo < r_hi <= 0.95, or r_2 = r_lo (d = 1);
                                  BMD_DESIGN_ALPHA3/4: r_lo = r_2, r_hi = r_3        */
    double r_4;                /* BMD_DESIGN_ALPHA4: the fourth fraction r_4        */
} bmd_problem_desc;

/* Version of this header the library was built from (BMD_ABI_VERSION). */
int32_t bmd_abi_version(void);

/* Last error message of the calling thread ("" if none). */
const char *bmd_last_error(void);

/* Create a problem (Sec. 2.1 inputs: r via the cutoffs, I_3, alpha0, prior).
 * Allocates the problem's device constants on the current device and launches
 * the per-design precompute (subgroup fraction r, critical values z1, z2) on
 * `stream`.  *out receives the handle; destroy it with bmd_destroy_problem.
 * ERANGE if some grid design has r > 0.95 (the bivariate quadrature supports
 * correlations sqrt(r) <= 0.975), or rho_b > 0.5.  Alpha design space: EINVAL
 * unless the prior is BMD_EFFECT_PAPER_GAUSS and the rule
 * BMD_ALPHA_FWER_EQUAL; ERANGE unless d is 1 or 2, the problem is a grid,
 * 0 < q_lo < q_hi < alpha0 and the r range is as stated above. */
bmd_status bmd_create_problem(const bmd_problem_desc *desc, bmd_problem **out, void *stream);

/* Release a problem and its device memory (synchronises the device).  NULL-safe. */
void bmd_destroy_problem(bmd_problem *p);

/* Number of grid designs G = prod m_j (0 for continuous-design problems). */
int64_t bmd_grid_size(const bmd_problem *p);

/* Gauss-Hermite nodes the problem uses for orthant probabilities at precision
 * prec (chosen at creation when desc.gh_nodes is 0); -1 for a bad argument. */
int32_t bmd_gh_nodes(const bmd_problem *p, int32_t prec);

/* Which kernel the designs x draws sweep of bmd_eval_grid uses for this
 * problem: BMD_SWEEP_DIRECT (one design per thread; one biomarker, the
 * logistic indicator, the paper's Formula 10 prior, or the environment
 * variable BMD_SWEEP=direct at creation) or BMD_SWEEP_MATRIX (16x16 design
 * tiles of the Sec. 2.2 sweep whose responder-overlap sums over the
 * Gauss-Hermite nodes run on the matrix cores as rank-K products).
 * Returns -1 for a NULL problem or a continuous-design one. */
enum { BMD_SWEEP_DIRECT = 0, BMD_SWEEP_MATRIX = 1 };
int32_t bmd_sweep_kind(const bmd_problem *p);

/* Monte Carlo estimate of the expected power (Formula 5) at every grid design
 * from draws k = 0 .. n_draws-1:
 *   d_mean[g] = (1/M) sum_k (1 - Phi_2(z1 - mu1_k, z2 - mu2_gk; sqrt r_g)),
 *   d_var[g]  = sample variance of the summands (may be NULL).
 * Both are FP64 arrays of length G in row-major design order (axis 0 slowest).
 * prec selects the integrand precision (sums are FP64 in both).
 * ESTATE for continuous-design problems; ERANGE if n_draws is 0 or > 2^40. */
bmd_status bmd_eval_grid(bmd_problem *p, uint64_t n_draws, int32_t prec,
                         double *d_mean, double *d_var, void *stream);

/* bmd_eval_grid for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results: the same kernels on the same draws, so d_mean
 * and d_var equal bmd_eval_grid's bit for bit.  The draws and per-slice
 * partial sums go to a fixed device array of BMD_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on until the process ends (its
 * address is looked up once per device by bmd_create_problem); this call
 * makes no allocation and no library call that allocates.  ERANGE when the
 * sweep needs more than the scratch: draws take about
 * M (d K + 12) * 4 bytes in FP32 (8 in FP64, K = bmd_gh_nodes) plus
 * 16 G bytes per draw slice (about ten slices at G = 64^3).  Every call on a
 * device shares that device's scratch: calls that overlap in time on one
 * device (different streams, or several host threads) race and give wrong
 * results; calls ordered on one stream are safe. */
bmd_status bmd_eval_grid_noalloc(bmd_problem *p, uint64_t n_draws, int32_t prec,
                                 double *d_mean, double *d_var, void *stream);

/* Nadaraya-Watson smoothing with the product Gaussian kernel
 * K(g,h) = prod_j exp(-((q_j(g) - q_j(h)) / b_j)^2 / 2), untruncated, applied
 * separably along each axis (the default smoother in place of the paper's
 * thin-plate spline, Sec. 2.3, which bmd_smooth_tps fits).  d_in and d_out are
 * FP64 arrays of length G and must not alias.  prec: FP64 uses FP64 matrix
 * cores; FP32_COMP uses FP32 matrix cores with FP32 accumulation.
 * BMD_DESIGN_ALPHA3/4 and BMD_DESIGN_NESTED3/4 grids sum over
 * the designs whose value is not NaN only (the designs that exist), which stay
 * NaN; other problems propagate NaN like any value. */
bmd_status bmd_smooth(bmd_problem *p, const double *d_in, double *d_out, int32_t prec,
                      void *stream);

/* Maximiser of a surface (the best grid point, Sec. 2.3): index g* of the
 * largest value, ties to the lowest index, NaN never wins.  Writes *h_index,
 * *h_value and, if h_cell is not NULL, the d grid indices of g*; a surface
 * with no value above -DBL_MAX other than NaN gives index 0 and value NaN.
 * Synchronises `stream` (returns the result on the host). */
bmd_status bmd_argmax(bmd_problem *p, const double *d_surface, int64_t *h_index,
                      double *h_value, int32_t *h_cell, void *stream);

/* Objective and its gradient at B continuous design points (the smoothness of
 * Appendix A.3 made explicit for the Newton step of Sec. 2.3):
 *   d_q       [B*d] FP64 cutoff quantiles, row-major, in [q_lo, q_hi] (to 1e-12);
 *             points outside get NaN outputs
 *   d_obj     [B]   FP64 Monte Carlo objective (as bmd_eval_grid's mean)
 *   d_grad_q  [B*d] d obj_b / d q_b,j (may be NULL)
 *   d_grad_mu [B*2] d obj_b / d (mu_b0, mu_b1) (may be NULL)
 * Draws are generated into the problem's workspace in passes of at most 4 GB
 * (environment variable BMD_GRAD_BUDGET, in bytes, overrides the limit) and
 * read by every point; results do not depend on the pass size.  Works on grid
 * and continuous problems; requires BMD_EFFECT_STEP and BMD_DESIGN_CUTOFFS
 * (ENOTSUP otherwise). */
bmd_status bmd_grad_design(bmd_problem *p, const double *d_q, int64_t B, uint64_t n_draws,
                           int32_t prec, double *d_obj, double *d_grad_q, double *d_grad_mu,
                           void *stream);

/* Optimal level split per design (Sec. 2.4's "optimal power" at each design,
 * for the n = 2 nested tests): for each first-test level h_alpha1[k] (host,
 * n_alpha values in (0, alpha0)) the second level of every design is put on
 * its FWER boundary (rule BMD_ALPHA_SPLIT), the grid is swept on draws
 * 0..n_draws-1 (generated once), and
 *   d_best   [G] FP64 receives the largest Monte Carlo estimate over the levels,
 *   d_best_k [G] int32 (may be NULL) the index k of the level that gave it
 *            (ties: the lowest k).
 * One sweep per level.  The problem's own critical values are restored before
 * the call returns (a design precompute is re-launched on `stream`).  ESTATE
 * for a continuous problem or the alpha design space; ERANGE for n_alpha
 * outside [1, 4096] or a level outside (0, alpha0). */
bmd_status bmd_eval_grid_levels(bmd_problem *p, uint64_t n_draws, int32_t prec, const double *h_alpha1,
                                int32_t n_alpha, double *d_best, int32_t *d_best_k, void *stream);

/* Optimal level split per design found by search (Sec. 2.4's "optimal power"
 * at each design, n = 2 nested tests): for every design, golden-section search
 * of the first level alpha_1 over [a_lo, a_hi] (0 < a_lo < a_hi < alpha0),
 * the second level on the design's FWER boundary, on the estimate of Formula 5
 * with draws 0..n_draws-1 (generated once, shared by every level).  The two
 * interior points split the bracket by the golden ratio; each of the n_iter
 * steps drops the part beyond the lower one (ties keep the left part) and
 * evaluates one new level, leaving a bracket (a_hi - a_lo) 0.618^(n_iter + 1)
 * wide; the two ends of the range are evaluated last, so a maximum at an end
 * is found exactly.  The call runs 4 + n_iter sweeps.
 *   d_best   [G] FP64 the largest estimate seen for each design
 *   d_alpha1 [G] FP64 the level that gave it (the first one seen on ties)
 * A local search: a design whose power has several maxima over the range may
 * end at a local one.  The problem's own critical values are restored before
 * the call returns.  ESTATE for a continuous problem or an alpha design space;
 * ERANGE for the range or n_iter outside [0, 200]. */
bmd_status bmd_optimize_levels(bmd_problem *p, uint64_t n_draws, int32_t prec, double a_lo, double a_hi,
                               int32_t n_iter, double *d_best, double *d_alpha1, void *stream);

/* The paper's two-layer sampling estimate of the expected power at every grid
 * design (Formula 7, the inner layer of Formula 6 in place of the exact
 * Phi_Sigma of Formula 5), for the Formula 10 prior:
 *   P(g) = 1 - (1/(N1 N2)) sum_{k<N1} sum_{l<N2} [x_j^(l) <= z_j - mu_j^(k) for all j],
 * outer draws k = 0..N1-1 (the draws of bmd_eval_grid), inner draws
 * l = 0..N2-1 of the null statistics with the nested correlations of
 * Appendix A.1 (Formula 1), shared by every outer draw: n standard normals per
 * l from the Philox stream whose fourth counter word has its top bit set
 * (counter (l lo, l hi, scenario, 0x80000000 | b)), chained as x_1 = e_1,
 * x_{i+1} = sqrt(r_{i+1}/r_i) x_i + sqrt(1 - r_{i+1}/r_i) e_{i+1}.  n = 2
 * (cutoff designs, BMD_DESIGN_ALPHA), 3 (BMD_DESIGN_ALPHA3) or 4
 * (BMD_DESIGN_ALPHA4).
 *   d_mean [G] FP64 the estimate (NaN for designs without a valid level split)
 *   d_var  [G] FP64 (may be NULL) an unbiased estimate of its variance: the
 *          comparisons are counted in blocks_outer x blocks_inner blocks
 *          (consecutive outer draws x consecutive inner draws) and the block
 *          means give the two-way crossed random-effects estimate
 *          (MS_A + MS_B - MS_E)/(A B) of sigma_1^2/N1 + sigma_2^2/N2 +
 *          sigma_12^2/(N1 N2) (the Hoeffding parts of the indicator), which
 *          may come out slightly negative; Appendix A.2's bound 1/(4 N1 N2)
 *          keeps only the last term.
 * prec: the comparisons in FP64, or in FP32 with both sides rounded (counts
 * may then differ from FP64's where a comparison falls within FP32 rounding).
 * ENOTSUP unless the effect is BMD_EFFECT_PAPER_GAUSS; ESTATE for continuous
 * problems; ERANGE unless blocks_outer, blocks_inner are in [2, 64],
 * n_outer is a multiple of blocks_outer (at most 2^31), n_inner a multiple of
 * 1024 and of 256 blocks_inner (at most 2^26), and a block holds fewer than
 * 2^32 comparisons. */
bmd_status bmd_eval_grid_two_layer(bmd_problem *p, uint64_t n_outer, uint64_t n_inner, int32_t prec,
                                   int32_t blocks_outer, int32_t blocks_inner, double *d_mean,
                                   double *d_var, void *stream);

/* Formula 5 estimate and its derivative in the first level alpha_1 at every
 * grid design, on draws 0..n_draws-1 (Appendix A.3 differentiates the power
 * under the integral; for the nested pair the chain rule runs through both
 * critical values):
 *   d_dmean[g] = (1/M) sum_k d(1 - Phi_2(z1 - mu1_k, z2 - mu2_gk; rho_g))/d alpha_1
 * with dz1/d alpha_1 = -1/phi(z1); under BMD_ALPHA_SPLIT the second level
 * stays on the design's FWER boundary, so z2 moves with z1 as
 * dz2/dz1 = -phi(z1) Phi((z2 - rho z1)/s) / (phi(z2) Phi((z1 - rho z2)/s)),
 * s = sqrt(1 - rho^2); under BMD_ALPHA_FIXED z2 stays (a second test switched
 * off leaves Appendix A.3's one-test form, mean of phi(z1 - mu1)/phi(z1)).
 *   d_mean  [G] FP64 the estimate (as bmd_eval_grid's mean up to FP32
 *           summation order)
 *   d_dmean [G] FP64 its alpha_1 derivative
 * Same sweep and draws as bmd_eval_grid, the derivative summed beside the
 * value.  ESTATE for a continuous problem or an alpha design space; ENOTSUP
 * for rules other than SPLIT and FIXED; ERANGE if alpha_fixed[0] is 0 or
 * n_draws is 0 or > 2^40. */
bmd_status bmd_eval_grid_dalpha(bmd_problem *p, uint64_t n_draws, int32_t prec, double *d_mean,
                                double *d_dmean, void *stream);

/* Optimal level split per design found from the derivative (Sec. 2.3's
 * derivative-driven search, Sec. 2.4's optimal power at each design, n = 2
 * nested tests): for every design, a root of d P / d alpha_1 (from the sweep
 * of bmd_eval_grid_dalpha) in [a_lo, a_hi] (0 < a_lo < a_hi < alpha0) by
 * bracketed false position with the Illinois halving, the second level on the
 * design's FWER boundary, draws 0..n_draws-1 generated once.  The ends are
 * probed first; a derivative <= 0 at a_lo or >= 0 at a_hi ends the design's
 * search at that end.  Each of the n_iter steps probes the secant root of the
 * bracket (its midpoint if that root is not strictly inside) and keeps the
 * end across the sign change; a zero derivative or a bracket below tol ends
 * the design's search (its best level is probed again until all designs
 * finish).  The call runs 2 + n_iter sweeps.
 *   d_best   [G] FP64 the largest estimate seen for each design
 *   d_alpha1 [G] FP64 the level that gave it (the first one seen on ties)
 * Near the root the derivative locates the level to the precision of the
 * derivative, where the golden-section search of bmd_optimize_levels is left
 * with the square root of the precision of the estimate.  A local search: a
 * design with several stationary points may end at one that is not the
 * largest.  The problem's own critical values and rule are restored before
 * the call returns.  ESTATE for a continuous problem or an alpha design space;
 * ERANGE for the range, n_iter outside [0, 200] or tol < 0. */
bmd_status bmd_optimize_levels_newton(bmd_problem *p, uint64_t n_draws, int32_t prec, double a_lo,
                                      double a_hi, int32_t n_iter, double tol, double *d_best,
                                      double *d_alpha1, void *stream);

/* Continuous refinement of a design (Sec. 2.3: the best grid point refined by
 * a local gradient method): projected gradient ascent inside the box
 * [q_lo, q_hi]^d on bmd_grad_design's objective (draws 0..n_draws-1 in every
 * evaluation, so the objective is one deterministic function of q; smooth for
 * indicator_width > 0).  Each iteration evaluates, in one bmd_grad_design call
 * of 8 points, the steps q + t_j g / max|g| with t_j = s 2^-j (j = 0..7),
 * clipped to the box, and accepts the first whose objective gains at least
 * 1e-4 g.(q_j - q) (Armijo); s starts at 0.05 and becomes twice the accepted
 * t_j, at most 0.1.  Stops when no trial gains, when the accepted move is below
 * tol in every coordinate, or after max_iter iterations.
 *   h_q0   [d] host, start point (clipped to the box)
 *   h_q    [d] host, result;  *h_obj its objective;  *h_iters accepted steps
 * Synchronises `stream`; allocates and frees a few hundred bytes of device
 * memory.  ENOTSUP unless the prior is BMD_EFFECT_STEP and the design space is
 * the cutoffs; ERANGE for max_iter outside [0, 10000] or tol < 0. */
bmd_status bmd_refine_design(bmd_problem *p, const double *h_q0, uint64_t n_draws, int32_t prec,
                             int32_t max_iter, double tol, double *h_q, double *h_obj, int32_t *h_iters,
                             void *stream);

/* Batched evaluation of n independent grid problems (the families of design
 * problems of Sec. 3) in one call: d_means[i] (FP64, [G_i], device) receives
 * problem i's mean surface for n_draws[i] draws, equal to bmd_eval_grid's up to
 * the order of the FP64 slice sums.  All problems must live on one device.
 * Problems are taken in order in groups whose draws fit half the free device
 * memory, at most 16 GB (environment variable BMD_BATCH_BUDGET, in bytes,
 * overrides the limit); each group is one captured HIP graph: draws of every
 * problem, one sweep launch per (biomarker count, kernel kind) over a list of
 * (problem, design tile, draw slice) items, finalize.  The call allocates and
 * frees its workspace.  h_wall_ms (may be NULL, [n], host) receives each
 * problem's completion time in ms after the first workgroup of the call
 * started, from the device clock.  Synchronises `stream`.  EINVAL for NULL
 * arguments or problems on different devices, ESTATE for continuous problems,
 * ERANGE for n outside [1, 65536] or n_draws outside [1, 2^40], ENOMEM if a
 * group's workspace cannot be allocated. */
bmd_status bmd_eval_batch(bmd_problem *const *ps, int32_t n, const uint64_t *n_draws,
                          int32_t prec, double *const *d_means, double *h_wall_ms,
                          void *stream);

/* The smoothed surface at a continuous design (the fitted surface of Sec. 2.3,
 * evaluated between grid points): the Nadaraya-Watson ratio of bmd_smooth,
 *   S(q) = sum_h K(q, q_h) f_h / sum_h K(q, q_h),
 * K = prod_j exp(-((q_j - q_{h,j}) / b_j)^2 / 2) over the grid designs h whose
 * value d_surface[h] (FP64, length G, typically bmd_eval_grid's mean) is not
 * NaN.  At a grid design it equals bmd_smooth's FP64 output there when no
 * value is NaN (bmd_smooth propagates NaN except on BMD_DESIGN_ALPHA3/4 and NESTED3/4 grids,
 * where it skips NaN designs as this call does).
 *   h_q     [d]    the design (any finite point; the grid's box is its range)
 *   h_value        S(q)
 *   h_grad  [d]    dS/dq_j (may be NULL)
 *   h_hess  [d*d]  d2S/dq_j dq_l, row-major (may be NULL)
 * FP64 sums over the grid in a fixed order; synchronises the stream.  ERANGE
 * when no design with a value carries weight at q. */
bmd_status bmd_smooth_at(bmd_problem *p, const double *d_surface, const double *h_q, double *h_value,
                         double *h_grad, double *h_hess, void *stream);

/* The best point of the smoothed surface refined by Newton's method (Sec. 2.3:
 * the best fitted point, then a local Newton search on the fitted surface):
 * from h_q0 (typically the grid design bmd_argmax returns for bmd_smooth's
 * output), steps -H^-1 grad S where the surface is locally concave (Cholesky
 * of -H), else along the gradient by a tenth of the smallest bandwidth; each
 * step projected into the grid's box and halved until it raises S by the
 * Armijo fraction 1e-4 of its first-order gain.  Stops after max_iter steps,
 * when a step moves every coordinate by at most tol, or when no halving is
 * accepted.  h_q [d] the final design, h_value S there, h_iters the steps
 * taken.  Synchronises the stream. */
bmd_status bmd_refine_smoothed(bmd_problem *p, const double *d_surface, const double *h_q0, int32_t max_iter,
                               double tol, double *h_q, double *h_value, int32_t *h_iters, void *stream);

/* Thin-plate spline smoothing of a grid surface (Sec. 2.3 fits a thin-plate
 * spline to the noisy estimates and maximises the fitted surface).  The
 * spline of order 2 in d = 1, 2, 3 dimensions on the grid's unit-box
 * coordinates u_j = (q_j - lo_j) / (hi_j - lo_j):
 *   f(u) = sum_i c_i phi(|u - u_i|) + a_0 + sum_j a_j u_j,
 *   phi(r) = r^3 (d = 1), r^2 log r (d = 2), -r (d = 3),
 * with centres at the designs whose value in d_in is not NaN and the
 * coefficients of the smoothing system (Phi + lambda I) c + P a = y,
 * P^T c = 0, P = [1, u] (lambda = 0 interpolates; larger values smooth, and
 * lambda -> infinity leaves the least-squares plane).
 *   d_in   [G] FP64 grid surface, NaN for designs without a value
 *   lambda      >= 0, finite
 *   d_out  [G] FP64 fitted surface at every design, NaN where d_in is NaN
 *               (must not alias d_in)
 *   h_n         number of designs fitted (may be NULL)
 * FP64 on the device: Householder elimination of the polynomial block, a
 * blocked Cholesky factorisation of the reduced (n - d - 1)^2 system, memory
 * about 8 n^2 bytes, allocated for the call.  The fit (centres and
 * coefficients) stays with the problem for bmd_tps_at and bmd_refine_tps until
 * the next call or bmd_destroy_problem.  ENOTSUP for d > 3; ERANGE when fewer
 * than d + 2 or more than 16,384 designs have a value, or when they do not
 * determine the spline (all on one hyperplane); the previous fit is kept on
 * any error.  Synchronises the stream. */
bmd_status bmd_smooth_tps(bmd_problem *p, const double *d_in, double lambda, double *d_out, int64_t *h_n,
                          void *stream);

/* Value, gradient and Hessian of the last bmd_smooth_tps fit at the design
 * h_q [d] (design coordinates; any finite point), as bmd_smooth_at: h_grad [d]
 * and h_hess [d*d] may be NULL.  At a centre its own term adds nothing to the
 * derivatives (r^2 log r's Hessian diverges there and -r has a kink).  FP64;
 * ESTATE without a fit; synchronises the stream. */
bmd_status bmd_tps_at(bmd_problem *p, const double *h_q, double *h_value, double *h_grad, double *h_hess,
                      void *stream);

/* Newton's method on the last bmd_smooth_tps fit from h_q0 (Sec. 2.3: the
 * best point of the fitted spline, refined on it), with the steps, safeguards
 * and stopping rules of bmd_refine_smoothed.  ESTATE without a fit. */
bmd_status bmd_refine_tps(bmd_problem *p, const double *h_q0, int32_t max_iter, double tol, double *h_q,
                          double *h_value, int32_t *h_iters, void *stream);

/* Launch settings of bmd_eval_batch.  Each sweep launch of a batch runs one
 * kind of problem (d biomarkers; kind 1 the matrix-core tile sweep of grids
 * with d >= 2 under the step prior and the exact indicator, kind 0 the
 * one-design-per-thread sweep); its settings are the tile body's draws per
 * LDS chunk, the rounds of resident workgroups its work list is sliced into
 * and the kernel's launch-bound variant.  mode 1 (the default): the first
 * batch that holds a kind on a device, in a precision, tunes its settings on
 * a calibration run of that batch's problems of the kind (draw counts scaled
 * to about 4e9 evaluations; chunk, then variant, then rounds, each candidate
 * timed on the device) and later batches reuse them; mode 0: fixed settings
 * (the one-problem sweep's chunk, 8 rounds, variant 0); mode 2: forget the
 * tuned settings (tune again on next use).  The settings change the draw
 * slicing, so means may differ from the fixed settings' in the last bits of
 * their FP64 sums.  Process-wide; not to be called while a batch runs. */
bmd_status bmd_batch_autotune(int32_t mode);

/* The tuned settings of launch kind (d, kind) in precision prec on the current
 * device: h_out[0] draws per LDS chunk (0 = the one-problem sweep's),
 * [1] rounds of resident workgroups, [2] launch-bound variant, [3] waves per
 * SIMD that variant keeps (0 = no bound), [4] the calibration launch's time in
 * microseconds.  ESTATE when no batch has tuned that kind yet. */
bmd_status bmd_batch_settings(int32_t prec, int32_t d, int32_t kind, int32_t *h_out /*[5]*/);

/* ---- profiling ------------------------------------------------------------ */

#define BMD_PROFILE_PHASES 5
/* Turn per-phase timing on (enable != 0) or off.  While on, bmd_eval_grid,
 * bmd_smooth and bmd_argmax record HIP events around their kernels on the
 * stream they launch on. */
bmd_status bmd_profile(bmd_problem *p, int32_t enable);

/* Device milliseconds of the latest profiled calls, h_ms[BMD_PROFILE_PHASES]:
 * [0] draw kernel, [1] grid sweep kernel, [2] finalize kernel, [3] smoothing
 * kernels, [4] argmax kernels (0 for phases not run since profiling began).
 * Synchronises on the recorded events. */
bmd_status bmd_profile_read(bmd_problem *p, double *h_ms);

/* ---- inspection (bit-exactness of sample generation and grid indexing) ---- */

#define BMD_DRAW_FIELDS 17
/* Draws k0 .. k0+n-1 as the kernels generate them.
 *   d_u      [n*8]  FP64 uniforms in consumption order (unused slots 0)
 *   d_fields [n*BMD_DRAW_FIELDS] FP64: b0, b1, P(R), e1, e2, tau[6], t[6]
 *            (step prior: b0, b1, P(R), tau, t = Phi^-1(tau); paper prior: e1, e2;
 *            BMD_DESIGN_ALPHA3/4 also the third normal e3 in the tau[0] slot,
 *            BMD_DESIGN_ALPHA4 the fourth e4 in the tau[1] slot) */
bmd_status bmd_draws(bmd_problem *p, uint64_t k0, uint64_t n, double *d_u, double *d_fields,
                     void *stream);

#define BMD_DESIGN_FIELDS 16
/* Design quantities for grid designs g0 .. g0+n-1:
 *   d_fields [n*BMD_DESIGN_FIELDS] FP64: q[6], c[6] = Phi^-1(q), r, sqrt(r), z1, z2
 *            (alpha design spaces: c[] is 0, except BMD_DESIGN_ALPHA3/4: c[0] = r_3
 *            and c[1] = z3, NaN when the design has no third level of three
 *            populations; BMD_DESIGN_ALPHA4 also c[2] = r_4 and c[3] = z4, NaN
 *            when the design has no fourth level; BMD_DESIGN_NESTED3: c[0] = r_3,
 *            c[1] = z3 (= z1 = z2), NaN for designs that do not exist;
 *            BMD_DESIGN_NESTED4 also c[2] = r_4 and c[3] = z4 (= z3)) */
bmd_status bmd_designs(bmd_problem *p, int64_t g0, int64_t n, double *d_fields, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BMD_H */
