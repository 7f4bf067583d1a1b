/*
 * Plain CPU oracle for the biomarker-cutoff design objective of
 * Lu, Zhou, Xing & Zhang, "The Optimal Design of Clinical Trials with
 * Potential Biomarker Effects, A Novel Computational Approach" (arXiv 2005.10494).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * Everything is FP64 and written for clarity, not speed: integrals are
 * evaluated by adaptive Gauss-Kronrod quadrature of their defining
 * one-dimensional forms, roots by bisection, sums by pairwise summation.
 *
 * Reading of the paper used throughout (the "signature" reading):
 *   - d correlated biomarkers X ~ N_d(0, (1-rho_b) I + rho_b 11'), one cutoff
 *     quantile q_j per biomarker; the subgroup S = {x_j > Phi^-1(q_j) for all j}
 *     has population fraction r (Sec. 2.1, the proportion r_i of a subset).
 *   - two nested tests, full population and S, so the null Z-correlation is
 *     sqrt(r) (Formula 1, Appendix A.1).
 *   - equal critical values chosen so the family-wise error equals alpha0
 *     (Formula 2), or Bonferroni, or fixed levels.
 *   - expected power over a prior on the effects (Formula 4), estimated by the
 *     outer Monte Carlo average of Formula 5 with an exact bivariate normal CDF.
 */
#ifndef BMD_ORACLE_H
#define BMD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_ALPHA_FWER_EQUAL = 0, OR_ALPHA_BONFERRONI = 1, OR_ALPHA_FIXED = 2, OR_ALPHA_SPLIT = 3 };
enum { OR_EFFECT_STEP = 0, OR_EFFECT_PAPER_GAUSS = 1 };
enum { OR_DESIGN_CUTOFFS = 0, OR_DESIGN_ALPHA = 1, OR_DESIGN_ALPHA3 = 2, OR_DESIGN_ALPHA4 = 3, OR_DESIGN_NESTED3 = 4,
       OR_DESIGN_NESTED4 = 5 };

typedef struct {
    int32_t d;              /* number of biomarkers (cutoff axes), 1..6          */
    int32_t m[6];           /* grid points per axis (grid problems only)         */
    double q_lo, q_hi;      /* cutoff-quantile range of the grid                 */
    double rho_b;           /* biomarker equicorrelation, 0 <= rho_b < 1         */
    double info;            /* information units I (paper: I_3)                 */
    double alpha0;          /* family-wise error rate                            */
    int32_t alpha_rule;     /* OR_ALPHA_*                                        */
    double alpha_fixed[2];  /* fixed levels (rule FIXED); 0 switches a test off;
                               rule SPLIT: alpha_fixed[0] is the first level and
                               the second is put on the FWER boundary (Formula 2) */
    int32_t effect;         /* OR_EFFECT_*                                       */
    double mu_b0, sd_b0;    /* step prior: baseline effect ~ N(mu_b0, sd_b0^2)   */
    double mu_b1, sd_b1;    /* step prior: responder effect ~ N(mu_b1, sd_b1^2)  */
    double tau_lo, tau_hi;  /* step prior: true cutoff quantile ~ U(lo, hi)      */
    double paper_a, paper_b, paper_events; /* Formula 10: D0(r)=a-b r, E events  */
    double width;           /* logistic indicator width (0 = exact indicator)    */
    double bandwidth[6];    /* Gaussian smoothing sd per axis, quantile units    */
    uint64_t seed;          /* Philox key                                        */
    uint32_t scenario;      /* third Philox counter word                         */
    /* Design space.  OR_DESIGN_CUTOFFS: the d cutoff quantiles above.
     * OR_DESIGN_ALPHA (Sec. 2.2-2.3, n = 2 nested populations, the paper's own
     * design variables): the last axis is the first test's level alpha_1 on
     * [q_lo, q_hi] inside (0, alpha0); alpha_2 follows from Formula 2 at FWER =
     * alpha0.  With d = 2, axis 0 is the subgroup fraction r_2 on [r_lo, r_hi];
     * with d = 1, r_2 = r_lo.  Paper prior (Formula 10) only.
     * OR_DESIGN_ALPHA3: n = 3 nested populations 1 > r_2 = r_lo > r_3 = r_hi
     * (Sec. 3's experiment); d = 2 axes alpha_1, alpha_2 on [q_lo, q_hi] and
     * alpha_3 on the FWER boundary (NaN designs where the first two levels
     * already spend alpha0).  Paper prior only.
     * OR_DESIGN_ALPHA4: n = 4 nested populations 1 > r_lo > r_hi > r_4 (the
     * three-threshold designs of Sec. 3); d = 3 axes alpha_1..alpha_3 on
     * [q_lo, q_hi] and alpha_4 on the FWER boundary (NaN designs where the first
     * three levels already spend alpha0).  Paper prior only.
     * OR_DESIGN_NESTED3: n = 3 nested populations cut from one biomarker by
     * two cutoffs, d = 2 axes q_1 < q_2 on [q_lo, q_hi]: the full population,
     * {x > Phi^-1(q_1)} (r_2 = 1 - q_1) and {x > Phi^-1(q_2)} (r_3 = 1 - q_2);
     * designs with q_1 >= q_2 or a partial correlation of the third on the
     * second population above 0.975 are NaN.  Step prior with one true cutoff
     * tau; alpha rule FWER_EQUAL (one z* for all three tests) or BONFERRONI.
     * OR_DESIGN_NESTED4: four nested populations from three cutoffs on one
     * biomarker, d = 3 axes q_1 < q_2 < q_3: the full population and
     * {x > Phi^-1(q_i)} (r_{i+1} = 1 - q_i); designs outside q_1 < q_2 < q_3,
     * with a partial correlation of the third on the second population (given
     * the first) or of the fourth and third (given the second) above 0.975, or
     * with r_3 > 0.95 r_2 are NaN.  Step prior, one z* (FWER_EQUAL) or
     * BONFERRONI (alpha0 / 4). */
    int32_t design_space;
    double r_lo, r_hi;
    double r_4;
} or_problem;

/* A design: cutoff quantiles and every quantity that depends on them only. */
typedef struct {
    double q[6], c[6];      /* quantiles and cutoffs c_j = Phi^-1(q_j)           */
    double r;               /* subgroup fraction                                 */
    double rho;             /* sqrt(r): null correlation of the two Z-statistics */
    double z1, z2;          /* critical values (may be +inf)                     */
    double r3, z3;          /* third population (OR_DESIGN_ALPHA3/4): r_3 and z3  */
    double r4, z4;          /* fourth population (OR_DESIGN_ALPHA4): r_4 and z4   */
} or_design;

/* One Monte Carlo draw of the effect parameters. */
typedef struct {
    double u[8];            /* the uniforms consumed by the draw                 */
    double b0, b1;          /* step prior effects                                */
    double tau[6], t[6];    /* true cutoff quantiles and cutoffs                 */
    double PR;              /* population fraction of responders                 */
    double e1, e2;          /* standard normals (paper Gaussian prior)           */
    double e3;              /* third normal (three populations)                  */
    double e4;              /* fourth normal (four populations)                  */
} or_draw;

/* ---- primitives -------------------------------------------------------- */
double or_Phi(double x);                 /* standard normal CDF (libm erfc)   */
double or_phi(double x);                 /* standard normal density           */
double or_Phiinv(double p);              /* root of Phi(x) = p                */
double or_quad(double (*f)(double, void *), void *ctx, double a, double b);
double or_bvn(double h, double k, double rho);     /* P(X<=h, Y<=k)          */
double or_bvn_density(double h, double k, double rho);
double or_tvn(double h1, double h2, double h3, double r12, double r13, double r23);   /* P(X_i <= h_i) */
double or_orthant(int d, const double *v, double rho_b);   /* P(X_j > v_j)    */
double or_zstar(double r, double alpha0);
double or_z2_fwer(double z1, double r, double alpha0);   /* second level on the FWER boundary */
double or_z3_fwer(double z1, double z2, double r2, double r3, double alpha0);   /* n = 3: third level */
double or_zstar3(double r2, double r3, double alpha0);   /* n = 3 at equal levels: 1 - Phi_3(z*,z*,z*) = alpha0 */
double or_qvn(const double *h, const double *R);   /* P(X_i <= h_i, i < 4), R 4 x 4 correlations */
double or_qvn_nested(const double *h, const double *r);   /* same, nested-population correlations of r[4] */
double or_zstar4(double r2, double r3, double r4, double alpha0);   /* 1 - Phi_4(z,z,z,z) = alpha0 */
double or_z4_fwer(double z1, double z2, double z3, double r2, double r3, double r4, double alpha0);   /* n = 4 */
double or_info_units(double alpha, double beta, double delta);
void   or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform52(uint32_t wa, uint32_t wb);

/* ---- model ------------------------------------------------------------- */
void   or_grid_point(const or_problem *p, int64_t g, double *q, int32_t *idx);
int64_t or_grid_size(const or_problem *p);
void   or_make_design(const or_problem *p, const double *q, or_design *out);
void   or_make_draw(const or_problem *p, uint64_t k, or_draw *out);
double or_overlap(const or_problem *p, const or_design *ds, const or_draw *dr);
double or_success(const or_problem *p, const or_design *ds, const or_draw *dr);

/* MC estimate (Formula 5) over draws k0..k0+M-1 at n design points q[n*d].
 * mean[i] = average success probability, var[i] = its sample variance. */
void   or_eval_points(const or_problem *p, int64_t n, const double *q,
                      uint64_t k0, uint64_t M, double *mean, double *var);
/* Same, at grid designs g_list[n]. */
void   or_eval_grid(const or_problem *p, int64_t n, const int64_t *g_list,
                    uint64_t k0, uint64_t M, double *mean, double *var);

/* ---- two-layer sampling estimator (Formulas 6 and 7) -------------------- */
/* Formula 7 at grid designs g_list[n] with outer draws 0..N1-1 and inner
 * draws 0..N2-1 (Formula 10 prior); mean[n], var[n] (may be NULL) the
 * unbiased block estimate of its variance from A x B blocks, blocks[n][A][B]
 * (may be NULL) the comparison counts. */
void   or_eval_grid_two_layer(const or_problem *p, int64_t n, const int64_t *g_list, uint64_t N1,
                              uint64_t N2, int A, int B, double *mean, double *var, uint32_t *blocks);

/* ---- derivative in the first level (Appendix A.3) ----------------------- */
/* d/d alpha_1 of one summand (cutoff designs, rule SPLIT or FIXED with
 * alpha_1 > 0): the chain rule through z1 and, under SPLIT, through the
 * second level on the FWER boundary. */
double or_dsuccess_dalpha1(const or_problem *p, const or_design *ds, const or_draw *dr);
/* Formula 5 estimate and its alpha_1 derivative at grid designs g_list[n]. */
void   or_eval_grid_dalpha(const or_problem *p, int64_t n, const int64_t *g_list,
                           uint64_t k0, uint64_t M, double *mean, double *dmean);

/* ---- smoothing and argmax ---------------------------------------------- */
void   or_smooth_direct(const or_problem *p, const double *in, double *out);
void   or_smooth_separable(const or_problem *p, const double *in, double *out);
void   or_smooth_masked(const or_problem *p, const double *in, double *out);
int64_t or_argmax(int64_t n, const double *v);
double or_smooth_at(const or_problem *p, const double *in, const double *q);   /* at a continuous design */

/* ---- gradient (forward mode, same draws) -------------------------------- */
void   or_grad_points(const or_problem *p, int64_t n, const double *q,
                      uint64_t k0, uint64_t M, double *obj,
                      double *grad_q, double *grad_mu);

/* ---- exact expectation (no Monte Carlo) -------------------------------- */
double or_exact_step(const or_problem *p, const double *q);    /* d <= 2 */
double or_exact_paper(const or_problem *p, const double *q);

/* ---- reporting ----------------------------------------------------------- */
int    or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
