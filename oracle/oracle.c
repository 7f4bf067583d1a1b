/*
 * Plain CPU oracle for the biomarker-cutoff design objective (arXiv 2005.10494).
 *
 * TEST INFRASTRUCTURE ONLY: see oracle.h.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this library.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared oracle.c -lm
 * (-ffp-contract=off keeps every product and sum separately rounded, which the
 * bit-exact grid coordinates and uniforms rely on).
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ======================================================================== */
/* Standard normal distribution                                             */
/* ======================================================================== */

/* Phi(x) = P(N(0,1) <= x), through the C library's complementary error
 * function, which keeps relative accuracy in the lower tail. */
double or_Phi(double x)
{
    if (x == INFINITY) return 1.0;
    if (x == -INFINITY) return 0.0;
    return 0.5 * erfc(-x / sqrt(2.0));
}

double or_phi(double x)
{
    return exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
}

/* Phi^-1(p): the root of Phi(x) = p.
 * Central region p in [1/4, 3/4]: Newton on erf(x/sqrt 2)/2 = p - 1/2, where
 * p - 1/2 is exact, so x keeps relative accuracy near 0.
 * Lower region: a rough start (Abramowitz & Stegun 26.2.23), then Newton on
 * log Phi(x) = log p, which converges in a few steps down to p ~ 1e-308.
 * Upper region: Phi^-1(p) = -Phi^-1(1-p); 1-p is exact for p in [1/2, 1). */
double or_Phiinv(double p)
{
    if (isnan(p) || p < 0.0 || p > 1.0) return NAN;
    if (p == 0.0) return -INFINITY;
    if (p == 1.0) return INFINITY;
    if (p == 0.5) return 0.0;
    if (p >= 0.25 && p <= 0.75) {
        double a = p - 0.5;
        double x = a * sqrt(2.0 * M_PI);
        for (int it = 0; it < 100; ++it) {
            double step = (0.5 * erf(x / sqrt(2.0)) - a) / or_phi(x);
            x -= step;
            if (step == 0.0 || fabs(step) <= 1e-17 * fabs(x)) break;
        }
        return x;
    }
    if (p > 0.5) return -or_Phiinv(1.0 - p);
    double t = sqrt(-2.0 * log(p));
    double x = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                         (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    for (int it = 0; it < 100; ++it) {
        double F = or_Phi(x);
        double step = log1p((F - p) / p) * F / or_phi(x);
        x -= step;
        if (step == 0.0 || fabs(step) <= 1e-17 * fabs(x)) break;
    }
    return x;
}

/* ======================================================================== */
/* Adaptive Gauss-Kronrod (7-point Gauss, 15-point Kronrod) quadrature      */
/* ======================================================================== */

static const double gk_x[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double gk_wk[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double gk_wg[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef double (*or_fn)(double, void *);

static double gk15(or_fn f, void *ctx, double a, double b, double *err)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c, ctx);
    double rk = fc * gk_wk[7], rg = fc * gk_wg[3];
    for (int j = 0; j < 7; ++j) {
        double dx = h * gk_x[j];
        double s = f(c - dx, ctx) + f(c + dx, ctx);
        rk += gk_wk[j] * s;
        if (j & 1) rg += gk_wg[j / 2] * s;
    }
    *err = fabs((rk - rg) * h);
    return rk * h;
}

static double gk_adapt(or_fn f, void *ctx, double a, double b, double tol, int depth)
{
    double err, r = gk15(f, ctx, a, b, &err);
    if (err <= tol || err <= 1e-15 * fabs(r) || depth >= 40) return r;
    double m = 0.5 * (a + b);
    return gk_adapt(f, ctx, a, m, 0.5 * tol, depth + 1) +
           gk_adapt(f, ctx, m, b, 0.5 * tol, depth + 1);
}

/* Integral of f over [a, b]: eight equal panels, each refined by bisection
 * until the Gauss/Kronrod difference is below 1e-17 absolute or 1e-15
 * relative. */
double or_quad(or_fn f, void *ctx, double a, double b)
{
    const int n0 = 8;
    double s = 0.0;
    for (int i = 0; i < n0; ++i) {
        double lo = a + (b - a) * i / n0;
        double hi = (i == n0 - 1) ? b : a + (b - a) * (i + 1) / n0;
        s += gk_adapt(f, ctx, lo, hi, 1e-17, 0);
    }
    return s;
}

/* ======================================================================== */
/* Bivariate normal CDF                                                     */
/* ======================================================================== */

typedef struct { double k, rho, sig; } bvn_ctx;

static double bvn_integrand(double x, void *v)
{
    const bvn_ctx *c = (const bvn_ctx *)v;
    return or_phi(x) * or_Phi((c->k - c->rho * x) / c->sig);
}

/* Phi_2(h, k; rho) = P(X <= h, Y <= k) for a standard bivariate normal with
 * correlation rho, from its definition by conditioning on X:
 *   Phi_2 = int_{-inf}^{h} phi(x) Phi((k - rho x) / sqrt(1 - rho^2)) dx.
 * This is the CDF Phi_Sigma of Formula 1 for n = 2. */
double or_bvn(double h, double k, double rho)
{
    if (isnan(h) || isnan(k) || isnan(rho)) return NAN;
    if (h == -INFINITY || k == -INFINITY) return 0.0;
    if (h == INFINITY) return or_Phi(k);
    if (k == INFINITY) return or_Phi(h);
    if (rho >= 1.0) return or_Phi(fmin(h, k));
    if (rho <= -1.0) {
        double v = or_Phi(h) - or_Phi(-k);
        return v > 0.0 ? v : 0.0;
    }
    if (k < h) { double t = h; h = k; k = t; }
    bvn_ctx c = {k, rho, sqrt((1.0 - rho) * (1.0 + rho))};
    double lo = fmin(-12.0, h - 10.0);
    return or_quad(bvn_integrand, &c, lo, h);
}

/* Standard trivariate normal CDF P(X1 <= h1, X2 <= h2, X3 <= h3) with
 * correlations r12, r13, r23, from its definition by conditioning on X1:
 *   int_{-inf}^{h1} phi(x) Phi_2((h2 - r12 x)/s12, (h3 - r13 x)/s13; r23.1) dx,
 * s1j = sqrt(1 - r1j^2), r23.1 = (r23 - r12 r13) / (s12 s13) (the partial
 * correlation).  Phi_Sigma of Formula 1 for n = 3. */
typedef struct { double h2, h3, r12, r13, s12, s13, r231; } tvn_ctx;

static double tvn_integrand(double x, void *ctx)
{
    const tvn_ctx *c = (const tvn_ctx *)ctx;
    return or_phi(x) * or_bvn((c->h2 - c->r12 * x) / c->s12, (c->h3 - c->r13 * x) / c->s13, c->r231);
}

double or_tvn(double h1, double h2, double h3, double r12, double r13, double r23)
{
    if (isnan(h1) || isnan(h2) || isnan(h3)) return NAN;
    if (h1 == -INFINITY || h2 == -INFINITY || h3 == -INFINITY) return 0.0;
    if (h1 == INFINITY) return or_bvn(h2, h3, r23);
    if (h2 == INFINITY) return or_bvn(h1, h3, r13);
    if (h3 == INFINITY) return or_bvn(h1, h2, r12);
    tvn_ctx c = {h2, h3, r12, r13, sqrt((1.0 - r12) * (1.0 + r12)), sqrt((1.0 - r13) * (1.0 + r13)), 0.0};
    c.r231 = (r23 - r12 * r13) / (c.s12 * c.s13);
    return or_quad(tvn_integrand, &c, fmin(-12.0, h1 - 10.0), h1);
}

/* Standard four-variate normal CDF P(X_i <= h_i, i = 1..4) with correlation
 * matrix R (row-major 4 x 4, unit diagonal), from its definition by
 * conditioning on X1: given X1 = x the other three are normal with means
 * R_1j x, sds s_1j = sqrt(1 - R_1j^2) and the partial correlations
 * R_jk.1 = (R_jk - R_1j R_1k) / (s_1j s_1k), so
 *   int_{-inf}^{h1} phi(x) Phi_3((h_j - R_1j x)/s_1j; R_.1) dx.
 * Phi_Sigma of Formula 1 for n = 4. */
typedef struct { double h[3], r1[3], s1[3], p23, p24, p34; } qvn_ctx;

static double qvn_integrand(double x, void *ctx)
{
    const qvn_ctx *c = (const qvn_ctx *)ctx;
    return or_phi(x) * or_tvn((c->h[0] - c->r1[0] * x) / c->s1[0], (c->h[1] - c->r1[1] * x) / c->s1[1],
                              (c->h[2] - c->r1[2] * x) / c->s1[2], c->p23, c->p24, c->p34);
}

double or_qvn(const double *h, const double *R)
{
    for (int i = 0; i < 4; ++i) {
        if (isnan(h[i])) return NAN;
        if (h[i] == -INFINITY) return 0.0;
    }
    if (h[0] == INFINITY) return or_tvn(h[1], h[2], h[3], R[1 * 4 + 2], R[1 * 4 + 3], R[2 * 4 + 3]);
    qvn_ctx c;
    for (int j = 0; j < 3; ++j) {
        c.h[j] = h[j + 1];
        c.r1[j] = R[j + 1];
        c.s1[j] = sqrt((1.0 - c.r1[j]) * (1.0 + c.r1[j]));
    }
    c.p23 = (R[1 * 4 + 2] - c.r1[0] * c.r1[1]) / (c.s1[0] * c.s1[1]);
    c.p24 = (R[1 * 4 + 3] - c.r1[0] * c.r1[2]) / (c.s1[0] * c.s1[2]);
    c.p34 = (R[2 * 4 + 3] - c.r1[1] * c.r1[2]) / (c.s1[1] * c.s1[2]);
    return or_quad(qvn_integrand, &c, fmin(-12.0, h[0] - 10.0), h[0]);
}

/* Density of the standard bivariate normal (the integrand of Plackett's
 * identity d Phi_2 / d rho = phi_2). */
double or_bvn_density(double h, double k, double rho)
{
    double om = (1.0 - rho) * (1.0 + rho);
    return exp(-(h * h - 2.0 * rho * h * k + k * k) / (2.0 * om)) / (2.0 * M_PI * sqrt(om));
}

/* ======================================================================== */
/* Equicorrelated orthant probabilities                                     */
/* ======================================================================== */
/*
 * With X_j = sqrt(rho_b) Z + sqrt(1 - rho_b) E_j (Z, E_j iid N(0,1)), the
 * event {X_j > v_j} given Z = z has probability Phi((sqrt(rho_b) z - v_j) /
 * sqrt(1 - rho_b)), independently across j.  Integrating over z gives every
 * orthant-type probability used below as a one-dimensional integral.
 *
 * Each axis contributes one factor.  Factor kinds:
 *   FK_CUT   Phi(a_j),                        a_j = (sqrt(rho) z - c_j)/sqrt(1-rho)
 *   FK_MIX   s_j Phi(a_j) + (1 - s_j) Phi(b_j), b_j likewise with t_j
 *   FK_DENS  phi(a_j)                         (derivative of FK_CUT in -c_j)
 *   FK_DMIX  Phi(a_j) - Phi(b_j)              (derivative of FK_MIX in s_j)
 */
enum { FK_CUT = 0, FK_MIX = 1, FK_DENS = 2, FK_DMIX = 3 };

typedef struct {
    int d;
    double c[6], t[6], s[6];
    int kind[6];
    double sr, sq;
} orth_ctx;

static double orth_integrand(double z, void *v)
{
    const orth_ctx *o = (const orth_ctx *)v;
    double prod = or_phi(z);
    for (int j = 0; j < o->d; ++j) {
        double a = (o->sr * z - o->c[j]) / o->sq;
        double f;
        switch (o->kind[j]) {
        case FK_CUT: f = or_Phi(a); break;
        case FK_DENS: f = or_phi(a); break;
        case FK_MIX: {
            double b = (o->sr * z - o->t[j]) / o->sq;
            f = o->s[j] * or_Phi(a) + (1.0 - o->s[j]) * or_Phi(b);
            break;
        }
        default: {
            double b = (o->sr * z - o->t[j]) / o->sq;
            f = or_Phi(a) - or_Phi(b);
            break;
        }
        }
        prod *= f;
    }
    return prod;
}

static double orth_integral(orth_ctx *o, double rho_b)
{
    o->sr = sqrt(rho_b);
    o->sq = sqrt(1.0 - rho_b);
    return or_quad(orth_integrand, o, -12.0, 12.0);
}

/* P(X_j > v_j for all j), X ~ N_d(0, (1-rho_b) I + rho_b 11'). */
double or_orthant(int d, const double *v, double rho_b)
{
    orth_ctx o;
    memset(&o, 0, sizeof o);
    o.d = d;
    for (int j = 0; j < d; ++j) { o.c[j] = v[j]; o.kind[j] = FK_CUT; }
    return orth_integral(&o, rho_b);
}

/* ======================================================================== */
/* Critical values                                                          */
/* ======================================================================== */

/* Family-wise error of two one-sided tests at a common critical value z with
 * null correlation rho (Formula 2 for n = 2):
 *   1 - Phi_2(z, z; rho) = 2 Phi(-z) - Phi_2(-z, -z; rho),
 * written in the second form so both terms keep relative accuracy. */
static double fwer_equal(double z, double rho)
{
    return 2.0 * or_Phi(-z) - or_bvn(-z, -z, rho);
}

/* Common critical value z* with FWER(z*) = alpha0, by bisection between the
 * one-test value (rho = 1) and the Bonferroni value (which is conservative). */
double or_zstar(double r, double alpha0)
{
    double rho = sqrt(r);
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(0.5 * alpha0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (fwer_equal(mid, rho) > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* One critical value z* for three nested tests at equal levels (Formula 2 with
 * n = 3 and alpha_1 = alpha_2 = alpha_3): 1 - Phi_3(z*, z*, z*) = alpha0 for the
 * null correlations sqrt(r2), sqrt(r3), sqrt(r3 / r2) of Appendix A.1, by
 * bisection between one test at level alpha0 and the Bonferroni value. */
double or_zstar3(double r2, double r3, double alpha0)
{
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(alpha0 / 3.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fwer = 1.0 - or_tvn(mid, mid, mid, sqrt(r2), sqrt(r3), sqrt(r3 / r2));
        if (fwer > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Second critical value z2 with FWER(z1, z2) = P(Z1 > z1 or Z2 > z2) =
 * Phi(-z1) + Phi(-z2) - Phi_2(-z1, -z2; sqrt r) = alpha0 (Formula 2 for n = 2
 * with the first level alpha_1 = Phi(-z1) given), by bisection: the FWER falls
 * in z2, is at least alpha0 where the second test alone has level alpha0 and
 * at most alpha0 where it has level alpha0 - alpha_1 (the union bound).
 * +inf when alpha_1 >= alpha0. */
double or_z2_fwer(double z1, double r, double alpha0)
{
    double a1 = or_Phi(-z1);
    if (!(a1 < alpha0)) return INFINITY;
    double rho = sqrt(r);
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(alpha0 - a1);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fwer = a1 + or_Phi(-mid) - or_bvn(-z1, -mid, rho);
        if (fwer > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* n = 3 nested populations 1 > r2 > r3 (null correlations sqrt(r2), sqrt(r3),
 * sqrt(r3/r2), Appendix A.1): the third critical value with FWER =
 * 1 - Phi_3(z1, z2, z3) = alpha0 given the first two, by bisection between the
 * third test alone at level alpha0 and the union bound (the first two tests
 * spend a12 = 1 - Phi_2(z1, z2; sqrt r2)).  NaN when a12 >= alpha0. */
double or_z3_fwer(double z1, double z2, double r2, double r3, double alpha0)
{
    double a12 = 1.0 - or_bvn(z1, z2, sqrt(r2));
    if (!(a12 < alpha0)) return NAN;
    double r12 = sqrt(r2), r13 = sqrt(r3), r23 = sqrt(r3 / r2);
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(alpha0 - a12);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (1.0 - or_tvn(z1, z2, mid, r12, r13, r23) > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Four-variate normal CDF for n = 4 nested populations with fractions
 * r[0] = 1 > r[1] > r[2] > r[3] (null correlations sqrt(r_j / r_i),
 * Appendix A.1).  Each population's statistic is the scaled sum over its
 * members, so the statistics form a Markov chain: given Z2, Z1 is independent
 * of (Z3, Z4), and given Z3, Z4 is independent of (Z1, Z2).  Integrating over
 * (Z2, Z3) = (x, y) with density phi(x) phi((y - a x)/s)/s, a = sqrt(r3/r2),
 * s = sqrt(1 - r3/r2):
 *   Phi_4(h) = int_{x <= h2} phi(x) Phi((h1 - b x)/sb)
 *              int_{y <= h3} phi((y - a x)/s)/s Phi((h4 - c y)/sc) dy dx,
 * b = sqrt(r2), sb = sqrt(1 - r2), c = sqrt(r4/r3), sc = sqrt(1 - r4/r3).
 * Two nested one-dimensional integrals of univariate CDFs: the form this
 * oracle evaluates for the n = 4 model; or_qvn (conditioning on Z1 through
 * Phi_3, any correlation matrix) is its check. */
typedef struct { double h1, h3, h4, a, s, b, sb, c, sc, x; } qvn4_ctx;

static double qvn4_inner(double y, void *ctx)
{
    const qvn4_ctx *c = (const qvn4_ctx *)ctx;
    return or_phi((y - c->a * c->x) / c->s) / c->s * or_Phi((c->h4 - c->c * y) / c->sc);
}

static double qvn4_outer(double x, void *ctx)
{
    qvn4_ctx c = *(const qvn4_ctx *)ctx;
    c.x = x;
    double f1 = or_Phi((c.h1 - c.b * x) / c.sb);
    if (f1 == 0.0) return 0.0;
    double lo = fmin(c.a * x - 12.0 * c.s, c.h3 - 10.0 * c.s);
    double inner = c.h3 == INFINITY ? or_Phi((c.h4 - c.c * c.a * x) / sqrt(c.c * c.c * c.s * c.s + c.sc * c.sc))
                                    : or_quad(qvn4_inner, &c, lo, c.h3);
    return or_phi(x) * f1 * inner;
}

double or_qvn_nested(const double *h, const double *r)
{
    for (int i = 0; i < 4; ++i) {
        if (isnan(h[i])) return NAN;
        if (h[i] == -INFINITY) return 0.0;
    }
    qvn4_ctx c = {h[0], h[2], h[3], sqrt(r[2] / r[1]), sqrt(1.0 - r[2] / r[1]), sqrt(r[1]), sqrt(1.0 - r[1]),
                  sqrt(r[3] / r[2]), sqrt(1.0 - r[3] / r[2]), 0.0};
    double hi = h[1] == INFINITY ? 12.0 : h[1];
    return or_quad(qvn4_outer, &c, fmin(-12.0, hi - 10.0), hi);
}

/* One critical value z* for four nested populations 1 > r2 > r3 > r4 with
 * 1 - Phi_4(z*, z*, z*, z*) = alpha0 (Formula 2 with equal levels), by
 * bisection between one test at level alpha0 and the Bonferroni value. */
double or_zstar4(double r2, double r3, double r4, double alpha0)
{
    double r[4] = {1.0, r2, r3, r4};
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(alpha0 / 4.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double h[4] = {mid, mid, mid, mid};
        if (1.0 - or_qvn_nested(h, r) > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* n = 4 nested populations 1 > r2 > r3 > r4: the fourth critical value with
 * FWER = 1 - Phi_4(z1, z2, z3, z4) = alpha0 given the first three, by
 * bisection between the fourth test alone at level alpha0 and the union bound
 * (the first three spend a123 = 1 - Phi_3(z1, z2, z3)).  NaN when
 * a123 >= alpha0. */
double or_z4_fwer(double z1, double z2, double z3, double r2, double r3, double r4, double alpha0)
{
    double r[4] = {1.0, r2, r3, r4};
    double a123 = 1.0 - or_tvn(z1, z2, z3, sqrt(r2), sqrt(r3), sqrt(r3 / r2));
    if (!(a123 < alpha0)) return NAN;
    double lo = -or_Phiinv(alpha0), hi = -or_Phiinv(alpha0 - a123);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double h[4] = {z1, z2, z3, mid};
        if (1.0 - or_qvn_nested(h, r) > alpha0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Information units needed for a one-sided level-alpha test with power
 * 1 - beta at hazard reduction delta (Sec. 3, the I_3 sizing formula). */
double or_info_units(double alpha, double beta, double delta)
{
    double za = -or_Phiinv(alpha), zb = -or_Phiinv(beta);
    double l = log1p(-delta);
    return (za + zb) * (za + zb) / (l * l);
}

/* ======================================================================== */
/* Counter-based random numbers                                             */
/* ======================================================================== */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011): each round multiplies counter words
 * 0 and 2 by fixed 32-bit constants, mixes the high halves with words 1 and 3
 * and the key, and the key is advanced by two Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on (0,1) from two words: the top 26 bits of each form a 52-bit
 * integer n, and u = (n + 1/2) 2^-52.  Every step is exact in FP64, so
 * u is never 0 or 1 and 1 - u is again such a value. */
double or_uniform52(uint32_t wa, uint32_t wb)
{
    uint64_t n = ((uint64_t)(wa >> 6) << 26) | (uint64_t)(wb >> 6);
    return ((double)n + 0.5) * 0x1p-52;
}

/* The uniforms of draw k: Philox blocks with key (seed lo, seed hi) and
 * counter (k lo, k hi, scenario, b) for b = 0, 1, ...; uniform i takes words
 * 2i and 2i+1 of the concatenated output. */
static void draw_uniforms(const or_problem *p, uint64_t k, int nu, double *u)
{
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    uint32_t words[16];
    int nblk = (2 * nu + 3) / 4;
    for (int b = 0; b < nblk; ++b) {
        uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), p->scenario, (uint32_t)b};
        or_philox4x32_10(ctr, key, words + 4 * b);
    }
    for (int i = 0; i < nu; ++i) u[i] = or_uniform52(words[2 * i], words[2 * i + 1]);
}

/* ======================================================================== */
/* Designs and draws                                                        */
/* ======================================================================== */

int64_t or_grid_size(const or_problem *p)
{
    int64_t G = 1;
    for (int j = 0; j < p->d; ++j) G *= p->m[j];
    return G;
}

/* Grid design g (row-major, axis 0 slowest): q_j = q_lo + ((q_hi - q_lo) i_j)
 * / (m_j - 1), each operation rounded separately in this order. */
/* Coordinate range of grid axis j: the subgroup-fraction axis of the alpha
 * design space, else [q_lo, q_hi]. */
static void axis_range(const or_problem *p, int j, double *lo, double *hi)
{
    if (p->design_space == OR_DESIGN_ALPHA && p->d == 2 && j == 0) {
        *lo = p->r_lo;
        *hi = p->r_hi;
    } else {
        *lo = p->q_lo;
        *hi = p->q_hi;
    }
}

void or_grid_point(const or_problem *p, int64_t g, double *q, int32_t *idx)
{
    for (int j = p->d - 1; j >= 0; --j) {
        int64_t i = g % p->m[j];
        g /= p->m[j];
        double lo, hi;
        axis_range(p, j, &lo, &hi);
        double span = hi - lo;
        double t = span * (double)i;
        t = t / (double)(p->m[j] - 1);
        q[j] = lo + t;
        if (idx) idx[j] = (int32_t)i;
    }
}

/* Design quantities: cutoffs, subgroup fraction r (the proportion r_i of
 * Sec. 2.1), correlation sqrt(r) of the nested tests (Appendix A.1) and the
 * critical values from the chosen alpha rule (Formula 2). */
void or_make_design(const or_problem *p, const double *q, or_design *o)
{
    memset(o, 0, sizeof *o);
    if (p->design_space == OR_DESIGN_ALPHA4) {
        /* (alpha_1, alpha_2, alpha_3) for four nested populations, alpha_4 on
         * the FWER boundary (Formula 2 with n = 4). */
        for (int j = 0; j < 3; ++j) o->q[j] = q[j];
        o->r = p->r_lo;
        o->rho = sqrt(o->r);
        o->r3 = p->r_hi;
        o->r4 = p->r_4;
        o->z1 = -or_Phiinv(q[0]);
        o->z2 = -or_Phiinv(q[1]);
        o->z3 = -or_Phiinv(q[2]);
        o->z4 = or_z4_fwer(o->z1, o->z2, o->z3, o->r, o->r3, o->r4, p->alpha0);
        return;
    }
    if (p->design_space == OR_DESIGN_ALPHA3) {
        /* (alpha_1, alpha_2) for three nested populations, alpha_3 on the FWER
         * boundary (Formula 2 with n = 3). */
        o->q[0] = q[0];
        o->q[1] = q[1];
        o->r = p->r_lo;
        o->rho = sqrt(o->r);
        o->r3 = p->r_hi;
        o->z1 = -or_Phiinv(q[0]);
        o->z2 = -or_Phiinv(q[1]);
        o->z3 = or_z3_fwer(o->z1, o->z2, o->r, o->r3, p->alpha0);
        return;
    }
    if (p->design_space == OR_DESIGN_NESTED3) {
        /* Two cutoffs on one biomarker: populations all, x > c_1 and x > c_2. */
        o->q[0] = q[0];
        o->q[1] = q[1];
        o->c[0] = or_Phiinv(q[0]);
        o->c[1] = or_Phiinv(q[1]);
        o->r = 1.0 - q[0];
        o->rho = sqrt(o->r);
        o->r3 = 1.0 - q[1];
        int ok = q[0] < q[1] && o->r3 * (1.0 - o->r) <= 0.975 * 0.975 * o->r * (1.0 - o->r3);
        double z = !ok ? NAN
                 : p->alpha_rule == OR_ALPHA_BONFERRONI ? -or_Phiinv(p->alpha0 / 3.0)
                                                        : or_zstar3(o->r, o->r3, p->alpha0);
        o->z1 = o->z2 = o->z3 = z;
        return;
    }
    if (p->design_space == OR_DESIGN_NESTED4) {
        /* Three cutoffs on one biomarker: populations all, x > c_1, x > c_2, x > c_3. */
        for (int j = 0; j < 3; ++j) {
            o->q[j] = q[j];
            o->c[j] = or_Phiinv(q[j]);
        }
        o->r = 1.0 - q[0];
        o->rho = sqrt(o->r);
        o->r3 = 1.0 - q[1];
        o->r4 = 1.0 - q[2];
        double r2 = o->r, r3 = o->r3, r4 = o->r4;
        int ok = q[0] < q[1] && q[1] < q[2] && r3 * (1.0 - r2) <= 0.975 * 0.975 * r2 * (1.0 - r3) &&
                 r4 * (r2 - r3) <= 0.975 * 0.975 * r3 * (r2 - r4) && r3 <= 0.95 * r2;
        double z = !ok ? NAN
                 : p->alpha_rule == OR_ALPHA_BONFERRONI ? -or_Phiinv(p->alpha0 / 4.0)
                                                        : or_zstar4(r2, r3, r4, p->alpha0);
        o->z1 = o->z2 = o->z3 = o->z4 = z;
        return;
    }
    if (p->design_space == OR_DESIGN_ALPHA) {
        /* (r_2, alpha_1) or alpha_1 alone: the nested pair of Sec. 2.2 with the
         * level split on the FWER boundary of Formula 2. */
        for (int j = 0; j < p->d; ++j) o->q[j] = q[j];
        o->r = (p->d == 2) ? q[0] : p->r_lo;
        o->rho = sqrt(o->r);
        o->z1 = -or_Phiinv(q[p->d - 1]);
        o->z2 = or_z2_fwer(o->z1, o->r, p->alpha0);
        return;
    }
    for (int j = 0; j < p->d; ++j) {
        o->q[j] = q[j];
        o->c[j] = or_Phiinv(q[j]);
    }
    o->r = (p->d == 1) ? 1.0 - q[0] : or_orthant(p->d, o->c, p->rho_b);
    o->rho = sqrt(o->r);
    switch (p->alpha_rule) {
    case OR_ALPHA_FWER_EQUAL:
        o->z1 = o->z2 = or_zstar(o->r, p->alpha0);
        break;
    case OR_ALPHA_BONFERRONI:
        o->z1 = o->z2 = -or_Phiinv(0.5 * p->alpha0);
        break;
    case OR_ALPHA_SPLIT:
        o->z1 = -or_Phiinv(p->alpha_fixed[0]);
        o->z2 = or_z2_fwer(o->z1, o->r, p->alpha0);
        break;
    default:
        o->z1 = p->alpha_fixed[0] > 0.0 ? -or_Phiinv(p->alpha_fixed[0]) : INFINITY;
        o->z2 = p->alpha_fixed[1] > 0.0 ? -or_Phiinv(p->alpha_fixed[1]) : INFINITY;
        break;
    }
}

/* One draw from the prior f(Delta) of Formula 4.
 * Step prior: baseline effect b0, extra effect b1 in responders, true cutoff
 * quantile tau_j per biomarker; responders R = {x_j > Phi^-1(tau_j) all j}.
 * Paper prior (Formula 10): two standard normals for the Gaussian effects. */
void or_make_draw(const or_problem *p, uint64_t k, or_draw *o)
{
    memset(o, 0, sizeof *o);
    if (p->effect == OR_EFFECT_STEP) {
        int d = (p->design_space == OR_DESIGN_NESTED3 || p->design_space == OR_DESIGN_NESTED4) ? 1 : p->d;   /* one biomarker */
        draw_uniforms(p, k, 2 + d, o->u);
        o->b0 = p->mu_b0 + p->sd_b0 * or_Phiinv(o->u[0]);
        o->b1 = p->mu_b1 + p->sd_b1 * or_Phiinv(o->u[1]);
        for (int j = 0; j < d; ++j) {
            double span = p->tau_hi - p->tau_lo;
            double x = span * o->u[2 + j];
            o->tau[j] = p->tau_lo + x;
            o->t[j] = or_Phiinv(o->tau[j]);
        }
        o->PR = (d == 1) ? 1.0 - o->tau[0] : or_orthant(d, o->t, p->rho_b);
    } else if (p->design_space == OR_DESIGN_ALPHA3) {
        draw_uniforms(p, k, 3, o->u);
        o->e1 = or_Phiinv(o->u[0]);
        o->e2 = or_Phiinv(o->u[1]);
        o->e3 = or_Phiinv(o->u[2]);
    } else if (p->design_space == OR_DESIGN_ALPHA4) {
        draw_uniforms(p, k, 4, o->u);
        o->e1 = or_Phiinv(o->u[0]);
        o->e2 = or_Phiinv(o->u[1]);
        o->e3 = or_Phiinv(o->u[2]);
        o->e4 = or_Phiinv(o->u[3]);
    } else {
        draw_uniforms(p, k, 2, o->u);
        o->e1 = or_Phiinv(o->u[0]);
        o->e2 = or_Phiinv(o->u[1]);
    }
}

static double logistic(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Fraction of the population that is both in the subgroup S and a responder:
 * P(x_j > max(c_j, t_j) for all j).  Axis j takes c_j when q_j > tau_j.  With a
 * logistic width w > 0 the axis factor is the mix s_j [cut at c_j] +
 * (1 - s_j) [cut at t_j], s_j = 1 / (1 + exp(-(q_j - tau_j)/w)). */
double or_overlap(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    int d = p->d;
    if (d == 1) {
        double q = ds->q[0], tau = dr->tau[0];
        if (p->width > 0.0) {
            double s = logistic((q - tau) / p->width);
            return 1.0 - (s * q + (1.0 - s) * tau);
        }
        return 1.0 - (q > tau ? q : tau);
    }
    orth_ctx o;
    memset(&o, 0, sizeof o);
    o.d = d;
    for (int j = 0; j < d; ++j) {
        if (p->width > 0.0) {
            o.kind[j] = FK_MIX;
            o.c[j] = ds->c[j];
            o.t[j] = dr->t[j];
            o.s[j] = logistic((ds->q[j] - dr->tau[j]) / p->width);
        } else {
            o.kind[j] = FK_CUT;
            o.c[j] = (ds->q[j] > dr->tau[j]) ? ds->c[j] : dr->t[j];
        }
    }
    return orth_integral(&o, p->rho_b);
}

/* Effects on the paper's Delta scale for the two populations. */
static void effects(const or_problem *p, const or_design *ds, const or_draw *dr,
                    double *d1, double *d2, double *O_out)
{
    if (p->effect == OR_EFFECT_STEP) {
        double O = or_overlap(p, ds, dr);
        *d1 = dr->b0 + dr->b1 * dr->PR;
        *d2 = dr->b0 + dr->b1 * O / ds->r;
        if (O_out) *O_out = O;
    } else {
        double r = ds->r, E = p->paper_events;
        double th1 = -log1p(-(p->paper_a - p->paper_b));
        double th2 = -log1p(-(p->paper_a - p->paper_b * r));
        double s1 = 1.0 / sqrt(E / 4.0), s2 = 1.0 / sqrt(E * r / 4.0);
        *d1 = th1 + s1 * dr->e1;
        *d2 = th2 + s2 * (sqrt(r) * dr->e1 + sqrt(1.0 - r) * dr->e2);
        if (O_out) *O_out = 0.0;
    }
}

/* Success probability for one design and one draw: one minus the CDF of the
 * alternative distribution (Formula 3) at the critical values, i.e. one
 * summand of Formula 5. */
/* Three nested populations under Formula 10: Delta_i = theta_i + sigma_i Y_i
 * with standard normals Y of the nested null correlations (corr(Y_i, Y_j) =
 * sqrt(r_j / r_i)): Y1 = e1, Y2 = sqrt(r2) e1 + sqrt(1 - r2) e2,
 * Y3 = sqrt(r3) e1 + sqrt(r3 (1 - r2) / r2) e2 + sqrt(1 - r3 / r2) e3. */
static double success3(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    if (isnan(ds->z3)) return NAN;
    double r[3] = {1.0, ds->r, ds->r3}, E = p->paper_events, I = p->info;
    double Y[3] = {dr->e1, sqrt(r[1]) * dr->e1 + sqrt(1.0 - r[1]) * dr->e2,
                   sqrt(r[2]) * dr->e1 + sqrt(r[2] * (1.0 - r[1]) / r[1]) * dr->e2 + sqrt(1.0 - r[2] / r[1]) * dr->e3};
    double z[3] = {ds->z1, ds->z2, ds->z3}, h[3];
    for (int i = 0; i < 3; ++i) {
        double th = -log1p(-(p->paper_a - p->paper_b * r[i]));
        double sg = 1.0 / sqrt(E * r[i] / 4.0);
        h[i] = z[i] - sqrt(r[i] * I) * (th + sg * Y[i]);
    }
    return 1.0 - or_tvn(h[0], h[1], h[2], sqrt(r[1]), sqrt(r[2]), sqrt(r[2] / r[1]));
}

/* Four nested populations under Formula 10: the standard normals Y of the
 * nested null correlations, each population's statistic being the scaled sum
 * over its members, follow Y_1 = e1 and
 * Y_{i+1} = sqrt(r_{i+1}/r_i) Y_i + sqrt(1 - r_{i+1}/r_i) e_{i+1}
 * (the inner population's sum is a fraction of the outer one's plus an
 * independent part); for i <= 3 this is the three-population construction. */
static double success4(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    if (isnan(ds->z4)) return NAN;
    double r[4] = {1.0, ds->r, ds->r3, ds->r4}, E = p->paper_events, I = p->info;
    double e[4] = {dr->e1, dr->e2, dr->e3, dr->e4}, Y[4];
    Y[0] = e[0];
    for (int i = 1; i < 4; ++i) Y[i] = sqrt(r[i] / r[i - 1]) * Y[i - 1] + sqrt(1.0 - r[i] / r[i - 1]) * e[i];
    double z[4] = {ds->z1, ds->z2, ds->z3, ds->z4}, h[4];
    for (int i = 0; i < 4; ++i) {
        double th = -log1p(-(p->paper_a - p->paper_b * r[i]));
        double sg = 1.0 / sqrt(E * r[i] / 4.0);
        h[i] = z[i] - sqrt(r[i] * I) * (th + sg * Y[i]);
    }
    return 1.0 - or_qvn_nested(h, r);
}

/* Three nested populations cut from one biomarker (step prior): population i
 * has fraction r_i and responders R = {x > t}, P(R and x > c_i) = 1 - max(q_i, tau),
 * so Delta_i = b0 + b1 (1 - max(q_i, tau)) / r_i (q_0 = 0, r_1 = 1) and the
 * drift is sqrt(r_i I) Delta_i (Formula 3); the summand is 1 - Phi_3 at
 * z* - drift with the null correlations of Appendix A.1. */
static double success_nested3(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    if (isnan(ds->z3)) return NAN;
    double q[3] = {0.0, ds->q[0], ds->q[1]}, r[3] = {1.0, ds->r, ds->r3}, h[3];
    double z[3] = {ds->z1, ds->z2, ds->z3};
    for (int i = 0; i < 3; ++i) {
        double delta = dr->b0 + dr->b1 * (1.0 - fmax(q[i], dr->tau[0])) / r[i];
        h[i] = z[i] - sqrt(r[i] * p->info) * delta;
    }
    return 1.0 - or_tvn(h[0], h[1], h[2], sqrt(r[1]), sqrt(r[2]), sqrt(r[2] / r[1]));
}

/* Four populations from three cutoffs: as success_nested3 with q_3, r_4 and
 * the nested Phi_4. */
static double success_nested4(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    if (isnan(ds->z4)) return NAN;
    double q[4] = {0.0, ds->q[0], ds->q[1], ds->q[2]}, r[4] = {1.0, ds->r, ds->r3, ds->r4}, h[4];
    for (int i = 0; i < 4; ++i) {
        double delta = dr->b0 + dr->b1 * (1.0 - fmax(q[i], dr->tau[0])) / r[i];
        h[i] = ds->z4 - sqrt(r[i] * p->info) * delta;
    }
    return 1.0 - or_qvn_nested(h, r);
}

double or_success(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    if (p->design_space == OR_DESIGN_NESTED4) return success_nested4(p, ds, dr);
    if (p->design_space == OR_DESIGN_NESTED3) return success_nested3(p, ds, dr);
    if (p->design_space == OR_DESIGN_ALPHA4) return success4(p, ds, dr);
    if (p->design_space == OR_DESIGN_ALPHA3) return success3(p, ds, dr);
    double d1, d2;
    effects(p, ds, dr, &d1, &d2, NULL);
    double mu1 = sqrt(p->info) * d1;
    double mu2 = sqrt(ds->r * p->info) * d2;
    return 1.0 - or_bvn(ds->z1 - mu1, ds->z2 - mu2, ds->rho);
}

/* ======================================================================== */
/* Monte Carlo estimate (Formula 5)                                         */
/* ======================================================================== */

static double pairwise_sum(const double *x, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += x[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise_sum(x, h) + pairwise_sum(x + h, n - h);
}

static void mean_var(double *vals, int64_t M, double *mean, double *var)
{
    double m = pairwise_sum(vals, M) / (double)M;
    *mean = m;
    if (var) {
        for (int64_t k = 0; k < M; ++k) vals[k] = (vals[k] - m) * (vals[k] - m);
        *var = M > 1 ? pairwise_sum(vals, M) / (double)(M - 1) : 0.0;
    }
}

static or_draw *make_draws(const or_problem *p, uint64_t k0, uint64_t M)
{
    or_draw *dr = (or_draw *)malloc(sizeof(or_draw) * (size_t)M);
    if (!dr) return NULL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < (int64_t)M; ++k) or_make_draw(p, k0 + (uint64_t)k, &dr[k]);
    return dr;
}

void or_eval_points(const or_problem *p, int64_t n, const double *q,
                    uint64_t k0, uint64_t M, double *mean, double *var)
{
    or_draw *dr = make_draws(p, k0, M);
    double *vals = (double *)malloc(sizeof(double) * (size_t)M);
    if (!dr || !vals) { free(dr); free(vals); return; }
    for (int64_t i = 0; i < n; ++i) {
        or_design ds;
        or_make_design(p, q + i * p->d, &ds);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < (int64_t)M; ++k) vals[k] = or_success(p, &ds, &dr[k]);
        mean_var(vals, (int64_t)M, &mean[i], var ? &var[i] : NULL);
    }
    free(vals);
    free(dr);
}

void or_eval_grid(const or_problem *p, int64_t n, const int64_t *g_list,
                  uint64_t k0, uint64_t M, double *mean, double *var)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)(n * p->d));
    if (!q) return;
    for (int64_t i = 0; i < n; ++i) or_grid_point(p, g_list[i], q + i * p->d, NULL);
    or_eval_points(p, n, q, k0, M, mean, var);
    free(q);
}

/* ======================================================================== */
/* Two-layer sampling estimator (Formulas 6 and 7)                          */
/* ======================================================================== */
/*
 * Formula 6 replaces Phi_Sigma(b) by the share of N2 draws x^(l) of the null
 * statistics (Formula 1) that lie below b in every coordinate; Formula 7
 * averages that over the N1 prior draws, one set of x^(l) for all of them:
 *   P = 1 - (1/(N1 N2)) sum_k sum_l [x^(l)_j <= z_j - sqrt(r_j I) Delta^(k)_j, all j].
 * The inner draw l takes its uniforms from the Philox stream whose fourth
 * counter word has its top bit set, turns them into standard normals e_j and
 * builds the nested null correlations sqrt(r_j / r_i) of Appendix A.1 by the
 * chain x_1 = e_1, x_{i+1} = sqrt(r_{i+1}/r_i) x_i + sqrt(1 - r_{i+1}/r_i) e_{i+1}.
 *
 * The variance (corrected Appendix A.2).  The indicator h(Delta, x) has the
 * Hoeffding parts h1(Delta) = E_x h, h2(x) = E_Delta h and a remainder, which
 * are uncorrelated, so with theta = E h
 *   Var(mean h) = s1/N1 + s2/N2 + (theta (1 - theta) - s1 - s2)/(N1 N2),
 * s1 = Var h1, s2 = Var h2; A.2 keeps only theta (1 - theta)/(N1 N2).  Counting
 * the comparisons in A x B blocks (consecutive outer draws x consecutive inner
 * draws), the block means follow a two-way crossed random-effects model, and
 * (MS_A + MS_B - MS_E)/(A B) estimates that variance without bias.
 */
static void inner_draw(const or_problem *p, uint64_t l, int n, const double *r, double *x)
{
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    uint32_t w[8];
    for (int b = 0; b < 2; ++b) {
        uint32_t ctr[4] = {(uint32_t)l, (uint32_t)(l >> 32), p->scenario, 0x80000000u | (uint32_t)b};
        or_philox4x32_10(ctr, key, w + 4 * b);
    }
    for (int i = 0; i < n; ++i) {
        double e = or_Phiinv(or_uniform52(w[2 * i], w[2 * i + 1]));
        x[i] = (i == 0) ? e : sqrt(r[i] / r[i - 1]) * x[i - 1] + sqrt(1.0 - r[i] / r[i - 1]) * e;
    }
}

/* Thresholds b_j = z_j - sqrt(r_j I) Delta_j of outer draw dr for design ds
 * under Formula 10 (Delta_i = theta_i + sigma_i Y_i, Y the chain of the draw's
 * normals); n = 2, 3 or 4.  Returns the fractions r_1..r_n in r. */
static int outer_thresholds(const or_problem *p, const or_design *ds, const or_draw *dr, double *b, double *r)
{
    int n = p->design_space == OR_DESIGN_ALPHA4 ? 4 : p->design_space == OR_DESIGN_ALPHA3 ? 3 : 2;
    double rr[4] = {1.0, ds->r, ds->r3, ds->r4}, z[4] = {ds->z1, ds->z2, ds->z3, ds->z4};
    double e[4] = {dr->e1, dr->e2, dr->e3, dr->e4}, Y[4];
    for (int i = 0; i < n; ++i) {
        Y[i] = (i == 0) ? e[0] : sqrt(rr[i] / rr[i - 1]) * Y[i - 1] + sqrt(1.0 - rr[i] / rr[i - 1]) * e[i];
        double th = -log1p(-(p->paper_a - p->paper_b * rr[i]));
        double sg = 1.0 / sqrt(p->paper_events * rr[i] / 4.0);
        b[i] = z[i] - sqrt(rr[i] * p->info) * (th + sg * Y[i]);
        r[i] = rr[i];
    }
    return n;
}

void or_eval_grid_two_layer(const or_problem *p, int64_t ng, const int64_t *g_list, uint64_t N1,
                            uint64_t N2, int A, int B, double *mean, double *var, uint32_t *blocks)
{
    or_draw *dr = make_draws(p, 0, N1);
    double *x = (double *)malloc(sizeof(double) * 4 * (size_t)N2);
    uint32_t *cnt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)A * B);
    double *R = (double *)malloc(sizeof(double) * (size_t)A), *C = (double *)malloc(sizeof(double) * (size_t)B);
    if (!dr || !x || !cnt || !R || !C) { free(dr); free(x); free(cnt); free(R); free(C); return; }
    uint64_t SA = N1 / (uint64_t)A, SB = N2 / (uint64_t)B;
    for (int64_t i = 0; i < ng; ++i) {
        double q[6], b[4], r[4];
        or_design ds;
        or_grid_point(p, g_list[i], q, NULL);
        or_make_design(p, q, &ds);
        int n = outer_thresholds(p, &ds, &dr[0], b, r);
        int bad = isnan(ds.z1) || isnan(ds.z2) || (n >= 3 && isnan(ds.z3)) || (n >= 4 && isnan(ds.z4));
        memset(cnt, 0, sizeof(uint32_t) * (size_t)A * B);
        if (bad) {
            mean[i] = NAN;
            if (var) var[i] = NAN;
            if (blocks) memcpy(blocks + i * A * B, cnt, sizeof(uint32_t) * (size_t)A * B);
            continue;
        }
        for (uint64_t l = 0; l < N2; ++l) inner_draw(p, l, n, r, x + 4 * l);
        for (uint64_t k = 0; k < N1; ++k) {
            outer_thresholds(p, &ds, &dr[k], b, r);
            for (uint64_t l = 0; l < N2; ++l) {
                int below = 1;
                for (int j = 0; j < n; ++j) below = below && (x[4 * l + j] <= b[j]);
                cnt[(k / SA) * B + l / SB] += below;
            }
        }
        uint64_t T = 0;
        for (int t = 0; t < A * B; ++t) T += cnt[t];
        mean[i] = 1.0 - (double)T / ((double)N1 * (double)N2);
        if (blocks) memcpy(blocks + i * A * B, cnt, sizeof(uint32_t) * (size_t)A * B);
        if (var) {
            double cell = (double)SA * (double)SB, M = 0.0;
            for (int a = 0; a < A; ++a) {
                double s = 0.0;
                for (int c = 0; c < B; ++c) s += cnt[a * B + c] / cell;
                R[a] = s / B;
                M += R[a];
            }
            M /= A;
            for (int c = 0; c < B; ++c) {
                double s = 0.0;
                for (int a = 0; a < A; ++a) s += cnt[a * B + c] / cell;
                C[c] = s / A;
            }
            double sa = 0.0, sc = 0.0, se = 0.0;
            for (int a = 0; a < A; ++a) sa += (R[a] - M) * (R[a] - M);
            for (int c = 0; c < B; ++c) sc += (C[c] - M) * (C[c] - M);
            for (int a = 0; a < A; ++a)
                for (int c = 0; c < B; ++c) {
                    double d = cnt[a * B + c] / cell - R[a] - C[c] + M;
                    se += d * d;
                }
            double msa = B * sa / (A - 1), msb = A * sc / (B - 1), mse = se / ((double)(A - 1) * (B - 1));
            var[i] = (msa + msb - mse) / ((double)A * B);
        }
    }
    free(dr); free(x); free(cnt); free(R); free(C);
}

/* ======================================================================== */
/* Derivative in the first level (Appendix A.3, two nested tests)           */
/* ======================================================================== */
/*
 * Appendix A.3 differentiates the power under the integral: with one test,
 * dP/d alpha = E[phi(z - mu) / phi(z)].  For the nested pair the summand is
 * 1 - F(z1 - mu1, z2 - mu2), F(h, k) = Phi_2(h, k; rho), and by the chain rule
 *   d/d alpha_1 = -(dF/dh dz1/d alpha_1 + dF/dk dz2/d alpha_1),
 * with the textbook partials dF/dh = phi(h) Phi((k - rho h)/s),
 * dF/dk = phi(k) Phi((h - rho k)/s), s = sqrt(1 - rho^2), and
 * z1 = Phi^-1(1 - alpha_1), so dz1/d alpha_1 = -1/phi(z1).  A fixed second
 * level gives dz2/d alpha_1 = 0 (and a switched-off one leaves
 * F(h, +inf) = Phi(h)); a second level on the FWER boundary, F(z1, z2) =
 * 1 - alpha0, moves with z1 as dz2/dz1 = -(dF/dh)/(dF/dk) at (z1, z2).
 */
static double bvn_dh(double h, double k, double rho)
{
    if (isinf(k)) return or_phi(h);
    return or_phi(h) * or_Phi((k - rho * h) / sqrt(1.0 - rho * rho));
}

double or_dsuccess_dalpha1(const or_problem *p, const or_design *ds, const or_draw *dr)
{
    double d1, d2;
    effects(p, ds, dr, &d1, &d2, NULL);
    const double h = ds->z1 - sqrt(p->info) * d1;
    const double k = ds->z2 - sqrt(ds->r * p->info) * d2;
    const double dz1 = -1.0 / or_phi(ds->z1);
    double dz2 = 0.0;
    if (p->alpha_rule == OR_ALPHA_SPLIT)
        dz2 = -bvn_dh(ds->z1, ds->z2, ds->rho) / bvn_dh(ds->z2, ds->z1, ds->rho) * dz1;
    const double dFk = isinf(k) ? 0.0 : bvn_dh(k, h, ds->rho);
    return -(bvn_dh(h, k, ds->rho) * dz1 + dFk * dz2);
}

void or_eval_grid_dalpha(const or_problem *p, int64_t n, const int64_t *g_list,
                         uint64_t k0, uint64_t M, double *mean, double *dmean)
{
    or_draw *dr = make_draws(p, k0, M);
    double *vals = (double *)malloc(sizeof(double) * (size_t)M);
    double *dv = (double *)malloc(sizeof(double) * (size_t)M);
    if (!dr || !vals || !dv) { free(dr); free(vals); free(dv); return; }
    for (int64_t i = 0; i < n; ++i) {
        double q[6];
        or_design ds;
        or_grid_point(p, g_list[i], q, NULL);
        or_make_design(p, q, &ds);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < (int64_t)M; ++k) {
            vals[k] = or_success(p, &ds, &dr[k]);
            dv[k] = or_dsuccess_dalpha1(p, &ds, &dr[k]);
        }
        mean[i] = pairwise_sum(vals, (int64_t)M) / (double)M;
        dmean[i] = pairwise_sum(dv, (int64_t)M) / (double)M;
    }
    free(dv);
    free(vals);
    free(dr);
}

/* ======================================================================== */
/* Smoothing and argmax                                                     */
/* ======================================================================== */
/*
 * Nadaraya-Watson smoothing of the grid surface with a product Gaussian
 * kernel K(g,h) = prod_j exp(-((q_j(g) - q_j(h)) / b_j)^2 / 2), untruncated:
 * S(g) = sum_h K(g,h) f(h) / sum_h K(g,h).  This stands in for the paper's
 * thin-plate-spline fit of the noisy estimates (Sec. 2.3).
 */
void or_smooth_direct(const or_problem *p, const double *in, double *out)
{
    int d = p->d;
    int64_t G = or_grid_size(p);
    double *q = (double *)malloc(sizeof(double) * (size_t)(G * d));
    if (!q) return;
    for (int64_t g = 0; g < G; ++g) or_grid_point(p, g, q + g * d, NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < G; ++g) {
        double num = 0.0, den = 0.0;
        for (int64_t h = 0; h < G; ++h) {
            double e = 0.0;
            for (int j = 0; j < d; ++j) {
                double x = (q[g * d + j] - q[h * d + j]) / p->bandwidth[j];
                e += -0.5 * x * x;
            }
            double w = exp(e);
            num += w * in[h];
            den += w;
        }
        out[g] = num / den;
    }
    free(q);
}

/* The smoother over a grid whose surface is NaN at some designs (three
 * nested populations: designs without a third level): the same kernel sum
 * over the designs that have a value only; designs without one stay NaN.
 * This is the surface fit of Sec. 2.3 taken over the evaluated points. */
void or_smooth_masked(const or_problem *p, const double *in, double *out)
{
    int d = p->d;
    int64_t G = or_grid_size(p);
    double *q = (double *)malloc(sizeof(double) * (size_t)(G * d));
    if (!q) return;
    for (int64_t g = 0; g < G; ++g) or_grid_point(p, g, q + g * d, NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < G; ++g) {
        if (isnan(in[g])) {
            out[g] = NAN;
            continue;
        }
        double num = 0.0, den = 0.0;
        for (int64_t h = 0; h < G; ++h) {
            if (isnan(in[h])) continue;
            double e = 0.0;
            for (int j = 0; j < d; ++j) {
                double x = (q[g * d + j] - q[h * d + j]) / p->bandwidth[j];
                e += -0.5 * x * x;
            }
            double w = exp(e);
            num += w * in[h];
            den += w;
        }
        out[g] = num / den;
    }
    free(q);
}

/* The smoothed surface at a continuous design q (Sec. 2.3's fitted surface,
 * evaluated between grid points): the Nadaraya-Watson ratio
 *   S(q) = sum_h K(q, q_h) f_h / sum_h K(q, q_h),
 * K = prod_j exp(-((q_j - q_{h,j}) / b_j)^2 / 2) over the grid designs h, the
 * designs whose value is NaN skipped.  At a grid design it is the value
 * or_smooth_masked gives there. */
double or_smooth_at(const or_problem *p, const double *in, const double *q)
{
    int d = p->d;
    int64_t G = or_grid_size(p);
    double num = 0.0, den = 0.0;
#pragma omp parallel for reduction(+ : num, den) schedule(static)
    for (int64_t h = 0; h < G; ++h) {
        if (isnan(in[h])) continue;
        double qh[6];
        or_grid_point(p, h, qh, NULL);
        double e = 0.0;
        for (int j = 0; j < d; ++j) {
            double x = (q[j] - qh[j]) / p->bandwidth[j];
            e += -0.5 * x * x;
        }
        double w = exp(e);
        num += w * in[h];
        den += w;
    }
    return num / den;
}

/* The same smoother through its factorisation: the row-normalised product
 * kernel is the product of row-normalised one-axis kernels, applied one axis
 * at a time. */
void or_smooth_separable(const or_problem *p, const double *in, double *out)
{
    int d = p->d;
    int64_t G = or_grid_size(p);
    double *a = (double *)malloc(sizeof(double) * (size_t)G);
    double *b = (double *)malloc(sizeof(double) * (size_t)G);
    if (!a || !b) { free(a); free(b); return; }
    memcpy(a, in, sizeof(double) * (size_t)G);
    int64_t inner = G;
    for (int j = 0; j < d; ++j) {
        int m = p->m[j];
        inner /= m;                    /* product of axis sizes after j */
        int64_t outer = G / (inner * m);
        double *W = (double *)malloc(sizeof(double) * (size_t)m * m);
        double *qa = (double *)malloc(sizeof(double) * (size_t)m);
        double lo, hi;
        axis_range(p, j, &lo, &hi);
        for (int i = 0; i < m; ++i) {
            double span = hi - lo;
            double t = span * (double)i;
            t = t / (double)(m - 1);
            qa[i] = lo + t;
        }
        for (int i = 0; i < m; ++i) {
            double den = 0.0;
            for (int h = 0; h < m; ++h) {
                double x = (qa[i] - qa[h]) / p->bandwidth[j];
                W[i * m + h] = exp(-0.5 * x * x);
                den += W[i * m + h];
            }
            for (int h = 0; h < m; ++h) W[i * m + h] /= den;
        }
#pragma omp parallel for schedule(static)
        for (int64_t o = 0; o < outer; ++o)
            for (int i = 0; i < m; ++i)
                for (int64_t s = 0; s < inner; ++s) {
                    double acc = 0.0;
                    for (int h = 0; h < m; ++h) acc += W[i * m + h] * a[(o * m + h) * inner + s];
                    b[(o * m + i) * inner + s] = acc;
                }
        double *tmp = a; a = b; b = tmp;
        free(W);
        free(qa);
    }
    memcpy(out, a, sizeof(double) * (size_t)G);
    free(a);
    free(b);
}

/* Index of the largest value; ties go to the lowest index (the best point on
 * the smoothed surface, Sec. 2.3). */
int64_t or_argmax(int64_t n, const double *v)
{
    int64_t best = 0;
    for (int64_t i = 1; i < n; ++i)
        if (v[i] > v[best]) best = i;
    return best;
}

/* ======================================================================== */
/* Gradient: forward-mode derivatives on the same draws                     */
/* ======================================================================== */

typedef struct {
    double dr[6];     /* d r / d q_j     */
    double drho[6];   /* d sqrt(r)/d q_j */
    double dz1[6], dz2[6];
} design_tangent;

/* d r / d q_j for the subgroup fraction, and the implicit derivative of the
 * common critical value through Formula 2:
 *   dz/drho = -phi_2(z,z;rho) / (2 phi(z) Phi(z sqrt((1-rho)/(1+rho)))). */
static void design_derivs(const or_problem *p, const or_design *ds, design_tangent *t)
{
    memset(t, 0, sizeof *t);
    int d = p->d;
    for (int j = 0; j < d; ++j) {
        if (d == 1) {
            t->dr[j] = -1.0;
        } else {
            orth_ctx o;
            memset(&o, 0, sizeof o);
            o.d = d;
            for (int l = 0; l < d; ++l) { o.c[l] = ds->c[l]; o.kind[l] = FK_CUT; }
            o.kind[j] = FK_DENS;
            double I = orth_integral(&o, p->rho_b);
            t->dr[j] = -I / sqrt(1.0 - p->rho_b) / or_phi(ds->c[j]);
        }
        t->drho[j] = t->dr[j] / (2.0 * ds->rho);
    }
    if (p->alpha_rule == OR_ALPHA_FWER_EQUAL) {
        double z = ds->z1, rho = ds->rho;
        double dzdrho = -or_bvn_density(z, z, rho) /
                        (2.0 * or_phi(z) * or_Phi(z * sqrt((1.0 - rho) / (1.0 + rho))));
        for (int j = 0; j < d; ++j) t->dz1[j] = t->dz2[j] = dzdrho * t->drho[j];
    }
}

/* d O / d q_j for one draw. */
static void overlap_derivs(const or_problem *p, const or_design *ds, const or_draw *dr,
                           double *dO)
{
    int d = p->d;
    double w = p->width;
    if (d == 1) {
        double q = ds->q[0], tau = dr->tau[0];
        if (w > 0.0) {
            double s = logistic((q - tau) / w);
            double sp = s * (1.0 - s) / w;
            dO[0] = -(s + sp * (q - tau));
        } else {
            dO[0] = (q > tau) ? -1.0 : 0.0;
        }
        return;
    }
    double isq = 1.0 / sqrt(1.0 - p->rho_b);
    for (int j = 0; j < d; ++j) {
        orth_ctx o;
        memset(&o, 0, sizeof o);
        o.d = d;
        if (w > 0.0) {
            double s[6];
            for (int l = 0; l < d; ++l) {
                s[l] = logistic((ds->q[l] - dr->tau[l]) / w);
                o.kind[l] = FK_MIX; o.c[l] = ds->c[l]; o.t[l] = dr->t[l]; o.s[l] = s[l];
            }
            /* d/dq_j of [s Phi(a) + (1-s) Phi(b)] = s' (Phi(a) - Phi(b))
             *   + s phi(a) (-1/sqrt(1-rho_b)) (1/phi(c_j)). */
            double sp = s[j] * (1.0 - s[j]) / w;
            o.kind[j] = FK_DMIX;
            double Ia = orth_integral(&o, p->rho_b);
            o.kind[j] = FK_DENS;
            double Ib = orth_integral(&o, p->rho_b);
            dO[j] = sp * Ia - s[j] * Ib * isq / or_phi(ds->c[j]);
        } else {
            int flag = ds->q[j] > dr->tau[j];
            if (!flag) { dO[j] = 0.0; continue; }
            for (int l = 0; l < d; ++l) {
                o.kind[l] = FK_CUT;
                o.c[l] = (ds->q[l] > dr->tau[l]) ? ds->c[l] : dr->t[l];
            }
            o.kind[j] = FK_DENS;
            double I = orth_integral(&o, p->rho_b);
            dO[j] = -I * isq / or_phi(ds->c[j]);
        }
    }
}

void or_grad_points(const or_problem *p, int64_t n, const double *q,
                    uint64_t k0, uint64_t M, double *obj,
                    double *grad_q, double *grad_mu)
{
    int d = p->d;
    int nv = d + 3;                       /* value, d design partials, two mu partials */
    or_draw *dr = make_draws(p, k0, M);
    double *vals = (double *)malloc(sizeof(double) * (size_t)M * nv);
    double *col = (double *)malloc(sizeof(double) * (size_t)M);
    if (!dr || !vals || !col) { free(dr); free(vals); free(col); return; }
    double sI = sqrt(p->info);
    for (int64_t i = 0; i < n; ++i) {
        or_design ds;
        design_tangent tg;
        or_make_design(p, q + i * d, &ds);
        design_derivs(p, &ds, &tg);
        double r = ds.r, sr = sqrt(r), srI = sqrt(r * p->info);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < (int64_t)M; ++k) {
            const or_draw *w = &dr[k];
            double d1, d2, O, dO[6];
            effects(p, &ds, w, &d1, &d2, &O);
            overlap_derivs(p, &ds, w, dO);
            double h = ds.z1 - sI * d1, kk = ds.z2 - srI * d2, rho = ds.rho;
            double pv = or_bvn(h, kk, rho);
            double om = sqrt((1.0 - rho) * (1.0 + rho));
            double ph, pk, pr;
            if (kk == INFINITY) { ph = or_phi(h); pk = 0.0; pr = 0.0; }
            else if (h == INFINITY) { ph = 0.0; pk = or_phi(kk); pr = 0.0; }
            else {
                ph = or_phi(h) * or_Phi((kk - rho * h) / om);
                pk = or_phi(kk) * or_Phi((h - rho * kk) / om);
                pr = or_bvn_density(h, kk, rho);
            }
            double *v = vals + (size_t)k * nv;
            v[0] = 1.0 - pv;
            for (int j = 0; j < d; ++j) {
                double drj = tg.dr[j];
                double dmu2 = sI * (w->b0 * drj / (2.0 * sr) +
                                    w->b1 * (dO[j] / sr - O * drj / (2.0 * r * sr)));
                double dh = tg.dz1[j];
                double dk = tg.dz2[j] - dmu2;
                v[1 + j] = -(ph * dh + pk * dk + pr * tg.drho[j]);
            }
            v[1 + d] = -(ph * (-sI) + pk * (-srI));
            v[2 + d] = -(ph * (-sI * w->PR) + pk * (-srI * O / r));
        }
        for (int c = 0; c < nv; ++c) {
            for (int64_t k = 0; k < (int64_t)M; ++k) col[k] = vals[(size_t)k * nv + c];
            double m;
            mean_var(col, (int64_t)M, &m, NULL);
            if (c == 0) obj[i] = m;
            else if (c <= d) grad_q[i * d + (c - 1)] = m;
            else grad_mu[i * 2 + (c - 1 - d)] = m;
        }
    }
    free(col);
    free(vals);
    free(dr);
}

/* ======================================================================== */
/* Exact expectations                                                       */
/* ======================================================================== */
/*
 * Step prior: given the true cutoffs tau, (Delta_1, Delta_2) is a linear map
 * A(tau) of the Gaussian (b0, b1), so the two Z-statistics are jointly normal
 * with mean S A mu_b and covariance Sigma_Z + S A Sigma_b A' S, S =
 * diag(sqrt(I), sqrt(r I)).  The conditional failure probability is then one
 * bivariate normal CDF, and the expected power integrates it over the uniform
 * prior of tau, split where tau_j crosses q_j (the kink of max(c_j, t_j)).
 */
static double cond_fail(const or_problem *p, const or_design *ds, const double *tau)
{
    int d = p->d;
    or_draw dr;
    memset(&dr, 0, sizeof dr);
    for (int j = 0; j < d; ++j) { dr.tau[j] = tau[j]; dr.t[j] = or_Phiinv(tau[j]); }
    dr.PR = (d == 1) ? 1.0 - tau[0] : or_orthant(d, dr.t, p->rho_b);
    double O = or_overlap(p, ds, &dr);
    double r = ds->r, I = p->info;
    double a1 = dr.PR, a2 = O / r;           /* rows (1, a1) and (1, a2) of A */
    double m1 = sqrt(I) * (p->mu_b0 + p->mu_b1 * a1);
    double m2 = sqrt(r * I) * (p->mu_b0 + p->mu_b1 * a2);
    double v0 = p->sd_b0 * p->sd_b0, v1 = p->sd_b1 * p->sd_b1;
    double V11 = 1.0 + I * (v0 + v1 * a1 * a1);
    double V22 = 1.0 + r * I * (v0 + v1 * a2 * a2);
    double V12 = sqrt(r) + sqrt(I) * sqrt(r * I) * (v0 + v1 * a1 * a2);
    double s1 = sqrt(V11), s2 = sqrt(V22);
    return or_bvn((ds->z1 - m1) / s1, (ds->z2 - m2) / s2, V12 / (s1 * s2));
}

typedef struct {
    const or_problem *p;
    const or_design *ds;
    double tau[2];
    int axis;
} exact_ctx;

static double exact_integrand(double x, void *v);

/* Integral over tau_axis..tau_{d-1} of cond_fail, with earlier taus fixed. */
static double exact_level(exact_ctx *e)
{
    const or_problem *p = e->p;
    double lo = p->tau_lo, hi = p->tau_hi;
    if (hi <= lo) {
        e->tau[e->axis] = lo;
        if (e->axis + 1 == p->d) return cond_fail(p, e->ds, e->tau);
        exact_ctx in = *e;
        in.axis = e->axis + 1;
        return exact_level(&in);
    }
    double s = e->ds->q[e->axis];
    if (s < lo) s = lo;
    if (s > hi) s = hi;
    double tot = 0.0;
    if (s > lo) tot += or_quad(exact_integrand, e, lo, s);
    if (hi > s) tot += or_quad(exact_integrand, e, s, hi);
    return tot / (hi - lo);
}

static double exact_integrand(double x, void *v)
{
    exact_ctx *e = (exact_ctx *)v;
    exact_ctx in = *e;
    in.tau[e->axis] = x;
    if (e->axis + 1 == e->p->d) return cond_fail(e->p, e->ds, in.tau);
    in.axis = e->axis + 1;
    return exact_level(&in);
}

double or_exact_step(const or_problem *p, const double *q)
{
    if (p->d > 2 || p->effect != OR_EFFECT_STEP) return NAN;
    or_design ds;
    or_make_design(p, q, &ds);
    exact_ctx e = {p, &ds, {0.0, 0.0}, 0};
    return 1.0 - exact_level(&e);
}

/* Paper prior (Formula 10) on the two nested populations: Delta ~
 * N(theta, Sigma_p) with theta_i = -log(1 - D0(r_i)), sigma_i = 1/sqrt(E r_i/4)
 * and correlation sqrt(r_2/r_1); then X ~ N(D theta, Sigma_Z + D Sigma_p D). */
double or_exact_paper(const or_problem *p, const double *q)
{
    if (p->effect != OR_EFFECT_PAPER_GAUSS) return NAN;
    or_design ds;
    or_make_design(p, q, &ds);
    if (p->design_space == OR_DESIGN_ALPHA4) {
        /* as for three populations: covariance (1 + 4 I / E) R */
        if (isnan(ds.z4)) return NAN;
        double r[4] = {1.0, ds.r, ds.r3, ds.r4}, z[4] = {ds.z1, ds.z2, ds.z3, ds.z4}, h[4];
        double s = sqrt(1.0 + 4.0 * p->info / p->paper_events);
        for (int i = 0; i < 4; ++i) {
            double th = -log1p(-(p->paper_a - p->paper_b * r[i]));
            h[i] = (z[i] - sqrt(r[i] * p->info) * th) / s;
        }
        return 1.0 - or_qvn_nested(h, r);
    }
    if (p->design_space == OR_DESIGN_ALPHA3) {
        /* X = D Delta + eps is Gaussian with covariance (1 + 4 I / E) R. */
        if (isnan(ds.z3)) return NAN;
        double r[3] = {1.0, ds.r, ds.r3}, z[3] = {ds.z1, ds.z2, ds.z3}, h[3];
        double s = sqrt(1.0 + 4.0 * p->info / p->paper_events);
        for (int i = 0; i < 3; ++i) {
            double th = -log1p(-(p->paper_a - p->paper_b * r[i]));
            h[i] = (z[i] - sqrt(r[i] * p->info) * th) / s;
        }
        return 1.0 - or_tvn(h[0], h[1], h[2], sqrt(r[1]), sqrt(r[2]), sqrt(r[2] / r[1]));
    }
    double r = ds.r, I = p->info, E = p->paper_events;
    double th1 = -log1p(-(p->paper_a - p->paper_b));
    double th2 = -log1p(-(p->paper_a - p->paper_b * r));
    double sg1 = 1.0 / sqrt(E / 4.0), sg2 = 1.0 / sqrt(E * r / 4.0);
    double m1 = sqrt(I) * th1, m2 = sqrt(r * I) * th2;
    double V11 = 1.0 + I * sg1 * sg1;
    double V22 = 1.0 + r * I * sg2 * sg2;
    double V12 = sqrt(r) + sqrt(I) * sqrt(r * I) * sqrt(r) * sg1 * sg2;
    double s1 = sqrt(V11), s2 = sqrt(V22);
    return 1.0 - or_bvn((ds.z1 - m1) / s1, (ds.z2 - m2) / s2, V12 / (s1 * s2));
}

/* Threads the OpenMP loops of this library run with (for reporting). */
int or_num_threads(void) { return omp_get_max_threads(); }
