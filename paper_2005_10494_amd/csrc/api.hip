// C ABI of libbmd: argument validation, problem construction, workspace
// management and the launch sequence of each entry point (see include/bmd.h).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bmd_internal.hpp"

namespace bmd {
// Smoothing over the designs whose value is not NaN (kernels_post.hip); NaN
// designs stay NaN; ws holds 4 G doubles.
hipError_t launch_smooth_masked(const bmd_problem* p, int prec, const double* in, double* out, double* ws,
                                hipStream_t s);
// One step of the per-design golden-section level search (kernels_setup.hip):
// st [8][G] search state, side [G]; writes the problem's z1, z2 when probing
// (end: 0 the next golden point, 1 the range's lower end, 2 its upper end).
hipError_t launch_levels_golden(const bmd_problem* p, int phase, bool probe, int end, double a_lo, double a_hi,
                                const double* mean, double* st, int32_t* side, hipStream_t s);
// One step of the derivative-driven level search (kernels_setup.hip): st
// [9][G] search state; writes the problem's z1, z2 for the next probe.
hipError_t launch_levels_newton(const bmd_problem* p, int phase, double a_lo, double a_hi, double tol,
                                const double* mean, const double* dmean, double* st, hipStream_t s);
}  // namespace bmd

using namespace bmd;

// Fixed device workspace of bmd_eval_grid_noalloc: the draw arrays and the
// per-slice partial sums of one sweep.  Each device holds its own copy for the
// life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_ptr), never by name.
static __device__ __align__(256) char scratch[BMD_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Look up this device's copy of `scratch` once (the device must be current).
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

bmd_status fail(bmd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

bmd_status hip_fail(hipError_t e, const char* what) {
    return fail(BMD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Keeps the caller's current device, switching to the problem's for the call.
struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) == hipSuccess && old != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

bool finite(double x) { return std::isfinite(x); }

double host_Phi(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Standard normal quantile on the host: bisection in the tails' bracket, then
// Newton polishing on erfc.
double host_quantile(double p) {
    if (p <= 0.0) return -INFINITY;
    if (p >= 1.0) return INFINITY;
    if (p > 0.5) return -host_quantile(1.0 - p);
    double lo = -40.0, hi = 0.0;
    for (int it = 0; it < 80; ++it) {
        double mid = 0.5 * (lo + hi);
        if (host_Phi(mid) < p) lo = mid; else hi = mid;
    }
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 3; ++it) {
        double dens = std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI);
        if (dens <= 0.0) break;
        x -= (host_Phi(x) - p) / dens;
    }
    return x;
}

double host_grid(double q_lo, double q_hi, int64_t i, int m) {
    double span = q_hi - q_lo;
    double t = span * static_cast<double>(i);
    t = t / static_cast<double>(m - 1);
    return q_lo + t;
}

// Orthant P(X_j > v_j) by the one-factor Gauss-Hermite rule (x[0..K), w[0..K)).
double host_orthant(const std::vector<double>& v, double rho, const double* x, const double* w, int K) {
    const double sr = std::sqrt(rho), sq = std::sqrt(1.0 - rho);
    double acc = 0.0;
    for (int m = 0; m < K; ++m) {
        double prod = w[m];
        for (double vj : v) prod *= host_Phi((sr * x[m] - vj) / sq);
        acc += prod;
    }
    return acc;
}

// Smallest Gauss-Hermite rule whose orthant probabilities match a 128-node
// reference to `target` relative error at probe points spanning the cutoffs
// the problem can produce (design cutoffs and drawn responder cutoffs).
int choose_gh(const bmd_problem_desc& d, double target) {
    if (d.d == 1 || d.design_space != BMD_DESIGN_CUTOFFS) return 4;   // closed forms; tables unused
    static const int cand[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128};
    std::vector<double> xr(128), wr(128);
    gauss_hermite_prob(128, xr.data(), wr.data());
    double lo_q = d.q_lo, hi_q = d.q_hi;
    if (d.effect == BMD_EFFECT_STEP) {
        lo_q = std::min(lo_q, d.tau_lo);
        hi_q = std::max(hi_q, d.tau_hi);
    }
    const double vlo = host_quantile(lo_q), vhi = host_quantile(hi_q);
    std::vector<std::vector<double>> probes;
    for (int s = 0; s <= 4; ++s) probes.push_back(std::vector<double>(d.d, vlo + (vhi - vlo) * s / 4.0));
    std::vector<double> mix(d.d);
    for (int j = 0; j < d.d; ++j) mix[j] = (j % 2) ? vlo : vhi;
    probes.push_back(mix);
    std::vector<double> ref;
    for (auto& v : probes) ref.push_back(host_orthant(v, d.rho_b, xr.data(), wr.data(), 128));
    for (int K : cand) {
        std::vector<double> x(K), w(K);
        gauss_hermite_prob(K, x.data(), w.data());
        double err = 0.0;
        for (size_t i = 0; i < probes.size(); ++i)
            err = std::max(err, std::fabs(host_orthant(probes[i], d.rho_b, x.data(), w.data(), K) - ref[i]) / ref[i]);
        if (err <= target) return K;
    }
    return 128;
}

bmd_status validate(const bmd_problem_desc* d, bool* grid) {
    if (!d) return fail(BMD_EINVAL, "desc is NULL");
    if (d->d < 1 || d->d > BMD_MAX_DIM) return fail(BMD_ERANGE, "d = %d outside 1..6", d->d);
    bool any = false, all = true;
    for (int j = 0; j < d->d; ++j) {
        if (d->m[j] != 0) any = true;
        if (d->m[j] < 2) all = false;
    }
    if (any && !all) return fail(BMD_ERANGE, "grid needs m_j >= 2 on every axis (or all zero)");
    *grid = any;
    if (any) {
        double G = 1.0;
        for (int j = 0; j < d->d; ++j) {
            if (d->m[j] > 100000) return fail(BMD_ERANGE, "m_%d = %d too large", j, d->m[j]);
            G *= d->m[j];
        }
        if (G > 2e9) return fail(BMD_ERANGE, "grid of %.3g designs exceeds 2e9", G);
        for (int j = 0; j < d->d; ++j)
            if (!finite(d->bandwidth[j]) || d->bandwidth[j] <= 0.0)
                return fail(BMD_ERANGE, "bandwidth_%d must be > 0", j);
    }
    if (!finite(d->q_lo) || !finite(d->q_hi) || !(0.0 < d->q_lo && d->q_lo < d->q_hi && d->q_hi < 1.0))
        return fail(BMD_ERANGE, "need 0 < q_lo < q_hi < 1");
    if (!finite(d->rho_b) || d->rho_b < 0.0 || d->rho_b > 0.5)
        return fail(BMD_ERANGE, "rho_b = %g outside [0, 0.5]", d->rho_b);
    if (!finite(d->info) || d->info <= 0.0) return fail(BMD_ERANGE, "info must be > 0");
    if (!finite(d->alpha0) || !(d->alpha0 > 0.0 && d->alpha0 < 0.5)) return fail(BMD_ERANGE, "alpha0 outside (0, 0.5)");
    if (d->alpha_rule < 0 || d->alpha_rule > 3) return fail(BMD_EINVAL, "unknown alpha_rule %d", d->alpha_rule);
    if (d->alpha_rule == BMD_ALPHA_SPLIT &&
        !(finite(d->alpha_fixed[0]) && d->alpha_fixed[0] > 0.0 && d->alpha_fixed[0] < d->alpha0))
        return fail(BMD_ERANGE, "the split rule needs 0 < alpha_fixed[0] < alpha0");
    if (d->alpha_rule == BMD_ALPHA_FIXED)
        for (int i = 0; i < 2; ++i)
            if (!finite(d->alpha_fixed[i]) || d->alpha_fixed[i] < 0.0 || d->alpha_fixed[i] >= 0.5)
                return fail(BMD_ERANGE, "alpha_fixed[%d] outside [0, 0.5)", i);
    if (d->effect == BMD_EFFECT_STEP) {
        const double v[] = {d->mu_b0, d->sd_b0, d->mu_b1, d->sd_b1, d->tau_lo, d->tau_hi};
        for (double x : v)
            if (!finite(x)) return fail(BMD_EINVAL, "non-finite prior parameter");
        if (d->sd_b0 < 0.0 || d->sd_b1 < 0.0) return fail(BMD_ERANGE, "prior sd must be >= 0");
        if (!(0.0 < d->tau_lo && d->tau_lo <= d->tau_hi && d->tau_hi < 1.0))
            return fail(BMD_ERANGE, "need 0 < tau_lo <= tau_hi < 1");
    } else if (d->effect == BMD_EFFECT_PAPER_GAUSS) {
        if (!finite(d->paper_a) || !finite(d->paper_b) || !finite(d->paper_events) || d->paper_events <= 0.0)
            return fail(BMD_ERANGE, "paper prior needs finite a, b and events > 0");
        if (!(d->paper_a < 1.0 && d->paper_a - d->paper_b < 1.0))
            return fail(BMD_ERANGE, "paper prior effect a - b r must stay below 1");
    } else {
        return fail(BMD_EINVAL, "unknown effect model %d", d->effect);
    }
    if (!finite(d->indicator_width) || d->indicator_width < 0.0) return fail(BMD_ERANGE, "indicator_width must be >= 0");
    if (d->gh_nodes != 0 && (d->gh_nodes < 4 || d->gh_nodes > kMaxGH || d->gh_nodes % 4 != 0))
        return fail(BMD_ERANGE, "gh_nodes must be 0 or a multiple of 4 in [4, 128]");
    if (d->design_space == BMD_DESIGN_ALPHA) {
        if (d->effect != BMD_EFFECT_PAPER_GAUSS || d->alpha_rule != BMD_ALPHA_FWER_EQUAL)
            return fail(BMD_EINVAL, "alpha designs need the Formula 10 prior and the FWER-boundary rule");
        if (!any || d->d > 2) return fail(BMD_ERANGE, "alpha designs are a grid over alpha_1 or (r_2, alpha_1)");
        if (!(d->q_hi < d->alpha0)) return fail(BMD_ERANGE, "alpha_1 range must lie inside (0, alpha0)");
        if (!finite(d->r_lo) || !finite(d->r_hi) || !(d->r_lo > 0.0 && d->r_hi <= 0.95) ||
            (d->d == 2 && !(d->r_lo < d->r_hi)))
            return fail(BMD_ERANGE, "need 0 < r_lo %s r_hi <= 0.95", d->d == 2 ? "<" : "and");
    } else if (d->design_space == BMD_DESIGN_ALPHA3) {
        if (d->effect != BMD_EFFECT_PAPER_GAUSS || d->alpha_rule != BMD_ALPHA_FWER_EQUAL)
            return fail(BMD_EINVAL, "alpha designs need the Formula 10 prior and the FWER-boundary rule");
        if (!any || d->d != 2) return fail(BMD_ERANGE, "three-population designs are a grid over (alpha_1, alpha_2)");
        if (!(d->q_hi < d->alpha0)) return fail(BMD_ERANGE, "alpha_1 and alpha_2 ranges must lie inside (0, alpha0)");
        if (!finite(d->r_lo) || !finite(d->r_hi) || !(0.0 < d->r_hi && d->r_hi < d->r_lo && d->r_lo <= 0.9))
            return fail(BMD_ERANGE, "need 0 < r_3 = r_hi < r_2 = r_lo <= 0.9");
        if (d->r_hi * (1.0 - d->r_lo) > 0.975 * 0.975 * d->r_lo * (1.0 - d->r_hi))
            return fail(BMD_ERANGE, "partial correlation of the third on the second population exceeds 0.975");
    } else if (d->design_space == BMD_DESIGN_ALPHA4) {
        if (d->effect != BMD_EFFECT_PAPER_GAUSS || d->alpha_rule != BMD_ALPHA_FWER_EQUAL)
            return fail(BMD_EINVAL, "alpha designs need the Formula 10 prior and the FWER-boundary rule");
        if (!any || d->d != 3)
            return fail(BMD_ERANGE, "four-population designs are a grid over (alpha_1, alpha_2, alpha_3)");
        if (!(d->q_hi < d->alpha0)) return fail(BMD_ERANGE, "level ranges must lie inside (0, alpha0)");
        const double r2 = d->r_lo, r3 = d->r_hi, r4 = d->r_4;
        if (!finite(r2) || !finite(r3) || !finite(r4) || !(0.0 < r4 && r4 < r3 && r3 < r2 && r2 <= 0.9))
            return fail(BMD_ERANGE, "need 0 < r_4 < r_3 = r_hi < r_2 = r_lo <= 0.9");
        // the first three levels use the three-population rule; the
        // bivariate part of Phi_4 needs a correlation inside its node table,
        // and r_3 / r_2, r_4 / r_2 bound the panel count
        if (r3 * (1.0 - r2) > 0.975 * 0.975 * r2 * (1.0 - r3))
            return fail(BMD_ERANGE, "partial correlation of the third on the second population exceeds 0.975");
        if (r4 * (r2 - r3) > 0.975 * 0.975 * r3 * (r2 - r4))
            return fail(BMD_ERANGE, "partial correlation of the fourth and third populations given the second "
                                    "exceeds 0.975");
        if (r3 > 0.95 * r2) return fail(BMD_ERANGE, "need r_3 <= 0.95 r_2");
    } else if (d->design_space == BMD_DESIGN_NESTED3) {
        if (d->effect != BMD_EFFECT_STEP)
            return fail(BMD_EINVAL, "two-cutoff designs need the step prior (one biomarker)");
        if (d->alpha_rule != BMD_ALPHA_FWER_EQUAL && d->alpha_rule != BMD_ALPHA_BONFERRONI)
            return fail(BMD_EINVAL, "two-cutoff designs need rule FWER_EQUAL or BONFERRONI");
        if (!any || d->d != 2) return fail(BMD_ERANGE, "two-cutoff designs are a grid over (q_1, q_2)");
        if (!(d->q_lo >= 0.1 && d->q_hi < 1.0))
            return fail(BMD_ERANGE, "two-cutoff designs need 0.1 <= q_lo and q_hi < 1 (r_2 <= 0.9)");
        if (d->indicator_width != 0.0) return fail(BMD_ERANGE, "two-cutoff designs use the exact indicator");
        if (static_cast<double>(d->m[0]) * d->m[1] > static_cast<double>(kNested3MaxTiles * kEvalBlock))
            return fail(BMD_ERANGE, "two-cutoff grids hold at most %lld designs",
                        static_cast<long long>(kNested3MaxTiles * kEvalBlock));
    } else if (d->design_space == BMD_DESIGN_NESTED4) {
        if (d->effect != BMD_EFFECT_STEP)
            return fail(BMD_EINVAL, "three-cutoff designs need the step prior (one biomarker)");
        if (d->alpha_rule != BMD_ALPHA_FWER_EQUAL && d->alpha_rule != BMD_ALPHA_BONFERRONI)
            return fail(BMD_EINVAL, "three-cutoff designs need rule FWER_EQUAL or BONFERRONI");
        if (!any || d->d != 3) return fail(BMD_ERANGE, "three-cutoff designs are a grid over (q_1, q_2, q_3)");
        if (!(d->q_lo >= 0.1 && d->q_hi < 1.0))
            return fail(BMD_ERANGE, "three-cutoff designs need 0.1 <= q_lo and q_hi < 1 (r_2 <= 0.9)");
        if (d->indicator_width != 0.0) return fail(BMD_ERANGE, "three-cutoff designs use the exact indicator");
        if (static_cast<double>(d->m[0]) * d->m[1] * d->m[2] > static_cast<double>(kNested3MaxTiles * kEvalBlock))
            return fail(BMD_ERANGE, "three-cutoff grids hold at most %lld designs",
                        static_cast<long long>(kNested3MaxTiles * kEvalBlock));
    } else if (d->design_space != BMD_DESIGN_CUTOFFS) {
        return fail(BMD_EINVAL, "unknown design_space %d", d->design_space);
    }
    return BMD_OK;
}

// Coordinate range of grid axis j (host copy of the device rule).
void axis_range(const bmd_problem_desc& d, int j, double* lo, double* hi) {
    if (d.design_space == BMD_DESIGN_ALPHA && d.d == 2 && j == 0) {
        *lo = d.r_lo;
        *hi = d.r_hi;
    } else {
        *lo = d.q_lo;
        *hi = d.q_hi;
    }
}

bmd_status ensure(void** buf, size_t* cap, size_t need) {
    if (*cap >= need && *buf) return BMD_OK;
    if (*buf) {
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    size_t want = std::max<size_t>(need, 1 << 20);
    hipError_t e = hipMalloc(buf, want);
    if (e != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return fail(BMD_ENOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
    }
    *cap = want;
    return BMD_OK;
}

template <typename T>
bmd_status upload(T** dst, const T* src, size_t n) {
    hipError_t e = hipMalloc(dst, sizeof(T) * std::max<size_t>(n, 1));
    if (e != hipSuccess) {
        *dst = nullptr;
        (void)hipGetLastError();
        return fail(BMD_ENOMEM, "device allocation of %zu bytes: %s", sizeof(T) * n, hipGetErrorString(e));
    }
    if (src && n) {
        e = hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    return BMD_OK;
}

void free_problem(bmd_problem* p) {
    if (!p) return;
    auto f = [](void* x) {
        if (x) (void)hipFree(x);
    };
    for (auto& t : p->tab) {
        f(t.gh);
        f(t.A);
        f(t.glw);
    }
    f(p->d_gl);
    f(p->d_ghp);
    f(p->d_r);
    f(p->d_z1);
    f(p->d_z2);
    f(p->d_z3);
    f(p->d_z4);
    f(p->d_order);
    f(p->d_W);
    f(p->d_Wf);
    f(p->d_ws);
    f(p->d_ws2);
    tps_release(p);
    for (auto& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

bool valid_prec(int32_t prec) { return prec == BMD_FP64 || prec == BMD_FP32_COMP; }

// Draw slices of a grid sweep: about kSweepRounds full rounds of resident
// workgroups, so the partly filled last round costs little; slices of at
// least 64 draws, whole draw chunks of the matrix-core sweep, and for that
// sweep no more staged draw bytes per slice than the problem's slice budget.
void sweep_slices(bmd_problem* p, int prec, int64_t M, int64_t* n_slices_out, int64_t* slice_len_out) {
    const int64_t bx = sweep_tiles(p, prec);
    if (p->sweep_bpc[prec] == 0) p->sweep_bpc[prec] = sweep_blocks_per_cu(p, prec);
    const int64_t resident = static_cast<int64_t>(p->n_cu) * p->sweep_bpc[prec];
    const int64_t chunk = sweep_chunk(p, prec);
    int64_t n_slices = (kSweepRounds * resident + bx - 1) / bx;
    const int64_t per_draw = sweep_staged_bytes_per_draw(p, prec);
    if (per_draw > 0 && p->slice_bytes > 0) {
        const int64_t len = std::max<int64_t>(chunk, p->slice_bytes / per_draw / chunk * chunk);
        n_slices = std::max<int64_t>(n_slices, (M + len - 1) / len);
    }
    n_slices = std::max<int64_t>(1, std::min<int64_t>({n_slices, (M + 63) / 64, 65535}));
    int64_t slice_len = (M + n_slices - 1) / n_slices;
    slice_len = (slice_len + chunk - 1) / chunk * chunk;
    *n_slices_out = (M + slice_len - 1) / slice_len;
    *slice_len_out = slice_len;
}

// Event i of the profiling pairs (phase = i / 2), recorded when profiling is on.
void mark(bmd_problem* p, int i, hipStream_t s) {
    if (!p->profiling) return;
    (void)hipEventRecord(p->ev[i], s);
    p->ev_used[i / 2] = true;
}

// The sweep of bmd_eval_grid into workspace ws: draws at ws, per-slice
// partial sums at ws + draw_bytes (every slice writes all its designs, so
// nothing needs clearing first).
bmd_status eval_grid_into(bmd_problem* p, int prec, int64_t M, int64_t n_slices, int64_t slice_len, void* ws,
                          size_t draw_bytes, double* d_mean, double* d_var, hipStream_t s) {
    double* partials = reinterpret_cast<double*>(static_cast<char*>(ws) + draw_bytes);
    mark(p, 0, s);
    HIP_TRY(launch_draws(p, prec, 0, M, ws, s), "draw kernel");
    mark(p, 1, s);
    mark(p, 2, s);
    HIP_TRY(launch_eval_grid(p, prec, M, ws, partials, static_cast<int>(n_slices), slice_len, d_var != nullptr, s),
            "eval kernel");
    mark(p, 3, s);
    mark(p, 4, s);
    HIP_TRY(launch_finalize(p, M, partials, static_cast<int>(n_slices), d_mean, d_var, s), "finalize kernel");
    mark(p, 5, s);
    return BMD_OK;
}

}  // namespace

extern "C" {

int32_t bmd_abi_version(void) { return BMD_ABI_VERSION; }

const char* bmd_last_error(void) { return g_err.c_str(); }

bmd_status bmd_create_problem(const bmd_problem_desc* desc, bmd_problem** out, void* stream) {
    g_err.clear();
    if (!out) return fail(BMD_EINVAL, "out is NULL");
    *out = nullptr;
    bool grid = false;
    bmd_status st = validate(desc, &grid);
    if (st != BMD_OK) return st;
    const bmd_problem_desc& d = *desc;

    // Subgroup fractions above 0.95 would need correlations beyond the
    // bivariate quadrature's supported range (sqrt(r) <= 0.975).
    std::vector<double> ghx(kPrecomputeGH), ghw(kPrecomputeGH);
    gauss_hermite_prob(kPrecomputeGH, ghx.data(), ghw.data());
    if (d.design_space == BMD_DESIGN_CUTOFFS) {
        double rmax;
        if (d.d == 1) rmax = 1.0 - d.q_lo;
        else rmax = host_orthant(std::vector<double>(d.d, host_quantile(d.q_lo)), d.rho_b, ghx.data(), ghw.data(),
                                 kPrecomputeGH);
        if (rmax > 0.95 + 1e-12)
            return fail(BMD_ERANGE, "subgroup fraction reaches %.6f > 0.95 at q_lo = %g", rmax, d.q_lo);
    }

    bmd_problem* p = new bmd_problem();
    p->desc = d;
    p->grid = grid;
    (void)hipGetDevice(&p->device);
    if (hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        p->n_cu < 1) {
        (void)hipGetLastError();
        p->n_cu = 1;
    }
    // set-up of the no-allocation sweep: this device's scratch address
    if (const hipError_t e = scratch_setup(p->device); e != hipSuccess) {
        delete p;
        (void)hipGetLastError();
        return hip_fail(e, "scratch address (hipGetSymbolAddress)");
    }
    DevProblem& P = p->P;
    std::memset(&P, 0, sizeof P);
    P.d = d.d;
    P.G = 0;
    P.mmax = 1;
    if (grid) {
        P.G = 1;
        for (int j = 0; j < d.d; ++j) {
            P.m[j] = d.m[j];
            P.G *= d.m[j];
            P.mmax = std::max(P.mmax, d.m[j]);
        }
        int64_t s = 1;
        for (int j = d.d - 1; j >= 0; --j) {
            P.stride[j] = s;
            s *= d.m[j];
        }
    }
    P.q_lo = d.q_lo;
    P.q_hi = d.q_hi;
    P.design_space = d.design_space;
    P.r_lo = d.r_lo;
    P.r_hi = d.r_hi;
    P.rho_b = d.rho_b;
    P.sr = std::sqrt(d.rho_b);
    P.sq = std::sqrt(1.0 - d.rho_b);
    P.info = d.info;
    P.sqrtI = std::sqrt(d.info);
    P.alpha0 = d.alpha0;
    P.alpha_rule = d.alpha_rule;
    if (d.alpha_rule == BMD_ALPHA_BONFERRONI) {
        P.zf1 = P.zf2 = -host_quantile(0.5 * d.alpha0);
    } else if (d.alpha_rule == BMD_ALPHA_SPLIT) {
        P.zf1 = -host_quantile(d.alpha_fixed[0]);   // z2 per design on the FWER boundary
    } else if (d.alpha_rule == BMD_ALPHA_FIXED) {
        P.zf1 = d.alpha_fixed[0] > 0.0 ? -host_quantile(d.alpha_fixed[0]) : INFINITY;
        P.zf2 = d.alpha_fixed[1] > 0.0 ? -host_quantile(d.alpha_fixed[1]) : INFINITY;
        P.zinf = (std::isinf(P.zf1) ? 1 : 0) | (std::isinf(P.zf2) ? 2 : 0);
    }
    P.effect = d.effect;
    P.mu_b0 = d.mu_b0;
    P.sd_b0 = d.sd_b0;
    P.mu_b1 = d.mu_b1;
    P.sd_b1 = d.sd_b1;
    P.tau_lo = d.tau_lo;
    P.tau_hi = d.tau_hi;
    P.paper_a = d.paper_a;
    P.paper_b = d.paper_b;
    P.paper_events = d.paper_events;
    if (d.effect == BMD_EFFECT_PAPER_GAUSS) {
        P.th1 = -std::log1p(-(d.paper_a - d.paper_b));
        P.sg1 = 1.0 / std::sqrt(d.paper_events / 4.0);
    }
    P.width = d.indicator_width;
    P.key0 = static_cast<uint32_t>(d.seed);
    P.key1 = static_cast<uint32_t>(d.seed >> 32);
    P.scenario = d.scenario_id;
    P.n_uniform = (d.design_space == BMD_DESIGN_NESTED3 || d.design_space == BMD_DESIGN_NESTED4) ? 3
                  : d.effect == BMD_EFFECT_STEP              ? 2 + d.d
                  : d.design_space == BMD_DESIGN_ALPHA3 ? 3
                  : d.design_space == BMD_DESIGN_ALPHA4 ? 4
                                                        : 2;
    P.r_4 = d.r_4;
    {
        // BMD_SWEEP=direct selects the direct (vector-unit) sweep for every grid
        // problem; both sweeps compute the same estimate (used by the tests).
        const char* sw = std::getenv("BMD_SWEEP");
        p->force_direct = sw && std::strcmp(sw, "direct") == 0;
        // BMD_SLICE_BYTES overrides the staged-draw budget of a sweep slice
        // (bytes, 0 = no limit; for measurements)
        if (const char* sb = std::getenv("BMD_SLICE_BYTES")) p->slice_bytes = std::max<int64_t>(0, std::atoll(sb));
    }

    // Quadrature rules.
    std::vector<double> gl(kGLTable);
    gl_table(gl.data());
    std::vector<float> glf(gl.begin(), gl.end());
    const int K64 = d.gh_nodes ? d.gh_nodes : choose_gh(d, 1e-13);
    const int K32 = d.gh_nodes ? d.gh_nodes : choose_gh(d, 3e-8);
    const int Ks[2] = {K64, K32};
    std::vector<double> ghp(2 * kPrecomputeGH);
    std::copy(ghx.begin(), ghx.end(), ghp.begin());
    std::copy(ghw.begin(), ghw.end(), ghp.begin() + kPrecomputeGH);

    st = upload(&p->d_gl, gl.data(), gl.size());
    if (st == BMD_OK) st = upload(&p->d_ghp, ghp.data(), ghp.size());
    for (int prec = 0; prec < 2 && st == BMD_OK; ++prec) {
        const int K = Ks[prec];
        std::vector<double> x(K), w(K);
        gauss_hermite_prob(K, x.data(), w.data());
        std::vector<double>& gh = p->gh_host[prec];
        gh.assign(2 * K, 0.0);
        std::copy(x.begin(), x.end(), gh.begin());
        std::copy(w.begin(), w.end(), gh.begin() + K);
        p->tab[prec].K = K;
        st = upload(&p->tab[prec].gh, gh.data(), gh.size());
        if (st != BMD_OK) break;
        if (prec == BMD_FP64) {
            double* g = nullptr;
            st = upload(&g, gl.data(), gl.size());
            p->tab[prec].glw = g;
        } else {
            float* g = nullptr;
            st = upload(&g, glf.data(), glf.size());
            p->tab[prec].glw = g;
        }
        if (st != BMD_OK) break;
        if (grid) {
            const size_t n = static_cast<size_t>(d.d) * K * P.mmax;
            if (prec == BMD_FP64) {
                double* a = nullptr;
                st = upload<double>(&a, nullptr, n);
                p->tab[prec].A = a;
            } else {
                float* a = nullptr;
                st = upload<float>(&a, nullptr, n);
                p->tab[prec].A = a;
            }
        }
    }
    if (st == BMD_OK && grid) {
        st = upload<double>(&p->d_r, nullptr, P.G);
        if (st == BMD_OK) st = upload<double>(&p->d_z1, nullptr, P.G);
        if (st == BMD_OK) st = upload<double>(&p->d_z2, nullptr, P.G);
        if (st == BMD_OK && (d.design_space == BMD_DESIGN_ALPHA3 || d.design_space == BMD_DESIGN_ALPHA4 ||
                             d.design_space == BMD_DESIGN_NESTED3 || d.design_space == BMD_DESIGN_NESTED4))
            st = upload<double>(&p->d_z3, nullptr, P.G);
        if (st == BMD_OK && (d.design_space == BMD_DESIGN_ALPHA4 || d.design_space == BMD_DESIGN_NESTED4))
            st = upload<double>(&p->d_z4, nullptr, P.G);
        if (st == BMD_OK) st = upload<int32_t>(&p->d_order, nullptr, P.G);
        // Smoothing matrices.
        std::vector<double> W;
        for (int j = 0; j < d.d && st == BMD_OK; ++j) {
            const int m = d.m[j];
            p->w_off[j] = static_cast<int64_t>(W.size());
            std::vector<double> q(m);
            double lo, hi;
            axis_range(d, j, &lo, &hi);
            for (int i = 0; i < m; ++i) q[i] = host_grid(lo, hi, i, m);
            for (int i = 0; i < m; ++i) {
                double den = 0.0;
                const size_t row = W.size();
                for (int h = 0; h < m; ++h) {
                    const double z = (q[i] - q[h]) / d.bandwidth[j];
                    W.push_back(std::exp(-0.5 * z * z));
                    den += W.back();
                }
                for (int h = 0; h < m; ++h) W[row + h] /= den;
            }
        }
        std::vector<float> Wf(W.begin(), W.end());
        if (st == BMD_OK) st = upload(&p->d_W, W.data(), W.size());
        if (st == BMD_OK) st = upload(&p->d_Wf, Wf.data(), Wf.size());
    }
    if (st != BMD_OK) {
        std::string msg = g_err;
        free_problem(p);
        g_err = msg;
        return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_design_precompute(p, s);
    if (d.design_space == BMD_DESIGN_CUTOFFS) {   // the alpha design space has no cutoff axes
        if (e == hipSuccess) e = launch_axis_tables(p, BMD_FP64, s);
        if (e == hipSuccess) e = launch_axis_tables(p, BMD_FP32_COMP, s);
    }
    if (e != hipSuccess) {
        free_problem(p);
        return hip_fail(e, "setup kernels");
    }
    *out = p;
    return BMD_OK;
}

void bmd_destroy_problem(bmd_problem* p) {
    if (!p) return;
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    free_problem(p);
}

int64_t bmd_grid_size(const bmd_problem* p) { return p ? p->P.G : 0; }

int32_t bmd_gh_nodes(const bmd_problem* p, int32_t prec) {
    if (!p || !valid_prec(prec)) return -1;
    return p->tab[prec].K;
}

int32_t bmd_sweep_kind(const bmd_problem* p) {
    if (!p || !p->grid) return -1;
    return use_mfma_sweep(p) ? BMD_SWEEP_MATRIX : BMD_SWEEP_DIRECT;
}

bmd_status bmd_eval_grid(bmd_problem* p, uint64_t n_draws, int32_t prec, double* d_mean, double* d_var,
                         void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "eval_grid needs a grid problem");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_mean) return fail(BMD_EINVAL, "d_mean is NULL");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    const int64_t G = p->P.G;
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + 255) / 256 * 256;
    const size_t part_bytes = sizeof(double) * 2 * static_cast<size_t>(G) * n_slices;
    bmd_status st = ensure(&p->d_ws, &p->ws_cap, draw_bytes + part_bytes);
    if (st != BMD_OK) return st;
    return eval_grid_into(p, prec, M, n_slices, slice_len, p->d_ws, draw_bytes, d_mean, d_var, s);
}

bmd_status bmd_eval_grid_noalloc(bmd_problem* p, uint64_t n_draws, int32_t prec, double* d_mean, double* d_var,
                                 void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "eval_grid_noalloc needs a grid problem");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_mean) return fail(BMD_EINVAL, "d_mean is NULL");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + 255) / 256 * 256;
    const size_t part_bytes = sizeof(double) * 2 * static_cast<size_t>(p->P.G) * n_slices;
    if (draw_bytes + part_bytes > BMD_NOALLOC_SCRATCH_BYTES)
        return fail(BMD_ERANGE, "workspace of %zu bytes (draws %zu, partial sums %zu) exceeds the %zu-byte scratch",
                    draw_bytes + part_bytes, draw_bytes, part_bytes, static_cast<size_t>(BMD_NOALLOC_SCRATCH_BYTES));
    void* ws = scratch_ptr(p->device);
    if (!ws) return fail(BMD_EDEVICE, "no scratch address for device %d", p->device);
    return eval_grid_into(p, prec, M, n_slices, slice_len, ws, draw_bytes, d_mean, d_var, s);
}

// The level searches write a finite first critical value and a second one on
// the FWER boundary for every probe; their sweeps run under the split rule
// (no test switched off, the derivative's dz2/dz1 term on), and the
// problem's own rule comes back on restore() or at scope exit.  Kernel
// arguments are copied at launch, so restoring after the launches is safe.
struct SplitRuleScope {
    bmd_problem* p;
    int rule, zinf;
    bool on = true;
    explicit SplitRuleScope(bmd_problem* q) : p(q), rule(q->P.alpha_rule), zinf(q->P.zinf) {
        p->P.alpha_rule = BMD_ALPHA_SPLIT;
        p->P.zinf = 0;
    }
    void restore() {
        if (on) {
            p->P.alpha_rule = rule;
            p->P.zinf = zinf;
            on = false;
        }
    }
    ~SplitRuleScope() { restore(); }
};

bmd_status bmd_optimize_levels(bmd_problem* p, uint64_t n_draws, int32_t prec, double a_lo, double a_hi,
                               int32_t n_iter, double* d_best, double* d_alpha1, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ESTATE, "level search needs a grid of cutoff designs");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_best || !d_alpha1) return fail(BMD_EINVAL, "NULL d_best or d_alpha1");
    if (!std::isfinite(a_lo) || !std::isfinite(a_hi) || !(0.0 < a_lo && a_lo < a_hi && a_hi < p->P.alpha0))
        return fail(BMD_ERANGE, "need 0 < a_lo < a_hi < alpha0");
    if (n_iter < 0 || n_iter > 200) return fail(BMD_ERANGE, "n_iter must be in [0, 200]");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    const int64_t G = p->P.G;
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t al = 256;
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + al - 1) / al * al;
    const size_t part_bytes = (sizeof(double) * 2 * static_cast<size_t>(G) * n_slices + al - 1) / al * al;
    const size_t mean_bytes = (sizeof(double) * static_cast<size_t>(G) + al - 1) / al * al;
    const size_t state_bytes = sizeof(double) * 8 * static_cast<size_t>(G);
    bmd_status st = ensure(&p->d_ws, &p->ws_cap,
                           draw_bytes + part_bytes + mean_bytes + state_bytes + sizeof(int32_t) * G);
    if (st != BMD_OK) return st;
    char* base = static_cast<char*>(p->d_ws);
    double* partials = reinterpret_cast<double*>(base + draw_bytes);
    double* mean = reinterpret_cast<double*>(base + draw_bytes + part_bytes);
    double* state = reinterpret_cast<double*>(base + draw_bytes + part_bytes + mean_bytes);
    int32_t* side = reinterpret_cast<int32_t*>(base + draw_bytes + part_bytes + mean_bytes + state_bytes);
    HIP_TRY(launch_draws(p, prec, 0, M, p->d_ws, s), "draw kernel");
    // every probe has both critical values finite and the second on the FWER
    // boundary, whatever the problem's own rule
    SplitRuleScope split(p);
    hipError_t e = hipSuccess;
    // two interior points, n_iter golden steps, then the two ends of the range
    const int n_sweeps = 4 + n_iter;
    for (int ph = 0; ph <= n_sweeps && e == hipSuccess; ++ph) {
        const int end = ph == n_sweeps - 2 ? 1 : ph == n_sweeps - 1 ? 2 : 0;
        e = launch_levels_golden(p, ph, ph < n_sweeps, end, a_lo, a_hi, mean, state, side, s);
        if (e == hipSuccess && ph < n_sweeps)
            e = launch_eval_grid(p, prec, M, p->d_ws, partials, static_cast<int>(n_slices), slice_len, false, s);
        if (e == hipSuccess && ph < n_sweeps)
            e = launch_finalize(p, M, partials, static_cast<int>(n_slices), mean, nullptr, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d_best, state + 6 * G, sizeof(double) * G, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_alpha1, state + 7 * G, sizeof(double) * G, hipMemcpyDeviceToDevice, s);
    split.restore();
    // the problem's own critical values, whatever happened above
    const hipError_t er = launch_design_precompute(p, s);
    HIP_TRY(e, "level search");
    HIP_TRY(er, "design precompute");
    return BMD_OK;
}

bmd_status bmd_eval_grid_two_layer(bmd_problem* p, uint64_t n_outer, uint64_t n_inner, int32_t prec,
                                   int32_t blocks_outer, int32_t blocks_inner, double* d_mean, double* d_var,
                                   void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "the two-layer estimator needs a grid problem");
    if (p->P.effect != BMD_EFFECT_PAPER_GAUSS)
        return fail(BMD_ENOTSUP, "the two-layer estimator needs the Formula 10 prior (BMD_EFFECT_PAPER_GAUSS)");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_mean) return fail(BMD_EINVAL, "NULL d_mean");
    const int64_t A = blocks_outer, B = blocks_inner;
    if (A < 2 || A > 64 || B < 2 || B > 64) return fail(BMD_ERANGE, "blocks_outer and blocks_inner must be in [2, 64]");
    if (n_outer == 0 || n_outer > (1ull << 31) || n_outer % A != 0)
        return fail(BMD_ERANGE, "n_outer must be in [1, 2^31] and a multiple of blocks_outer");
    if (n_inner == 0 || n_inner > (1ull << 26) || n_inner % 1024 != 0 || n_inner % B != 0 || (n_inner / B) % 256 != 0)
        return fail(BMD_ERANGE, "n_inner must be a multiple of 1024 and of 256 blocks_inner, at most 2^26");
    const int64_t N1 = static_cast<int64_t>(n_outer), N2 = static_cast<int64_t>(n_inner);
    if (static_cast<double>(N1 / A) * static_cast<double>(N2 / B) >= 4294967296.0)
        return fail(BMD_ERANGE, "a block of (n_outer / blocks_outer) x (n_inner / blocks_inner) comparisons "
                                "must stay below 2^32");
    const int n = p->P.design_space == BMD_DESIGN_ALPHA3 ? 3 : p->P.design_space == BMD_DESIGN_ALPHA4 ? 4 : 2;
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t al = 256;
    const size_t draw_bytes = (draw_workspace_bytes(p, BMD_FP64, N1) + al - 1) / al * al;
    const size_t inner_bytes = (two_layer_inner_bytes(n, N2) + al - 1) / al * al;
    const size_t block_bytes = sizeof(uint32_t) * static_cast<size_t>(p->P.G) * A * B;
    bmd_status st = ensure(&p->d_ws, &p->ws_cap, draw_bytes + inner_bytes + block_bytes);
    if (st != BMD_OK) return st;
    char* base = static_cast<char*>(p->d_ws);
    double* inner = reinterpret_cast<double*>(base + draw_bytes);
    uint32_t* blocks = reinterpret_cast<uint32_t*>(base + draw_bytes + inner_bytes);
    HIP_TRY(launch_draws(p, BMD_FP64, 0, N1, p->d_ws, s), "draw kernel");
    HIP_TRY(launch_two_layer(p, prec, n, N1, N2, static_cast<int>(A), static_cast<int>(B), draws_fp64(p, N1, p->d_ws),
                             inner, blocks, d_mean, d_var, s),
            "two-layer kernels");
    return BMD_OK;
}

bmd_status bmd_eval_grid_dalpha(bmd_problem* p, uint64_t n_draws, int32_t prec, double* d_mean, double* d_dmean,
                                void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ESTATE, "the alpha_1 derivative needs a grid of cutoff designs");
    if (p->P.alpha_rule != BMD_ALPHA_SPLIT && p->P.alpha_rule != BMD_ALPHA_FIXED)
        return fail(BMD_ENOTSUP, "the alpha_1 derivative needs rule BMD_ALPHA_SPLIT or BMD_ALPHA_FIXED");
    if (!(p->desc.alpha_fixed[0] > 0.0)) return fail(BMD_ERANGE, "the first level alpha_1 must be > 0");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_mean || !d_dmean) return fail(BMD_EINVAL, "NULL d_mean or d_dmean");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + 255) / 256 * 256;
    const size_t part_bytes = sizeof(double) * 2 * static_cast<size_t>(p->P.G) * n_slices;
    bmd_status st = ensure(&p->d_ws, &p->ws_cap, draw_bytes + part_bytes);
    if (st != BMD_OK) return st;
    double* partials = reinterpret_cast<double*>(static_cast<char*>(p->d_ws) + draw_bytes);
    HIP_TRY(launch_draws(p, prec, 0, M, p->d_ws, s), "draw kernel");
    HIP_TRY(launch_eval_grid_dalpha(p, prec, M, p->d_ws, partials, static_cast<int>(n_slices), slice_len, s),
            "derivative sweep");
    HIP_TRY(launch_finalize_dalpha(p, M, partials, static_cast<int>(n_slices), d_mean, d_dmean, s), "finalize kernel");
    return BMD_OK;
}

bmd_status bmd_optimize_levels_newton(bmd_problem* p, uint64_t n_draws, int32_t prec, double a_lo, double a_hi,
                                      int32_t n_iter, double tol, double* d_best, double* d_alpha1, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ESTATE, "level search needs a grid of cutoff designs");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_best || !d_alpha1) return fail(BMD_EINVAL, "NULL d_best or d_alpha1");
    if (!std::isfinite(a_lo) || !std::isfinite(a_hi) || !(0.0 < a_lo && a_lo < a_hi && a_hi < p->P.alpha0))
        return fail(BMD_ERANGE, "need 0 < a_lo < a_hi < alpha0");
    if (n_iter < 0 || n_iter > 200 || !(tol >= 0.0)) return fail(BMD_ERANGE, "n_iter in [0, 200] and tol >= 0");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    const int64_t G = p->P.G;
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t al = 256;
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + al - 1) / al * al;
    const size_t part_bytes = (sizeof(double) * 2 * static_cast<size_t>(G) * n_slices + al - 1) / al * al;
    const size_t mean_bytes = (sizeof(double) * static_cast<size_t>(G) + al - 1) / al * al;
    const size_t state_bytes = sizeof(double) * 9 * static_cast<size_t>(G);
    bmd_status st = ensure(&p->d_ws, &p->ws_cap, draw_bytes + part_bytes + 2 * mean_bytes + state_bytes);
    if (st != BMD_OK) return st;
    char* base = static_cast<char*>(p->d_ws);
    double* partials = reinterpret_cast<double*>(base + draw_bytes);
    double* mean = reinterpret_cast<double*>(base + draw_bytes + part_bytes);
    double* dmean = reinterpret_cast<double*>(base + draw_bytes + part_bytes + mean_bytes);
    double* state = reinterpret_cast<double*>(base + draw_bytes + part_bytes + 2 * mean_bytes);
    HIP_TRY(launch_draws(p, prec, 0, M, p->d_ws, s), "draw kernel");
    SplitRuleScope split(p);   // probes as in bmd_optimize_levels
    hipError_t e = hipSuccess;
    // the two ends of the range, then n_iter false-position steps
    const int n_sweeps = 2 + n_iter;
    for (int ph = 0; ph <= n_sweeps && e == hipSuccess; ++ph) {
        e = launch_levels_newton(p, ph, a_lo, a_hi, tol, mean, dmean, state, s);
        if (e == hipSuccess && ph < n_sweeps)
            e = launch_eval_grid_dalpha(p, prec, M, p->d_ws, partials, static_cast<int>(n_slices), slice_len, s);
        if (e == hipSuccess && ph < n_sweeps)
            e = launch_finalize_dalpha(p, M, partials, static_cast<int>(n_slices), mean, dmean, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d_best, state + 5 * G, sizeof(double) * G, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_alpha1, state + 6 * G, sizeof(double) * G, hipMemcpyDeviceToDevice, s);
    split.restore();
    // the problem's own critical values, whatever happened above
    const hipError_t er = launch_design_precompute(p, s);
    HIP_TRY(e, "level search");
    HIP_TRY(er, "design precompute");
    return BMD_OK;
}

bmd_status bmd_eval_grid_levels(bmd_problem* p, uint64_t n_draws, int32_t prec, const double* h_alpha1,
                                int32_t n_alpha, double* d_best, int32_t* d_best_k, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ESTATE, "level splits need a grid of cutoff designs");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!h_alpha1 || !d_best) return fail(BMD_EINVAL, "NULL h_alpha1 or d_best");
    if (n_alpha < 1 || n_alpha > 4096) return fail(BMD_ERANGE, "n_alpha must be in [1, 4096]");
    for (int k = 0; k < n_alpha; ++k)
        if (!std::isfinite(h_alpha1[k]) || !(h_alpha1[k] > 0.0 && h_alpha1[k] < p->P.alpha0))
            return fail(BMD_ERANGE, "level %d = %g outside (0, alpha0)", k, h_alpha1[k]);
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    const int64_t G = p->P.G;
    int64_t n_slices = 0, slice_len = 0;
    sweep_slices(p, prec, M, &n_slices, &slice_len);
    const size_t draw_bytes = (draw_workspace_bytes(p, prec, M) + 255) / 256 * 256;
    const size_t part_bytes = (sizeof(double) * 2 * static_cast<size_t>(G) * n_slices + 255) / 256 * 256;
    bmd_status st = ensure(&p->d_ws, &p->ws_cap, draw_bytes + part_bytes + sizeof(double) * G);
    if (st != BMD_OK) return st;
    double* partials = reinterpret_cast<double*>(static_cast<char*>(p->d_ws) + draw_bytes);
    double* mean = reinterpret_cast<double*>(static_cast<char*>(p->d_ws) + draw_bytes + part_bytes);
    HIP_TRY(launch_draws(p, prec, 0, M, p->d_ws, s), "draw kernel");
    hipError_t e = hipSuccess;
    for (int k = 0; k < n_alpha && e == hipSuccess; ++k) {
        e = launch_levels_z(p, -host_quantile(h_alpha1[k]), s);
        if (e == hipSuccess)
            e = launch_eval_grid(p, prec, M, p->d_ws, partials, static_cast<int>(n_slices), slice_len, false, s);
        if (e == hipSuccess) e = launch_finalize(p, M, partials, static_cast<int>(n_slices), mean, nullptr, s);
        if (e == hipSuccess) e = launch_levels_best(p, k, mean, d_best, d_best_k, s);
    }
    // the problem's own critical values, whatever happened above
    const hipError_t er = launch_design_precompute(p, s);
    HIP_TRY(e, "level sweeps");
    HIP_TRY(er, "design precompute");
    return BMD_OK;
}

bmd_status bmd_smooth(bmd_problem* p, const double* d_in, double* d_out, int32_t prec, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "smooth needs a grid problem");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_in || !d_out) return fail(BMD_EINVAL, "NULL surface pointer");
    if (d_in == d_out) return fail(BMD_EINVAL, "d_in and d_out must not alias");
    DeviceGuard guard(p->device);
    // designs without a third level are NaN: smooth over the others
    const bool masked = p->P.design_space == BMD_DESIGN_ALPHA3 || p->P.design_space == BMD_DESIGN_ALPHA4 ||
                        p->P.design_space == BMD_DESIGN_NESTED3 || p->P.design_space == BMD_DESIGN_NESTED4;
    bmd_status st = ensure(&p->d_ws2, &p->ws2_cap, sizeof(double) * static_cast<size_t>(p->P.G) * (masked ? 4 : 1));
    if (st != BMD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    mark(p, 6, s);
    if (masked)
        HIP_TRY(launch_smooth_masked(p, prec, d_in, d_out, static_cast<double*>(p->d_ws2), s), "smooth kernel");
    else
        HIP_TRY(launch_smooth(p, prec, d_in, d_out, static_cast<double*>(p->d_ws2), s), "smooth kernel");
    mark(p, 7, s);
    return BMD_OK;
}

bmd_status bmd_argmax(bmd_problem* p, const double* d_surface, int64_t* h_index, double* h_value, int32_t* h_cell,
                      void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "argmax needs a grid problem");
    if (!d_surface || !h_index || !h_value) return fail(BMD_EINVAL, "NULL pointer argument");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = p->P.G;
    const int n_part = static_cast<int>(std::min<int64_t>(1024, (n + 255) / 256));
    bmd_status st = ensure(&p->d_ws2, &p->ws2_cap, std::max<size_t>(sizeof(double) * n, 16 * 1024 + 256));
    if (st != BMD_OK) return st;
    double* pv = static_cast<double*>(p->d_ws2);
    int64_t* pi = reinterpret_cast<int64_t*>(static_cast<char*>(p->d_ws2) + 8 * 1024);
    mark(p, 8, s);
    HIP_TRY(launch_argmax(p, d_surface, n, pv, pi, n_part, s), "argmax kernels");
    mark(p, 9, s);
    double v;
    int64_t i;
    HIP_TRY(hipMemcpyAsync(&v, pv, sizeof v, hipMemcpyDeviceToHost, s), "argmax readback");
    HIP_TRY(hipMemcpyAsync(&i, pi, sizeof i, hipMemcpyDeviceToHost, s), "argmax readback");
    HIP_TRY(hipStreamSynchronize(s), "argmax sync");
    if (i == INT64_MAX) {
        i = 0;
        v = NAN;
    }
    *h_index = i;
    *h_value = v;
    if (h_cell) {
        int64_t rem = i;
        for (int j = 0; j < p->P.d; ++j) {
            h_cell[j] = static_cast<int32_t>(rem / p->P.stride[j]);
            rem -= static_cast<int64_t>(h_cell[j]) * p->P.stride[j];
        }
    }
    return BMD_OK;
}

bmd_status bmd_grad_design(bmd_problem* p, const double* d_q, int64_t B, uint64_t n_draws, int32_t prec,
                           double* d_obj, double* d_grad_q, double* d_grad_mu, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (!d_q || !d_obj) return fail(BMD_EINVAL, "NULL d_q or d_obj");
    if (B < 1 || B > (int64_t(1) << 30)) return fail(BMD_ERANGE, "B must be in [1, 2^30]");
    if (n_draws == 0 || n_draws > (1ull << 40)) return fail(BMD_ERANGE, "n_draws must be in [1, 2^40]");
    if (p->P.effect != BMD_EFFECT_STEP || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ENOTSUP, "grad_design needs the step prior and cutoff designs");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = static_cast<int64_t>(n_draws);
    const int chunk = grad_chunk(prec, p->P.d, p->tab[prec].K);
    // Draw slices: about kSweepRounds rounds of resident workgroups.
    const int lanes = grad_lanes(B);
    const int64_t bx = (B * lanes + 127) / 128;   // 128 threads per workgroup, `lanes` per point
    const int64_t resident = static_cast<int64_t>(p->n_cu) * grad_blocks_per_cu(p, prec);
    int64_t n_slices = (kSweepRounds * resident + bx - 1) / bx;
    n_slices = std::max<int64_t>(1, std::min<int64_t>({n_slices, (M + chunk - 1) / chunk, 65535}));
    // at least 16 draws per thread of a slice, so the per-point setup is amortised
    int64_t slice_len = std::max<int64_t>((M + n_slices - 1) / n_slices, std::min<int64_t>(M, 16 * lanes));
    slice_len = (slice_len + chunk - 1) / chunk * chunk;
    n_slices = (M + slice_len - 1) / slice_len;
    bmd_status st =
        ensure(&p->d_ws, &p->ws_cap, grad_workspace_bytes(p, prec, B, static_cast<int>(n_slices), M, slice_len));
    if (st != BMD_OK) return st;
    HIP_TRY(launch_grad(p, prec, d_q, B, M, p->d_ws, static_cast<int>(n_slices), slice_len, d_obj, d_grad_q,
                        d_grad_mu, s),
            "gradient kernels");
    return BMD_OK;
}

namespace {

struct DeviceBuffer {
    void* ptr = nullptr;
    ~DeviceBuffer() {
        if (ptr) (void)hipFree(ptr);
    }
};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Host plan of one problem of a batch.
struct BatchPlan {
    int key;              // launch group: 2 * d + (matrix-core sweep ? 1 : 0)
    int64_t G, M, tiles, chunk;
    int64_t slice_len = 0, n_slices = 0;
    size_t draw_bytes = 0, part_bytes = 0;
};

// Launch settings of one sweep launch kind (biomarker count, kernel kind) of
// a batch: the tile body's draws per LDS chunk, how many rounds of resident
// workgroups the launch's work list is sliced into, and the kernel's
// launch-bound variant.  Chosen per device and precision by the autotuner
// (tune_phase) on first use, or fixed.
struct BatchSettings {
    int chunk = 0;                 // 0: the one-problem sweep's chunk
    int rounds = kSweepRounds;
    int variant = 0;
    bool tuned = false;
    double ms = 0.0;               // calibration time of the chosen settings
};
using TuneKey = std::array<int, 3>;   // device, precision, launch key
std::mutex g_tune_mu;
std::map<TuneKey, BatchSettings> g_tune;
int g_tune_mode = 1;                  // 1: tune each launch kind on first use; 0: fixed settings

// One sweep launch of a group: its problems (indices into the group's plans),
// kernel variant, LDS and the slicing of its members.
struct Phase {
    int key = 0, rep = -1;   // rep: a problem of the phase (index in the group)
    size_t lds = 0;
    int grid = 0;
    BatchSettings set;
    std::vector<int> members;
};

// Plans the phases of the problems ps[0..n) with plans pl (slices written
// into pl): per launch key the settings of `sets` (defaults when absent).
// chunk < 0 marks a chunk that does not fit the LDS limit: false.
bool plan_phases(bmd_problem* const* ps, std::vector<BatchPlan>& pl, int prec, int n_cu,
                 const std::map<int, BatchSettings>& sets, std::vector<Phase>* out) {
    const int n = static_cast<int>(pl.size());
    std::vector<int> keys;
    for (const auto& b : pl)
        if (std::find(keys.begin(), keys.end(), b.key) == keys.end()) keys.push_back(b.key);
    std::sort(keys.begin(), keys.end());
    for (int key : keys) {
        Phase ph;
        ph.key = key;
        auto it = sets.find(key);
        if (it != sets.end()) ph.set = it->second;
        for (int i = 0; i < n; ++i)
            if (pl[i].key == key) {
                ph.members.push_back(i);
                if (ph.rep < 0) ph.rep = i;
                ph.lds = std::max(ph.lds, batch_phase_lds(ps[i], prec, ph.set.chunk));
            }
        if (ph.lds > 64 * 1024) return false;
        const int bpc = batch_phase_blocks_per_cu(ps[ph.rep], prec, ph.lds, ph.set.variant);
        ph.grid = n_cu * bpc;
        // Slices: about `rounds` items per resident workgroup over the phase.
        double work = 0.0;
        for (int i : ph.members) work += static_cast<double>(pl[i].tiles) * kEvalBlock * pl[i].M;
        const double target = work / (static_cast<double>(ph.set.rounds) * ph.grid) / kEvalBlock;
        for (int i : ph.members) {
            BatchPlan& b = pl[i];
            const int64_t ch = ph.set.chunk > 0 && b.chunk > 1 ? ph.set.chunk : b.chunk;
            const int64_t Mr = (b.M + ch - 1) / ch * ch;
            int64_t L = static_cast<int64_t>(std::ceil(std::max(target, 64.0) / ch)) * ch;
            L = std::max<int64_t>(ch, std::min<int64_t>(L, Mr));
            b.slice_len = L;
            b.n_slices = (b.M + L - 1) / L;
            b.part_bytes = align256(sizeof(double) * 2 * static_cast<size_t>(b.G) * b.n_slices);
        }
        out->push_back(std::move(ph));
    }
    return true;
}

// One group of problems ps[0..n) (batch indices first..first+n): draws,
// sweeps and finalize, captured in one graph and launched once (capture), or
// launched one by one with the sweep launches timed (phase_ms, per phase).
// Slices follow each launch kind's settings.
bmd_status run_batch_group(bmd_problem* const* ps, std::vector<BatchPlan> pl, int first, int prec,
                           double* const* d_means, int n_cu, hipStream_t cs, unsigned long long* d_tstart,
                           unsigned long long* d_tdone, int* d_left, bool restart_clock,
                           const std::map<int, BatchSettings>& sets, bool capture, std::vector<double>* phase_ms) {
    const int n = static_cast<int>(pl.size());
    std::vector<Phase> phases;
    if (!plan_phases(ps, pl, prec, n_cu, sets, &phases)) return fail(BMD_ERANGE, "batch chunk exceeds the LDS limit");
    // Work lists, costliest items first (the ragged last slice of a problem is cheaper).
    struct Item {
        int4 v;
        double c;
    };
    std::vector<std::vector<int4>> lists(phases.size());
    std::vector<int> items_per(n, 0);
    size_t n_items_total = 0;
    for (size_t f = 0; f < phases.size(); ++f) {
        std::vector<Item> list;
        for (int i : phases[f].members) {
            const BatchPlan& b = pl[i];
            for (int64_t t = 0; t < b.tiles; ++t)
                for (int64_t sl = 0; sl < b.n_slices; ++sl) {
                    const double draws = static_cast<double>(std::min<int64_t>(b.slice_len, b.M - sl * b.slice_len));
                    list.push_back({make_int4(i, static_cast<int>(t), static_cast<int>(sl), 0), draws});
                }
            items_per[i] = static_cast<int>(b.tiles * b.n_slices);
        }
        if (list.size() > (1u << 24)) return fail(BMD_ERANGE, "batch work list of %zu items is too large", list.size());
        std::stable_sort(list.begin(), list.end(), [](const Item& x, const Item& y) { return x.c > y.c; });
        for (const Item& it : list) lists[f].push_back(it.v);
        n_items_total += list.size();
    }

    // One device allocation: records, draw jobs, finals, items, counters, draws, partials.
    const size_t rec_b = batch_record_bytes(prec), job_b = draw_job_bytes(prec);
    size_t off = 0;
    const size_t o_rec = off;   off += align256(rec_b * n);
    const size_t o_job = off;   off += align256(job_b * n);
    const size_t o_fin = off;   off += align256(sizeof(BatchFinal) * n);
    const size_t o_items = off; off += align256(sizeof(int4) * std::max<size_t>(n_items_total, 1));
    const size_t o_ctr = off;   off += align256(sizeof(int) * n);   // items per problem
    std::vector<size_t> o_draw(n), o_part(n);
    for (int i = 0; i < n; ++i) { o_draw[i] = off; off += pl[i].draw_bytes; }
    for (int i = 0; i < n; ++i) { o_part[i] = off; off += pl[i].part_bytes; }
    DeviceBuffer buf;
    {
        hipError_t e = hipMalloc(&buf.ptr, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(BMD_ENOMEM, "batch workspace of %zu bytes: %s", off, hipGetErrorString(e));
        }
    }
    char* base = static_cast<char*>(buf.ptr);
    std::vector<char> host(o_draw.empty() ? o_ctr : o_draw[0], 0);   // everything before the draws
    std::vector<BatchFinal> fin(n);
    std::vector<int> chunk_of(n, 0);
    for (const Phase& ph : phases)
        for (int i : ph.members) chunk_of[i] = ph.set.chunk;
    int64_t draws_total = 0, designs_total = 0;
    for (int i = 0; i < n; ++i) {
        bmd_problem* p = ps[i];
        double* part = reinterpret_cast<double*>(base + o_part[i]);
        batch_fill_record(prec, host.data() + o_rec + rec_b * i, p, base + o_draw[i], pl[i].M, pl[i].slice_len, part,
                          first + i, chunk_of[i]);
        fill_draw_job(prec, host.data() + o_job + job_b * i, p, base + o_draw[i], pl[i].M, draws_total);
        fin[i] = BatchFinal{designs_total, pl[i].G, pl[i].M, static_cast<int>(pl[i].n_slices), part, d_means[i]};
        draws_total += pl[i].M;
        designs_total += pl[i].G;
    }
    std::memcpy(host.data() + o_fin, fin.data(), sizeof(BatchFinal) * n);
    {
        size_t k = 0;
        for (const auto& l : lists) {
            std::memcpy(host.data() + o_items + sizeof(int4) * k, l.data(), sizeof(int4) * l.size());
            k += l.size();
        }
    }
    std::memcpy(host.data() + o_ctr, items_per.data(), sizeof(int) * n);
    HIP_TRY(hipMemcpy(base, host.data(), host.size(), hipMemcpyHostToDevice), "batch upload");

    const int* d_items_per = reinterpret_cast<const int*>(base + o_ctr);
    auto launches = [&](std::vector<hipEvent_t>* ev) -> hipError_t {
        hipError_t le =
            launch_batch_reset(d_left, d_tdone, d_items_per, first, n, restart_clock ? d_tstart : nullptr, cs);
        if (le == hipSuccess) le = launch_draws_batch(prec, base + o_job, n, draws_total, cs);
        size_t k = 0;
        for (size_t f = 0; f < phases.size() && le == hipSuccess; ++f) {
            // records are indexed within the group; left / t_done by batch index
            BatchPhase ph{base + o_rec, reinterpret_cast<const int4*>(base + o_items) + k,
                          static_cast<int>(lists[f].size()), d_left, d_tstart, d_tdone};
            if (ev) le = hipEventRecord((*ev)[2 * f], cs);
            if (le == hipSuccess)
                le = launch_batch_phase(ps[phases[f].rep], prec, ph, phases[f].lds, phases[f].set.variant, cs);
            if (ev && le == hipSuccess) le = hipEventRecord((*ev)[2 * f + 1], cs);
            k += lists[f].size();
        }
        if (le == hipSuccess)
            le = launch_batch_finalize(reinterpret_cast<const BatchFinal*>(base + o_fin), n, designs_total, cs);
        return le;
    };
    if (!capture) {
        std::vector<hipEvent_t> ev(2 * phases.size(), nullptr);
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
        struct EventsGuard {
            std::vector<hipEvent_t>& v;
            ~EventsGuard() {
                for (auto e : v)
                    if (e) (void)hipEventDestroy(e);
            }
        } eg{ev};
        HIP_TRY(launches(&ev), "batch launches");
        HIP_TRY(hipStreamSynchronize(cs), "batch sync");
        if (phase_ms) {
            phase_ms->assign(phases.size(), 0.0);
            for (size_t f = 0; f < phases.size(); ++f) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 * f], ev[2 * f + 1]), "batch timing");
                (*phase_ms)[f] = ms;
            }
        }
        return BMD_OK;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const hipError_t le = launches(nullptr);
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "batch capture");
    }
    HIP_TRY(ce, "hipStreamEndCapture");
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    HIP_TRY(e, "batch graph");
    return BMD_OK;
}

// Autotuner of one launch kind: its problems ps[0..n) (plans pl) run with
// their draw counts scaled down to a calibration workload of about
// kTuneEvals evaluations, launched directly and timed with HIP events; the
// draws per LDS chunk, then the launch-bound variant, then the rounds of
// resident workgroups are searched in turn (coordinate descent from the
// fixed settings), each candidate timed twice and its faster run kept.
constexpr double kTuneEvals = 4e9;
bmd_status tune_phase(bmd_problem* const* ps, std::vector<BatchPlan> pl, int prec, int n_cu, hipStream_t cs,
                      unsigned long long* d_tstart, unsigned long long* d_tdone, int* d_left, BatchSettings* best) {
    const int n = static_cast<int>(pl.size());
    const int key = pl[0].key;
    double work = 0.0;
    for (const auto& b : pl) work += static_cast<double>(b.G) * static_cast<double>(b.M);
    const double scale = std::min(1.0, kTuneEvals / std::max(work, 1.0));
    int64_t G_total = 0;
    for (int i = 0; i < n; ++i) {
        BatchPlan& b = pl[i];
        b.M = std::max<int64_t>(std::min<int64_t>(b.M, 256), static_cast<int64_t>(std::ceil(b.M * scale)));
        b.draw_bytes = align256(draw_workspace_bytes(ps[i], prec, b.M));
        G_total += b.G;
    }
    DeviceBuffer means;
    {
        const hipError_t e = hipMalloc(&means.ptr, sizeof(double) * std::max<int64_t>(G_total, 1));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(BMD_ENOMEM, "batch tuning buffers: %s", hipGetErrorString(e));
        }
    }
    std::vector<double*> mp(n);
    {
        int64_t o = 0;
        for (int i = 0; i < n; ++i) {
            mp[i] = static_cast<double*>(means.ptr) + o;
            o += pl[i].G;
        }
    }
    auto time_of = [&](const BatchSettings& c, double* ms) -> bmd_status {
        std::map<int, BatchSettings> sets{{key, c}};
        double t = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            std::vector<double> phase_ms;
            bmd_status st = run_batch_group(ps, pl, 0, prec, mp.data(), n_cu, cs, d_tstart, d_tdone, d_left, true,
                                            sets, false, &phase_ms);
            if (st != BMD_OK) return st;
            t = std::min(t, phase_ms.empty() ? 0.0 : phase_ms[0]);
        }
        *ms = t;
        return BMD_OK;
    };
    const bool mf = pl[0].chunk > 1;
    const int step = prec == BMD_FP64 ? 4 : 8;
    std::vector<int> chunks;
    if (mf)
        for (int c = step; c <= 32; c += step) chunks.push_back(c);
    else
        chunks.push_back(0);
    const int n_var = batch_variants(ps[0], prec);
    BatchSettings cur;   // the fixed settings
    double t_cur = 0.0;
    bmd_status st = time_of(cur, &t_cur);
    if (st != BMD_OK) return st;
    auto consider = [&](BatchSettings c) -> bmd_status {
        // candidates whose LDS does not fit are skipped
        for (int i = 0; i < n; ++i)
            if (batch_phase_lds(ps[i], prec, c.chunk) > 64 * 1024) return BMD_OK;
        double t = 0.0;
        const bmd_status s2 = time_of(c, &t);
        if (s2 != BMD_OK) return s2;
        if (t < t_cur) {
            cur = c;
            t_cur = t;
        }
        return BMD_OK;
    };
    for (int c : chunks) {
        BatchSettings x = cur;
        x.chunk = c;
        if ((st = consider(x)) != BMD_OK) return st;
    }
    for (int v = 0; v < n_var; ++v) {
        BatchSettings x = cur;
        x.variant = v;
        if ((st = consider(x)) != BMD_OK) return st;
    }
    for (int r : {2, 4, 16}) {
        BatchSettings x = cur;
        x.rounds = r;
        if ((st = consider(x)) != BMD_OK) return st;
    }
    cur.tuned = true;
    cur.ms = t_cur;
    *best = cur;
    return BMD_OK;
}

// Value, gradient and Hessian of the smoothed surface at the continuous
// design q (sums from launch_smooth_local); synchronises the stream.
bmd_status smoothed_at(bmd_problem* p, const double* d_surface, const double* q, double* S, double* g, double* H,
                       hipStream_t s) {
    const int d = p->P.d;
    bmd_status st = ensure(&p->d_ws2, &p->ws2_cap, smooth_local_bytes() + 2 * kMaxDim * kMaxDim * sizeof(double) + 1024);
    if (st != BMD_OK) return st;
    double lo[kMaxDim], hi[kMaxDim];
    for (int j = 0; j < d; ++j) axis_range(p->desc, j, &lo[j], &hi[j]);
    double* ws = static_cast<double*>(p->d_ws2);
    double* out = ws + smooth_local_bytes() / sizeof(double);
    HIP_TRY(launch_smooth_local(p, d_surface, q, lo, hi, ws, out, s), "smoothing at a point");
    const int na = 1 + d + d * (d + 1) / 2;
    double acc[2 * (1 + kMaxDim + kMaxDim * (kMaxDim + 1) / 2)];
    HIP_TRY(hipMemcpyAsync(acc, out, sizeof(double) * 2 * na, hipMemcpyDeviceToHost, s), "smoothing readback");
    HIP_TRY(hipStreamSynchronize(s), "smoothing sync");
    const double* F = acc;
    const double* W = acc + na;
    if (!(W[0] > 0.0)) return fail(BMD_ERANGE, "no design with a value carries weight at this point");
    double Nj[kMaxDim], Dj[kMaxDim], Njl[kMaxDim][kMaxDim], Djl[kMaxDim][kMaxDim];
    int k = 1 + d;
    for (int j = 0; j < d; ++j) {
        Nj[j] = F[1 + j];
        Dj[j] = W[1 + j];
        for (int l = j; l < d; ++l, ++k) {
            Njl[j][l] = Njl[l][j] = F[k];
            Djl[j][l] = Djl[l][j] = W[k];
        }
    }
    for (int j = 0; j < d; ++j) {   // d2K/dq_j^2 also has -K / b_j^2
        const double b2 = p->desc.bandwidth[j] * p->desc.bandwidth[j];
        Njl[j][j] -= F[0] / b2;
        Djl[j][j] -= W[0] / b2;
    }
    const double D0 = W[0], val = F[0] / D0;
    double gg[kMaxDim];
    for (int j = 0; j < d; ++j) gg[j] = (Nj[j] - val * Dj[j]) / D0;
    *S = val;
    if (g)
        for (int j = 0; j < d; ++j) g[j] = gg[j];
    if (H)
        for (int j = 0; j < d; ++j)
            for (int l = 0; l < d; ++l)
                H[j * d + l] = (Njl[j][l] - val * Djl[j][l] - gg[j] * Dj[l] - gg[l] * Dj[j]) / D0;
    return BMD_OK;
}

// Solve (-H) x = g by Cholesky; false when -H is not positive definite.
bool newton_direction(int d, const double* H, const double* g, double* x) {
    double L[kMaxDim][kMaxDim] = {};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j <= i; ++j) {
            double sum = -H[i * d + j];
            for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(sum > 0.0)) return false;
                L[i][i] = std::sqrt(sum);
            } else {
                L[i][j] = sum / L[j][j];
            }
        }
    double y[kMaxDim];
    for (int i = 0; i < d; ++i) {
        double sum = g[i];
        for (int k = 0; k < i; ++k) sum -= L[i][k] * y[k];
        y[i] = sum / L[i][i];
    }
    for (int i = d - 1; i >= 0; --i) {
        double sum = y[i];
        for (int k = i + 1; k < d; ++k) sum -= L[k][i] * x[k];
        x[i] = sum / L[i][i];
    }
    return true;
}

}  // namespace

bmd_status bmd_refine_design(bmd_problem* p, const double* h_q0, uint64_t n_draws, int32_t prec, int32_t max_iter,
                             double tol, double* h_q, double* h_obj, int32_t* h_iters, void* stream) {
    g_err.clear();
    if (!p || !h_q0 || !h_q || !h_obj || !h_iters) return fail(BMD_EINVAL, "NULL argument");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (max_iter < 0 || max_iter > 10000 || !(tol >= 0.0)) return fail(BMD_ERANGE, "max_iter or tol out of range");
    if (p->P.effect != BMD_EFFECT_STEP || p->P.design_space != BMD_DESIGN_CUTOFFS)
        return fail(BMD_ENOTSUP, "refinement needs the step prior and cutoff designs");
    constexpr int kTrials = 8;
    constexpr double kFirstStep = 0.05, kMaxStep = 0.1, kArmijo = 1e-4;
    const int d = p->P.d;
    const double lo = p->P.q_lo, hi = p->P.q_hi;
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceBuffer buf;
    {
        const hipError_t e = hipMalloc(&buf.ptr, sizeof(double) * kTrials * (2 * d + 1));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(BMD_ENOMEM, "refinement buffers: %s", hipGetErrorString(e));
        }
    }
    double* d_q = static_cast<double*>(buf.ptr);
    double* d_g = d_q + kTrials * d;
    double* d_f = d_g + kTrials * d;
    std::vector<double> q(d), g(d), tq(kTrials * d), tg(kTrials * d), tf(kTrials);
    for (int j = 0; j < d; ++j) q[j] = std::min(hi, std::max(lo, h_q0[j]));
    // objective and gradient at the n points of tq (host) -> tf, tg
    auto evaluate = [&](int n) -> bmd_status {
        HIP_TRY(hipMemcpyAsync(d_q, tq.data(), sizeof(double) * n * d, hipMemcpyHostToDevice, s), "refine upload");
        const bmd_status st = bmd_grad_design(p, d_q, n, n_draws, prec, d_f, d_g, nullptr, s);
        if (st != BMD_OK) return st;
        HIP_TRY(hipMemcpyAsync(tf.data(), d_f, sizeof(double) * n, hipMemcpyDeviceToHost, s), "refine download");
        HIP_TRY(hipMemcpyAsync(tg.data(), d_g, sizeof(double) * n * d, hipMemcpyDeviceToHost, s), "refine download");
        HIP_TRY(hipStreamSynchronize(s), "refine sync");
        return BMD_OK;
    };
    std::copy(q.begin(), q.end(), tq.begin());
    bmd_status st = evaluate(1);
    if (st != BMD_OK) return st;
    double f = tf[0];
    std::copy(tg.begin(), tg.begin() + d, g.begin());
    double step = kFirstStep;
    int it = 0;
    while (it < max_iter) {
        double gn = 0.0;
        for (double x : g) gn = std::max(gn, std::fabs(x));
        if (gn == 0.0) break;
        double t[kTrials];
        for (int k = 0; k < kTrials; ++k) {
            t[k] = step * std::ldexp(1.0, -k);
            for (int j = 0; j < d; ++j)
                tq[k * d + j] = std::min(hi, std::max(lo, q[j] + (t[k] / gn) * g[j]));
        }
        st = evaluate(kTrials);
        if (st != BMD_OK) return st;
        int acc = -1;
        for (int k = 0; k < kTrials && acc < 0; ++k) {
            double slope = 0.0;
            for (int j = 0; j < d; ++j) slope += g[j] * (tq[k * d + j] - q[j]);
            if (tf[k] >= f + kArmijo * slope) acc = k;
        }
        if (acc < 0) break;
        ++it;
        double move = 0.0;
        for (int j = 0; j < d; ++j) {
            move = std::max(move, std::fabs(tq[acc * d + j] - q[j]));
            q[j] = tq[acc * d + j];
            g[j] = tg[acc * d + j];
        }
        f = tf[acc];
        step = std::min(2.0 * t[acc], kMaxStep);
        if (move < tol) break;
    }
    for (int j = 0; j < d; ++j) h_q[j] = q[j];
    *h_obj = f;
    *h_iters = it;
    return BMD_OK;
}

bmd_status bmd_smooth_at(bmd_problem* p, const double* d_surface, const double* h_q, double* h_value,
                         double* h_grad, double* h_hess, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "smooth_at needs a grid problem");
    if (!d_surface || !h_q || !h_value) return fail(BMD_EINVAL, "NULL pointer argument");
    for (int j = 0; j < p->P.d; ++j)
        if (!std::isfinite(h_q[j])) return fail(BMD_EINVAL, "q[%d] is not finite", j);
    DeviceGuard guard(p->device);
    return smoothed_at(p, d_surface, h_q, h_value, h_grad, h_hess, static_cast<hipStream_t>(stream));
}

extern "C++" {
namespace {

// Ascent on a deterministic surface from q0 (value, gradient and Hessian from
// eval(q, &f, g, H)): a Newton step where -H has a Cholesky factor, else a
// gradient step of a tenth of the smallest smoothing bandwidth; each step
// projected into the grid's box and halved until it gains the Armijo fraction
// 1e-4 of its first-order gain.  Stops after max_iter steps, when a step moves
// no coordinate by more than tol, or when no halving is accepted.
template <typename Eval>
bmd_status newton_ascent(bmd_problem* p, Eval eval, const double* h_q0, int32_t max_iter, double tol, double* h_q,
                         double* h_value, int32_t* h_iters) {
    const int d = p->P.d;
    double lo[kMaxDim], hi[kMaxDim], bmin = 1e300;
    for (int j = 0; j < d; ++j) {
        axis_range(p->desc, j, &lo[j], &hi[j]);
        if (!std::isfinite(h_q0[j])) return fail(BMD_EINVAL, "q0[%d] is not finite", j);
        bmin = std::min(bmin, p->desc.bandwidth[j]);
    }
    constexpr double kArmijo = 1e-4;
    double q[kMaxDim], g[kMaxDim], H[kMaxDim * kMaxDim], f = 0.0;
    for (int j = 0; j < d; ++j) q[j] = std::min(hi[j], std::max(lo[j], h_q0[j]));
    bmd_status st = eval(q, &f, g, H);
    if (st != BMD_OK) return st;
    int it = 0;
    while (it < max_iter) {
        double dir[kMaxDim];
        if (!newton_direction(d, H, g, dir)) {
            double gn = 0.0;
            for (int j = 0; j < d; ++j) gn = std::max(gn, std::fabs(g[j]));
            if (gn == 0.0) break;
            for (int j = 0; j < d; ++j) dir[j] = 0.1 * bmin * g[j] / gn;
        }
        double t = 1.0, qn[kMaxDim], fn = 0.0, gnext[kMaxDim], Hn[kMaxDim * kMaxDim];
        bool ok = false;
        for (int bt = 0; bt < 40 && !ok; ++bt, t *= 0.5) {
            double slope = 0.0;
            for (int j = 0; j < d; ++j) {
                qn[j] = std::min(hi[j], std::max(lo[j], q[j] + t * dir[j]));
                slope += g[j] * (qn[j] - q[j]);
            }
            st = eval(qn, &fn, gnext, Hn);
            if (st != BMD_OK) return st;
            ok = fn >= f + kArmijo * slope && slope >= 0.0;
        }
        if (!ok) break;
        ++it;
        double move = 0.0;
        for (int j = 0; j < d; ++j) {
            move = std::max(move, std::fabs(qn[j] - q[j]));
            q[j] = qn[j];
            g[j] = gnext[j];
        }
        std::copy(Hn, Hn + d * d, H);
        f = fn;
        if (move <= tol) break;
    }
    for (int j = 0; j < d; ++j) h_q[j] = q[j];
    *h_value = f;
    *h_iters = it;
    return BMD_OK;
}

// Value, gradient and Hessian of the problem's thin-plate spline fit at the
// design q (design coordinates); synchronises the stream.
bmd_status tps_at_design(bmd_problem* p, const double* q, double* S, double* g, double* H, hipStream_t s) {
    const int d = p->P.d;
    double u[kMaxDim], w[kMaxDim];
    for (int j = 0; j < d; ++j) {
        double lo, hi;
        axis_range(p->desc, j, &lo, &hi);
        w[j] = hi - lo;
        u[j] = (q[j] - lo) / w[j];
    }
    bmd_status st = ensure(&p->d_ws2, &p->ws2_cap, 16 * sizeof(double));
    if (st != BMD_OK) return st;
    double h[16];
    const hipError_t e = tps_at_unit(p, u, static_cast<double*>(p->d_ws2), h, s);
    if (e != hipSuccess) return fail(BMD_EDEVICE, "thin-plate spline at a point: %s", hipGetErrorString(e));
    *S = h[0];
    int k = 1 + d;
    for (int j = 0; j < d; ++j) {
        if (g) g[j] = h[1 + j] / w[j];
        for (int l = j; l < d; ++l, ++k)
            if (H) H[j * d + l] = H[l * d + j] = h[k] / (w[j] * w[l]);
    }
    return BMD_OK;
}

}  // namespace
}  // extern "C++"

bmd_status bmd_refine_smoothed(bmd_problem* p, const double* d_surface, const double* h_q0, int32_t max_iter,
                               double tol, double* h_q, double* h_value, int32_t* h_iters, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "refine_smoothed needs a grid problem");
    if (!d_surface || !h_q0 || !h_q || !h_value || !h_iters) return fail(BMD_EINVAL, "NULL pointer argument");
    if (max_iter < 0 || max_iter > 10000 || !(tol >= 0.0)) return fail(BMD_ERANGE, "max_iter or tol out of range");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto eval = [&](const double* q, double* f, double* g, double* H) {
        return smoothed_at(p, d_surface, q, f, g, H, s);
    };
    return newton_ascent(p, eval, h_q0, max_iter, tol, h_q, h_value, h_iters);
}

bmd_status bmd_smooth_tps(bmd_problem* p, const double* d_in, double lambda, double* d_out, int64_t* h_n,
                          void* stream) {
    g_err.clear();
    if (h_n) *h_n = 0;
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "thin-plate smoothing needs a grid problem");
    if (p->P.d > 3) return fail(BMD_ENOTSUP, "thin-plate splines are built for d = 1, 2, 3 (d = %d)", p->P.d);
    if (!d_in || !d_out) return fail(BMD_EINVAL, "NULL d_in or d_out");
    if (d_in == d_out) return fail(BMD_EINVAL, "d_out must not alias d_in");
    if (!std::isfinite(lambda) || lambda < 0.0) return fail(BMD_ERANGE, "lambda must be finite and >= 0");
    DeviceGuard guard(p->device);
    const TpsFitResult r = tps_fit_grid(p, d_in, lambda, d_out, static_cast<hipStream_t>(stream));
    if (h_n) *h_n = r.n;
    switch (r.code) {
        case kTpsOk: return BMD_OK;
        case kTpsCount:
            return fail(BMD_ERANGE, "%lld designs have a value; the thin-plate fit needs %d to %lld",
                        static_cast<long long>(r.n), p->P.d + 2, static_cast<long long>(kTpsMaxPoints));
        case kTpsSingular:
            return fail(BMD_ERANGE, "the designs with a value do not determine the thin-plate spline "
                                    "(they lie on a hyperplane, or the reduced system is not positive definite)");
        case kTpsNoMem: return fail(BMD_ENOMEM, "thin-plate fit of %lld designs", static_cast<long long>(r.n));
        default: return fail(BMD_EDEVICE, "thin-plate fit: %s", hipGetErrorString(r.err));
    }
}

bmd_status bmd_tps_at(bmd_problem* p, const double* h_q, double* h_value, double* h_grad, double* h_hess,
                      void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!h_q || !h_value) return fail(BMD_EINVAL, "NULL pointer argument");
    if (tps_dims(p) == 0) return fail(BMD_ESTATE, "no thin-plate fit: call bmd_smooth_tps first");
    for (int j = 0; j < p->P.d; ++j)
        if (!std::isfinite(h_q[j])) return fail(BMD_EINVAL, "q[%d] is not finite", j);
    DeviceGuard guard(p->device);
    return tps_at_design(p, h_q, h_value, h_grad, h_hess, static_cast<hipStream_t>(stream));
}

bmd_status bmd_refine_tps(bmd_problem* p, const double* h_q0, int32_t max_iter, double tol, double* h_q,
                          double* h_value, int32_t* h_iters, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!h_q0 || !h_q || !h_value || !h_iters) return fail(BMD_EINVAL, "NULL pointer argument");
    if (tps_dims(p) == 0) return fail(BMD_ESTATE, "no thin-plate fit: call bmd_smooth_tps first");
    if (max_iter < 0 || max_iter > 10000 || !(tol >= 0.0)) return fail(BMD_ERANGE, "max_iter or tol out of range");
    DeviceGuard guard(p->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto eval = [&](const double* q, double* f, double* g, double* H) { return tps_at_design(p, q, f, g, H, s); };
    return newton_ascent(p, eval, h_q0, max_iter, tol, h_q, h_value, h_iters);
}

bmd_status bmd_eval_batch(bmd_problem* const* ps, int32_t n, const uint64_t* n_draws, int32_t prec,
                          double* const* d_means, double* h_wall_ms, void* stream) {
    g_err.clear();
    if (!ps || !n_draws || !d_means) return fail(BMD_EINVAL, "NULL argument");
    if (n < 1 || n > 65536) return fail(BMD_ERANGE, "n must be in [1, 65536]");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    for (int i = 0; i < n; ++i) {
        if (!ps[i] || !d_means[i]) return fail(BMD_EINVAL, "problem or output %d is NULL", i);
        if (!ps[i]->grid) return fail(BMD_ESTATE, "problem %d has no grid", i);
        if (ps[i]->P.design_space == BMD_DESIGN_ALPHA3 || ps[i]->P.design_space == BMD_DESIGN_ALPHA4 ||
            ps[i]->P.design_space == BMD_DESIGN_NESTED3 || ps[i]->P.design_space == BMD_DESIGN_NESTED4)
            return fail(BMD_ENOTSUP, "problem %d: three- and four-population designs are not batched", i);
        if (ps[i]->device != ps[0]->device) return fail(BMD_EINVAL, "problems live on different devices");
        if (n_draws[i] == 0 || n_draws[i] > (1ull << 40)) return fail(BMD_ERANGE, "n_draws[%d] outside [1, 2^40]", i);
    }
    DeviceGuard guard(ps[0]->device);
    hipStream_t us = static_cast<hipStream_t>(stream);
    const int dev = ps[0]->device;
    int clock_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev), "device attribute");
    const int n_cu = ps[0]->n_cu;

    std::vector<BatchPlan> plan(n);
    for (int i = 0; i < n; ++i) {
        const bmd_problem* p = ps[i];
        BatchPlan& b = plan[i];
        const bool mf = use_mfma_sweep(p);
        b.key = 2 * p->P.d + (mf ? 1 : 0);
        b.G = p->P.G;
        b.M = static_cast<int64_t>(n_draws[i]);
        b.tiles = sweep_tiles(p, prec);
        b.chunk = mf ? sweep_chunk(p, prec) : 1;
        b.draw_bytes = align256(draw_workspace_bytes(p, prec, b.M));
    }
    // Groups of consecutive problems whose draws fit the memory budget: half
    // the free device memory, at most kBatchBudget.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = kBatchBudget;
    }
    size_t budget = std::min<size_t>(kBatchBudget, free_b / 2);
    if (const char* env = std::getenv("BMD_BATCH_BUDGET")) {   // bytes; small values force one problem per group
        const long long v = std::atoll(env);
        if (v > 0) budget = static_cast<size_t>(v);
    }

    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{cs};
    {
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hipError_t e = hipEventRecord(ev, us);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
        (void)hipEventDestroy(ev);
        HIP_TRY(e, "stream ordering");
    }
    // Clock and completion stamps, and per-problem item counts, for the whole batch.
    DeviceBuffer clk;
    HIP_TRY(hipMalloc(&clk.ptr, align256(sizeof(unsigned long long) * (n + 1)) + align256(sizeof(int) * n)),
            "batch clock buffer");
    unsigned long long* d_tstart = static_cast<unsigned long long*>(clk.ptr);
    unsigned long long* d_tdone = d_tstart + 1;
    int* d_left = reinterpret_cast<int*>(static_cast<char*>(clk.ptr) + align256(sizeof(unsigned long long) * (n + 1)));

    // Settings of every launch kind in the batch: tuned once per device,
    // precision and kind (on all of this batch's problems of that kind), or fixed.
    std::map<int, BatchSettings> sets;
    {
        std::vector<int> keys;
        for (const auto& b : plan)
            if (std::find(keys.begin(), keys.end(), b.key) == keys.end()) keys.push_back(b.key);
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (int key : keys) {
            const TuneKey tk{dev, prec, key};
            auto it = g_tune.find(tk);
            if (g_tune_mode == 1 && it == g_tune.end()) {
                std::vector<bmd_problem*> kp;
                std::vector<BatchPlan> kpl;
                for (int i = 0; i < n; ++i)
                    if (plan[i].key == key) {
                        kp.push_back(ps[i]);
                        kpl.push_back(plan[i]);
                    }
                BatchSettings best;
                const bmd_status st = tune_phase(kp.data(), kpl, prec, n_cu, cs, d_tstart, d_tdone, d_left, &best);
                if (st != BMD_OK) return st;
                it = g_tune.emplace(tk, best).first;
            }
            sets[key] = g_tune_mode == 1 ? it->second : BatchSettings{};
        }
    }
    for (int first = 0; first < n;) {
        int last = first;
        size_t bytes = 0;
        while (last < n && (last == first || bytes + plan[last].draw_bytes <= budget)) bytes += plan[last++].draw_bytes;
        std::vector<BatchPlan> group(plan.begin() + first, plan.begin() + last);
        bmd_status st = run_batch_group(ps + first, group, first, prec, d_means + first, n_cu, cs, d_tstart, d_tdone,
                                        d_left, first == 0, sets, true, nullptr);
        if (st != BMD_OK) return st;
        first = last;
    }
    if (h_wall_ms) {
        std::vector<unsigned long long> t(n + 1);
        HIP_TRY(hipMemcpy(t.data(), d_tstart, sizeof(unsigned long long) * (n + 1), hipMemcpyDeviceToHost),
                "batch readback");
        for (int i = 0; i < n; ++i)
            h_wall_ms[i] = t[i + 1] >= t[0] ? static_cast<double>(t[i + 1] - t[0]) / clock_khz : 0.0;
    }
    return BMD_OK;
}

bmd_status bmd_batch_autotune(int32_t mode) {
    g_err.clear();
    if (mode < 0 || mode > 2) return fail(BMD_EINVAL, "mode must be 0, 1 or 2");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (mode != 1) g_tune.clear();
    g_tune_mode = mode == 0 ? 0 : 1;
    return BMD_OK;
}

bmd_status bmd_batch_settings(int32_t prec, int32_t d, int32_t kind, int32_t* h_out) {
    g_err.clear();
    if (!h_out) return fail(BMD_EINVAL, "h_out is NULL");
    if (!valid_prec(prec)) return fail(BMD_EINVAL, "unknown precision %d", prec);
    if (d < 1 || d > kMaxDim || kind < 0 || kind > 1 || (d == 1 && kind == 1))
        return fail(BMD_ERANGE, "no launch kind (d = %d, kind = %d)", d, kind);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(TuneKey{dev, prec, 2 * d + kind});
    if (it == g_tune.end()) return fail(BMD_ESTATE, "no tuned settings for d = %d, kind = %d on device %d", d, kind, dev);
    const BatchSettings& b = it->second;
    h_out[0] = b.chunk;
    h_out[1] = b.rounds;
    h_out[2] = b.variant;
    h_out[3] = prec == BMD_FP32_COMP && kind == 1 ? (d <= 3 ? 5 : 4) - b.variant : 0;
    h_out[4] = static_cast<int32_t>(std::lround(b.ms * 1000.0));
    return BMD_OK;
}

bmd_status bmd_profile(bmd_problem* p, int32_t enable) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    DeviceGuard guard(p->device);
    if (enable && !p->ev[0])
        for (auto& e : p->ev) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    p->profiling = enable != 0;
    for (bool& u : p->ev_used) u = false;
    return BMD_OK;
}

bmd_status bmd_profile_read(bmd_problem* p, double* h_ms) {
    g_err.clear();
    if (!p || !h_ms) return fail(BMD_EINVAL, "NULL argument");
    if (!p->ev[0]) return fail(BMD_ESTATE, "profiling was never enabled");
    DeviceGuard guard(p->device);
    for (int ph = 0; ph < BMD_PROFILE_PHASES; ++ph) {
        h_ms[ph] = 0.0;
        if (!p->ev_used[ph]) continue;
        HIP_TRY(hipEventSynchronize(p->ev[2 * ph + 1]), "hipEventSynchronize");
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[2 * ph], p->ev[2 * ph + 1]), "hipEventElapsedTime");
        h_ms[ph] = ms;
    }
    return BMD_OK;
}

bmd_status bmd_draws(bmd_problem* p, uint64_t k0, uint64_t n, double* d_u, double* d_fields, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!d_u || !d_fields) return fail(BMD_EINVAL, "NULL output pointer");
    if (n == 0 || n > (1ull << 32)) return fail(BMD_ERANGE, "n must be in [1, 2^32]");
    DeviceGuard guard(p->device);
    HIP_TRY(launch_inspect_draws(p, k0, static_cast<int64_t>(n), d_u, d_fields, static_cast<hipStream_t>(stream)),
            "draw inspection kernel");
    return BMD_OK;
}

bmd_status bmd_designs(bmd_problem* p, int64_t g0, int64_t n, double* d_fields, void* stream) {
    g_err.clear();
    if (!p) return fail(BMD_EINVAL, "problem is NULL");
    if (!p->grid) return fail(BMD_ESTATE, "designs needs a grid problem");
    if (!d_fields) return fail(BMD_EINVAL, "NULL output pointer");
    if (g0 < 0 || n < 1 || g0 + n > p->P.G) return fail(BMD_ERANGE, "design range outside the grid");
    DeviceGuard guard(p->device);
    HIP_TRY(launch_inspect_designs(p, g0, n, d_fields, static_cast<hipStream_t>(stream)), "design inspection kernel");
    return BMD_OK;
}

}  // extern "C"
