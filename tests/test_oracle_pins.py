"""Pins of the CPU oracle against things other than itself.

Every check here compares the oracle with an independent source: values the
paper prints, published known-answer vectors, closed forms, scipy / mpmath
routines, brute force, invariants of the model, or Monte Carlo convergence to
an exactly integrated expectation.  None of them needs a GPU.
"""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, stats
from scipy.optimize import brentq
from scipy.special import ndtr, ndtri, owens_t

import oracle as O
from paper_2005_10494_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _bvn_owen(h, k, rho):
    """Phi_2 through Owen's T function (scipy), an independent identity."""
    if h == 0.0:
        h = 1e-300
    if k == 0.0:
        k = 1e-300
    sq = math.sqrt(1 - rho * rho)
    ah = (k - rho * h) / (h * sq)
    ak = (h - rho * k) / (k * sq)
    beta = 0.0 if h * k > 0 else 0.5
    return 0.5 * ndtr(h) + 0.5 * ndtr(k) - owens_t(h, ah) - owens_t(k, ak) - beta


def _mvn(cov, x):
    """scipy's MVN CDF (Genz's quasi-Monte Carlo algorithm), tight tolerances."""
    return stats.multivariate_normal.cdf(x, mean=np.zeros(len(x)), cov=cov,
                                         maxpts=200_000 * len(x), abseps=1e-9, releps=1e-9)


# ---------------------------------------------------------------- primitives

def test_philox_known_answers():
    for row in _golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = O.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_uniform_mapping_exact():
    # 52-bit integer n from the top 26 bits of two words; u = (n + 1/2) 2^-52.
    assert O.uniform52(0, 0) == 0.5 * 2.0 ** -52
    assert O.uniform52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert O.uniform52(0x80000000, 0) == 0.5 + 0.5 * 2.0 ** -52
    rng = np.random.default_rng(5)
    for wa, wb in rng.integers(0, 2 ** 32, size=(200, 2)):
        n = ((int(wa) >> 6) << 26) | (int(wb) >> 6)
        assert O.uniform52(wa, wb) == (n + 0.5) / 2.0 ** 52
        assert 0.0 < O.uniform52(wa, wb) < 1.0


def test_Phi_against_scipy_and_mpmath():
    for x in np.linspace(-37, 8, 181):
        with mpmath.workdps(40):
            ref = float(mpmath.ncdf(mpmath.mpf(float(x))))
        # relative condition number of Phi at x is about x^2 (for x << 0)
        tol = (8.0 + 2.0 * x * x) * 1.2e-16 * ref
        assert abs(O.Phi(x) - ref) <= tol
        assert abs(O.Phi(x) - ndtr(x)) <= 2 * tol
    assert abs(O.phi(1.3) - stats.norm.pdf(1.3)) < 1e-17


def test_Phiinv_roundtrip_and_scipy():
    ps = np.concatenate([10.0 ** -np.arange(1, 300, 7), np.linspace(0.01, 0.99, 99),
                         [1 - 2.0 ** -53, 2.0 ** -53, 0.5, 0.025, 0.975]])
    for p in ps:
        x = O.Phiinv(p)
        ref = ndtri(p)
        assert abs(x - ref) <= 4 * np.spacing(abs(ref)) + 1e-300, (p, x, ref)
    # against the 60-digit root of Phi(x) = p
    for p in 10.0 ** -np.arange(1, 300, 13):
        with mpmath.workdps(60):
            pm = mpmath.mpf(float(p))
            xr = float(mpmath.findroot(lambda t: mpmath.ncdf(t) - pm, mpmath.mpf(float(ndtri(p)))))
        assert abs(O.Phiinv(p) - xr) <= 2 * np.spacing(abs(xr)), p


def test_quadrature_product_cases():
    # rho_b = 0 (orthant) and rho = 0 (bvn): the integrands reduce to products
    for v in ([0.3], [0.1, -0.4], [0.0, 0.5, -1.0, 1.2]):
        ref = float(np.prod([ndtr(-x) for x in v]))
        assert abs(O.orthant(v, 0.0) - ref) < 1e-15
    assert abs(O.bvn(0.7, 0.2, 0.0) - ndtr(0.7) * ndtr(0.2)) < 4e-16


def test_bvn_against_owens_t_and_scipy():
    rng = np.random.default_rng(1)
    for _ in range(300):
        h, k = rng.uniform(-7, 5, size=2)
        rho = rng.uniform(0.0, 0.995)
        ref = _bvn_owen(h, k, rho)
        got = O.bvn(h, k, rho)
        assert abs(got - ref) <= 2e-15 + 1e-12 * ref, (h, k, rho, got, ref)
    for h, k, rho in [(0.3, -0.2, 0.6), (-1.1, -0.4, 0.97), (2.2, 2.2, 0.3), (-3.0, 1.0, 0.9)]:
        assert abs(O.bvn(h, k, rho) - _mvn([[1, rho], [rho, 1]], [h, k])) < 1e-12


def test_bvn_special_cases():
    for rho in (0.0, 0.2, 0.5, 0.9, 0.99):
        # Sheppard: Phi_2(0,0;rho) = 1/4 + asin(rho)/(2 pi)
        assert abs(O.bvn(0.0, 0.0, rho) - (0.25 + math.asin(rho) / (2 * math.pi))) < 2e-16
    assert O.bvn(1.0, math.inf, 0.5) == pytest.approx(ndtr(1.0), abs=1e-16)
    assert O.bvn(math.inf, -0.3, 0.5) == pytest.approx(ndtr(-0.3), abs=1e-16)
    assert O.bvn(-math.inf, 0.3, 0.5) == 0.0
    # symmetry in (h, k)
    assert abs(O.bvn(0.4, -1.2, 0.7) - O.bvn(-1.2, 0.4, 0.7)) < 1e-16
    # Plackett: d Phi_2 / d rho = phi_2 (central difference in mpmath-free FP64)
    h, k, rho, e = 0.3, -0.5, 0.6, 1e-5
    fd = (O.bvn(h, k, rho + e) - O.bvn(h, k, rho - e)) / (2 * e)
    assert abs(fd - O.bvn_density(h, k, rho)) < 1e-9


def test_orthant_identities():
    # rho_b = 1/2 and c = 0: 1/(d+1) (exchangeable Gaussians, probability that the
    # common factor ranks first)
    for d in range(1, 7):
        assert abs(O.orthant([0.0] * d, 0.5) - 1.0 / (d + 1)) < 1e-14
    # d = 3, c = 0: 1/8 + 3 asin(rho)/(4 pi)
    for rho in (0.1, 0.3, 0.45):
        assert abs(O.orthant([0.0] * 3, rho) - (0.125 + 3 * math.asin(rho) / (4 * math.pi))) < 1e-15
    # d = 2 reduces to a bivariate normal CDF
    for c1, c2, rho in [(0.3, -0.4, 0.3), (1.6, 1.2, 0.45), (-1.0, 2.0, 0.1)]:
        assert abs(O.orthant([c1, c2], rho) - _bvn_owen(-c1, -c2, rho)) < 1e-14
    # general d against scipy's MVN CDF (Genz) to its own accuracy
    rng = np.random.default_rng(3)
    for d in (3, 5):
        c = ndtri(rng.uniform(0.05, 0.95, d))
        cov = np.full((d, d), 0.3) + 0.7 * np.eye(d)
        ref = _mvn(cov, -c)
        assert abs(O.orthant(c, 0.3) - ref) < 1e-6 * ref   # QMC accuracy of the reference


def test_zstar_fwer_and_independent_values():
    for r in (0.05, 0.3, 0.5, 0.87, 0.95):
        z = O.zstar(r, 0.025)
        rho = math.sqrt(r)
        fwer = 1.0 - _bvn_owen(z, z, rho)
        assert abs(fwer - 0.025) < 1e-14
        # bracketing: one-test value <= z* <= Bonferroni value
        assert ndtri(0.975) <= z <= ndtri(1 - 0.0125)
    # independent root with scipy brentq on Owen's T
    z_ref = brentq(lambda z: 1 - _bvn_owen(z, z, math.sqrt(0.5)) - 0.025, 1.0, 6.0, xtol=1e-15)
    assert abs(O.zstar(0.5) - z_ref) < 1e-12


def test_info_units_paper_values():
    rows = {r[0]: r for r in _golden("paper_values.txt")}
    for key, delta in (("info_units_delta_0.25", 0.25), ("info_units_delta_0.20", 0.20)):
        val, tol = float(rows[key][1]), float(rows[key][2])
        assert abs(O.info_units(0.025, 0.1, delta) - val) <= tol


# ---------------------------------------------------------------- model

def test_grid_points_bit_exact_and_row_major():
    p = W.base_problem(3, [4, 5, 7], 0.3, 0.03)
    G = O.grid_size(p)
    assert G == 140
    for g in range(G):
        q, idx = O.grid_point(p, g)
        assert tuple(idx) == np.unravel_index(g, (4, 5, 7))
        for j, m in enumerate((4, 5, 7)):
            t = (0.95 - 0.05) * float(idx[j])
            t = t / float(m - 1)
            assert q[j] == 0.05 + t       # same operation order, so bit-equal
    q_last, _ = O.grid_point(p, G - 1)
    assert np.all(np.abs(q_last - 0.95) <= np.spacing(0.95))


def test_draw_uniforms_from_philox():
    p = W.plain_3d()
    k = 123456789012
    dr = O.make_draw(p, k)
    words = np.concatenate([O.philox([k & 0xFFFFFFFF, k >> 32, 0, b], [0, 0]) for b in range(3)])
    for i in range(5):
        assert dr["u"][i] == O.uniform52(words[2 * i], words[2 * i + 1])
    assert dr["b0"] == pytest.approx(0.0 + 0.1 * ndtri(dr["u"][0]), abs=1e-16)
    assert dr["b1"] == pytest.approx(0.5 + 0.2 * ndtri(dr["u"][1]), abs=1e-16)
    for j in range(3):
        assert dr["tau"][j] == 0.2 + (0.8 - 0.2) * dr["u"][2 + j]
    assert dr["PR"] == pytest.approx(_mvn(np.full((3, 3), 0.3) + 0.7 * np.eye(3), -dr["t"]), rel=5e-6)


def _degenerate_reference(q, tau, b0, b1, info=100.0):
    """Closed form for d = 1, zero prior variance and a fixed true cutoff,
    computed with scipy only."""
    r = 1.0 - q
    rho = math.sqrt(r)
    z = brentq(lambda z: 1 - _bvn_owen(z, z, rho) - 0.025, 1.0, 6.0, xtol=1e-15)
    PR, Ov = 1 - tau, 1 - max(q, tau)
    mu1 = math.sqrt(info) * (b0 + b1 * PR)
    mu2 = math.sqrt(r * info) * (b0 + b1 * Ov / r)
    return 1.0 - _bvn_owen(z - mu1, z - mu2, rho), z


def test_degenerate_prior_closed_form():
    p = W.plain_1d()
    for q, tau in [(0.5, 0.5), (0.3, 0.6), (0.8, 0.4)]:
        p.update(sd_b0=0.0, sd_b1=0.0, tau_lo=tau, tau_hi=tau, mu_b0=0.0, mu_b1=0.5)
        ref, z = _degenerate_reference(q, tau, 0.0, 0.5)
        for k in (0, 7, 99):
            assert abs(O.success(p, [q], k) - ref) < 1e-13
        assert abs(O.make_design(p, [q])["z1"] - z) < 1e-12
    # independently computed value at q = tau = 1/2
    p.update(tau_lo=0.5, tau_hi=0.5)
    assert abs(O.success(p, [0.5], 0) - 0.921493500270) < 5e-13


def test_null_prior_gives_alpha0_pathwise():
    # no effect at all: every design and every draw succeeds with probability
    # exactly alpha0 under the equal-FWER rule (Formula 2)
    for base in (W.plain_1d(), W.base_problem(3, [5, 5, 5], 0.3, 0.03)):
        p = dict(base)
        p.update(mu_b0=0.0, sd_b0=0.0, mu_b1=0.0, sd_b1=0.0)
        G = O.grid_size(p)
        for g in np.linspace(0, G - 1, 7).astype(int):
            q, _ = O.grid_point(p, g)
            for k in (0, 1, 2):
                assert abs(O.success(p, q, k) - 0.025) < 2e-15


def test_overlap_definition_brute_force():
    # O = P(X in S and X in R) against scipy's MVN CDF of the max cutoffs
    p = W.base_problem(3, [8, 8, 8], 0.3, 0.03)
    cov = np.full((3, 3), 0.3) + 0.7 * np.eye(3)
    for k in range(4):
        dr = O.make_draw(p, k)
        q = np.array([0.3, 0.55, 0.8])
        v = np.maximum(ndtri(q), dr["t"])
        assert O.overlap(p, q, k) == pytest.approx(_mvn(cov, -v), rel=5e-6)
    # d = 1 with a logistic width: 1 - (s q + (1-s) tau)
    p1 = W.plain_1d()
    p1["width"] = 0.01
    dr = O.make_draw(p1, 3)
    s = 1 / (1 + math.exp(-(0.5 - dr["tau"][0]) / 0.01))
    assert O.overlap(p1, [0.5], 3) == pytest.approx(1 - (s * 0.5 + (1 - s) * dr["tau"][0]), abs=1e-15)


def test_monotone_in_prior_means_and_alpha():
    q = [0.4, 0.6]
    p = W.base_problem(2, [5, 5], 0.3, 0.03)
    base = [O.success(p, q, k) for k in range(20)]
    for key in ("mu_b0", "mu_b1"):
        pp = dict(p)
        pp[key] += 0.05
        up = [O.success(pp, q, k) for k in range(20)]
        assert all(u > b for u, b in zip(up, base))
    pa = dict(p)
    pa["alpha0"] = 0.05
    assert all(O.success(pa, q, k) > b for k, b in enumerate(base))


def test_symmetry_under_axis_permutation_with_draws():
    p = W.base_problem(3, [5, 5, 5], 0.3, 0.03)
    q = np.array([0.25, 0.5, 0.7])
    perm = [2, 0, 1]
    for k in range(5):
        dr = O.make_draw(p, k)
        dr_p = dict(dr)
        dr_p["tau"] = dr["tau"][perm]
        dr_p["t"] = dr["t"][perm]
        a = O.success_with_draw(p, q, dr)
        b = O.success_with_draw(p, q[perm], dr_p)
        assert abs(a - b) < 1e-15
        assert 0.0 <= a <= 1.0


def test_exact_mode_degenerate_and_independent_values():
    p = W.plain_1d()
    # degenerate prior: exact expectation is the closed form itself
    pd = dict(p)
    pd.update(sd_b0=0.0, sd_b1=0.0, tau_lo=0.6, tau_hi=0.6)
    ref, _ = _degenerate_reference(0.3, 0.6, 0.0, 0.5)
    assert abs(O.exact_step(pd, [0.3]) - ref) < 1e-13
    # independently computed values (scipy Owen's T + Gauss-Legendre)
    assert abs(O.exact_step(p, [0.05 + 0.9 * 127 / 200]) - 0.702030122778) < 2e-12
    p2 = W.base_problem(2, [5, 5], 0.3, 0.03)
    assert abs(O.exact_step(p2, [0.5, 0.5]) - 0.501076392069) < 2e-12


def test_mc_converges_to_exact_at_inverse_sqrt_M():
    """RMS error of the oracle's Monte Carlo estimate over 10 seeds falls like
    M^-1/2 toward the exactly integrated expectation, and the errors are
    consistent with the CLT standard error (the corrected form of the paper's
    precision claim for Formula 5)."""
    p = W.plain_1d()
    q = [0.6]
    exact = O.exact_step(p, q)
    Ms = [1000, 10000, 100000]
    rms = []
    zs = []
    for M in Ms:
        errs = []
        for seed in range(10):
            pp = dict(p)
            pp["seed"] = seed
            m, v = O.eval_points(pp, np.array([q]), M)
            errs.append(m[0] - exact)
            zs.append((m[0] - exact) / math.sqrt(v[0] / M))
        rms.append(math.sqrt(np.mean(np.square(errs))))
    slope = np.polyfit(np.log10(Ms), np.log10(rms), 1)[0]
    assert -0.75 < slope < -0.3, (slope, rms)
    assert np.max(np.abs(zs)) < 4.5
    assert 0.4 < np.std(zs) < 1.6


def test_paper_prior_closed_form_and_printed_case_a():
    # Formula 10 with Delta0 = 0.25 everywhere, I_3 = 127, alpha = (0.025, 0):
    # the n = 1 limit of Sec. 3 case (a).  Closed form with scipy only:
    I = 127.0
    theta = -math.log(0.75)
    sig2 = 1.0 / 20.0
    closed = 1.0 - ndtr((ndtri(0.975) - math.sqrt(I) * theta) / math.sqrt(1 + I * sig2))
    p = W.plain_1d()
    p.update(effect="paper", paper_a=0.25, paper_b=0.0, paper_events=80.0, info=I,
             alpha_rule="fixed", alpha_fixed=(0.025, 0.0))
    assert abs(O.exact_paper(p, [0.5]) - closed) < 1e-14
    rows = {r[0]: r for r in _golden("paper_values.txt")}
    printed, tol = float(rows["case_a_best_power"][1]), float(rows["case_a_best_power"][2])
    assert abs(closed - printed) <= tol
    m, v = O.eval_points(p, np.array([[0.5]]), 20000)
    assert abs(m[0] - closed) < 4 * math.sqrt(v[0] / 20000)
    assert abs(m[0] - printed) <= tol


def test_paper_prior_two_populations_closed_form():
    # n = 2 nested populations under Formula 10: (1 + I/20) Sigma structure
    # (Sigma_p = Sigma_Z / 20 after scaling by D), so
    # P = 1 - Phi_2((z - D theta) / sqrt(1 + I/20); sqrt(r)).
    I, a, b = 211.0, 0.3, 0.1
    q = 0.635
    r = 1 - q
    p = W.plain_1d()
    p.update(effect="paper", paper_a=a, paper_b=b, paper_events=80.0, info=I)
    ds = O.make_design(p, [q])
    th1, th2 = -math.log(1 - (a - b)), -math.log(1 - (a - b * r))
    s = math.sqrt(1 + I / 20.0)
    h = (ds["z1"] - math.sqrt(I) * th1) / s
    k = (ds["z2"] - math.sqrt(r * I) * th2) / s
    closed = 1.0 - _bvn_owen(h, k, math.sqrt(r))
    assert abs(O.exact_paper(p, [q]) - closed) < 1e-13


# ---------------------------------------------------------------- smoothing

def test_smoothing_properties():
    p = W.base_problem(3, [6, 7, 5], 0.3, 0.03)
    p["bandwidth"] = [0.1, 0.2, 0.15]
    G = O.grid_size(p)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.2, 0.8, G)
    a = O.smooth_direct(p, f)
    b = O.smooth_separable(p, f)
    assert np.max(np.abs(a - b)) < 1e-14
    c = O.smooth_separable(p, np.full(G, 0.37))
    assert np.max(np.abs(c - 0.37)) < 1e-15
    # bandwidth -> 0 gives the identity
    p0 = dict(p)
    p0["bandwidth"] = [1e-4] * 3
    assert np.max(np.abs(O.smooth_separable(p0, f) - f)) < 1e-14
    # a surface symmetric under axis reversal stays symmetric
    ps = W.base_problem(2, [9, 9], 0.3, 0.05)
    f2 = rng.uniform(size=(9, 9))
    f2 = f2 + f2[::-1, ::-1]
    s2 = O.smooth_separable(ps, f2.ravel()).reshape(9, 9)
    assert np.max(np.abs(s2 - s2[::-1, ::-1])) < 1e-15
    # values stay within the input range (weights are positive and sum to one)
    assert a.min() >= f.min() - 1e-15 and a.max() <= f.max() + 1e-15


def test_smoothing_brute_force_1d():
    p = W.plain_1d()
    G = 201
    f = np.sin(np.linspace(0, 3, G))
    q = 0.05 + 0.9 * np.arange(G) / 200
    K = np.exp(-0.5 * ((q[:, None] - q[None, :]) / 0.02) ** 2)
    ref = (K @ f) / K.sum(1)
    assert np.max(np.abs(O.smooth_separable(p, f) - ref)) < 1e-14


def test_argmax_ties_lowest_index():
    assert O.argmax(np.array([0.1, 0.5, 0.5, 0.2])) == 1
    assert O.argmax(np.array([3.0])) == 0
    v = np.random.default_rng(2).uniform(size=1000)
    assert O.argmax(v) == int(np.argmax(v))


# ---------------------------------------------------------------- gradients

@pytest.mark.parametrize("d,width", [(1, 0.01), (2, 0.01), (3, 0.0), (5, 0.01)])
def test_gradient_matches_central_differences(d, width):
    p = W.base_problem(d, None, 0.3, 0.03, width=width)
    q = W.design_points(1, d, seed=11)[0]
    M = 400 if d < 5 else 200
    obj, gq, gmu = O.grad_points(p, q, M)
    # with the exact indicator the Monte Carlo objective has a kink wherever a
    # drawn true cutoff tau_j equals q_j; a small step keeps those out of the window
    h = 1e-4 if width > 0 else 1e-6
    for j in range(d):
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        fp = O.eval_points(p, qp, M, want_var=False)[0]
        fm = O.eval_points(p, qm, M, want_var=False)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(gq[0, j] - fd) <= 1e-6 + 1e-4 * abs(fd), (j, gq[0, j], fd)
    for i, key in enumerate(("mu_b0", "mu_b1")):
        pp, pm = dict(p), dict(p)
        pp[key] += h
        pm[key] -= h
        fd = (O.eval_points(pp, q, M, want_var=False)[0] - O.eval_points(pm, q, M, want_var=False)[0]) / (2 * h)
        assert abs(gmu[0, i] - fd) <= 1e-7 + 1e-5 * abs(fd), (key, gmu[0, i], fd)
    assert abs(obj[0] - O.eval_points(p, q, M, want_var=False)[0]) < 1e-15


def test_gradient_zero_under_null_prior():
    p = W.base_problem(3, None, 0.3, 0.03, width=0.01)
    p.update(mu_b0=0.0, sd_b0=0.0, mu_b1=0.0, sd_b1=0.0)
    obj, gq, gmu = O.grad_points(p, np.array([0.3, 0.5, 0.6]), 50)
    assert abs(obj[0] - 0.025) < 1e-14
    assert np.max(np.abs(gq)) < 1e-12
    assert np.all(gmu > 0)


# ---------------------------------------------------------------- alpha design space
# The paper's own design variables for n = 2 nested populations (Sec. 2.2-2.3):
# the first test's level alpha_1, with alpha_2 on the FWER boundary of Formula 2.

def _z2_scipy(z1, r, alpha0=0.025):
    """Second critical value from scipy: brentq on the FWER through Owen's T."""
    rho = math.sqrt(r)
    a1 = ndtr(-z1)
    f = lambda z2: a1 + ndtr(-z2) - _bvn_owen(-z1, -z2, rho) - alpha0  # noqa: E731
    return brentq(f, -ndtri(alpha0) - 1.0, -ndtri(alpha0 - a1) + 1.0, xtol=1e-14)


def _alpha_power_scipy(a1, r, I=211.0, a=0.3, b=0.1):
    """Condition (b) of Sec. 3 under Formula 10 (E = 80), closed form with scipy:
    P = 1 - Phi_2((z - D theta) / sqrt(1 + I/20); sqrt r)."""
    z1 = -ndtri(a1)
    z2 = _z2_scipy(z1, r)
    th1, th2 = -math.log(1 - (a - b)), -math.log(1 - (a - b * r))
    s = math.sqrt(1 + I / 20.0)
    return 1.0 - _bvn_owen((z1 - math.sqrt(I) * th1) / s, (z2 - math.sqrt(r * I) * th2) / s, math.sqrt(r))


def test_alpha_design_second_level_on_fwer_boundary():
    for r in (0.1, 0.365, 0.8):
        for a1 in (0.001, 0.0125, 0.024):
            z1 = -ndtri(a1)
            z2 = O.z2_fwer(z1, r)
            assert abs(z2 - _z2_scipy(z1, r)) < 1e-10, (r, a1)
            fwer = a1 + ndtr(-z2) - _bvn_owen(-z1, -z2, math.sqrt(r))
            assert abs(fwer - 0.025) < 1e-13
            # union bound and single-test bound bracket the second level
            assert 0.025 - a1 - 1e-15 <= ndtr(-z2) <= 0.025
    assert O.z2_fwer(-ndtri(0.025), 0.5) == math.inf


def test_alpha_design_condition_b_optimum():
    """At r_2 = 0.365 (the subgroup size of the paper's condition (b) optimum)
    the optimal level split maximises a closed form; the oracle's design
    quantities, its closed-form power and the maximiser of its surface agree
    with scipy's."""
    from scipy.optimize import minimize_scalar
    r = 0.365
    p = W.alpha_design(97, r=r)
    res = minimize_scalar(lambda x: -_alpha_power_scipy(x, r), bounds=(0.005, 0.024), method="bounded",
                          options={"xatol": 1e-9})
    a_star, p_star = res.x, -res.fun
    ds = O.make_design(p, [a_star])
    assert ds["r"] == r and abs(ds["z1"] + ndtri(a_star)) < 1e-12
    assert abs(ds["z2"] - _z2_scipy(ds["z1"], r)) < 1e-10
    assert abs(O.exact_paper(p, [a_star]) - p_star) < 1e-12
    grid = np.linspace(0.012, 0.020, 161)
    best = grid[int(np.argmax([O.exact_paper(p, [x]) for x in grid]))]
    assert abs(best - a_star) <= 0.5 * (grid[1] - grid[0]) + 1e-12
    # the optimum sits inside (0, alpha0) with both tests on: sum of levels > alpha0
    assert 0.012 < a_star < 0.02 and a_star + ndtr(-ds["z2"]) > 0.025


def test_alpha_design_limits_and_monte_carlo():
    r = 0.365
    p = W.alpha_design(5, r=r)
    I, th1 = 211.0, -math.log(1 - 0.2)
    s = math.sqrt(1 + I / 20.0)
    # alpha_1 = alpha0: the second test is off (z2 = +inf) and the power is the
    # one-population closed form of Sec. 3's condition (a) type
    one = 1.0 - ndtr((-ndtri(0.025) - math.sqrt(I) * th1) / s)
    assert O.make_design(p, [0.025])["z2"] == math.inf
    assert abs(O.exact_paper(p, [0.025]) - one) < 1e-13
    # the power is continuous there only through z2 -> inf, which is slow: the
    # prior's spread keeps the second test useful at tiny levels
    assert O.exact_paper(p, [0.025 * (1 - 1e-9)]) > one
    # Formula 5 on the oracle's draws converges to the closed form
    M = 20000
    q = np.array([[0.005], [0.0159], [0.022]])
    m, v = O.eval_points(p, q, M)
    for i in range(3):
        ex = O.exact_paper(p, q[i])
        assert abs(m[i] - ex) < 4 * math.sqrt(v[i] / M), (q[i], m[i], ex)


def test_alpha_design_grid_and_smoothing():
    p = W.alpha_design(6, m_r=5, r_range=(0.2, 0.8))
    G = O.grid_size(p)
    assert G == 30
    for g in range(G):
        q, idx = O.grid_point(p, g)
        assert tuple(idx) == np.unravel_index(g, (5, 6))
        assert q[0] == 0.2 + ((0.8 - 0.2) * float(idx[0])) / 4
        assert q[1] == 0.0005 + ((0.0245 - 0.0005) * float(idx[1])) / 5
        assert O.make_design(p, q)["r"] == q[0]
    f = np.random.default_rng(5).uniform(0.5, 0.8, G)
    assert np.max(np.abs(O.smooth_direct(p, f) - O.smooth_separable(p, f))) < 1e-14


# ---------------------------------------------------------------- derivative in alpha_1
# Appendix A.3 differentiates the power under the integral; for the nested pair
# the oracle's chain rule runs through z1 and, under the split rule, through the
# second level on the FWER boundary.

def _one_level_spec(rule, a1, a2=0.0, **kw):
    p = W.base_problem(2, [5, 4], 0.3, 0.05, alpha_rule=rule, alpha_fixed=(a1, a2))
    p.update(kw)
    return p


@pytest.mark.parametrize("rule,a2", [("split", 0.0), ("fixed", 0.015), ("fixed", 0.0)])
def test_dalpha_is_the_derivative_of_the_estimate(rule, a2):
    """On fixed draws the estimate is one smooth function of alpha_1: its
    central differences (step 1e-6, the second level re-solved on the boundary
    under "split") match the chain-rule derivative.  Dropping the dz2/dz1 term,
    a sign, or phi(z1)'s factor misses by orders of magnitude."""
    a1, h, M = 0.01, 1e-6, 300
    g = np.arange(20)
    m, d = O.eval_grid_dalpha(_one_level_spec(rule, a1, a2), g, M)
    mp, _ = O.eval_grid(_one_level_spec(rule, a1 + h, a2), g, M)
    mm, _ = O.eval_grid(_one_level_spec(rule, a1 - h, a2), g, M)
    m0, _ = O.eval_grid(_one_level_spec(rule, a1, a2), g, M)
    assert np.array_equal(m, m0)
    cd = (mp - mm) / (2 * h)
    assert np.max(np.abs(d - cd) / np.maximum(np.abs(cd), 1.0)) < 1e-6, (d, cd)
    assert np.max(np.abs(d)) > 0.1


def _point_mass_power(a1, r, I, a, b, rule, a2=0.0):
    """A prior with all its mass at one effect (E -> infinity in Formula 10):
    the power 1 - Phi_2(z1 - sqrt(I) theta_1, z2 - sqrt(r I) theta_2; sqrt r)
    with scipy's Owen's T and brentq for the boundary."""
    z1 = -ndtri(a1)
    z2 = _z2_scipy(z1, r) if rule == "split" else (-ndtri(a2) if a2 > 0 else math.inf)
    th1, th2 = -math.log(1 - (a - b)), -math.log(1 - (a - b * r))
    h, k = z1 - math.sqrt(I) * th1, z2 - math.sqrt(r * I) * th2
    if math.isinf(k):
        return 1.0 - ndtr(h)
    return 1.0 - _bvn_owen(h, k, math.sqrt(r))


@pytest.mark.parametrize("rule,a2", [("split", 0.0), ("fixed", 0.0), ("fixed", 0.02)])
def test_dalpha_point_mass_prior_exact(rule, a2):
    """With (almost) no prior spread every draw is the same effect, so the
    estimate's derivative is the closed-form power's, differentiated here by
    central differences of the scipy expression (step 1e-6)."""
    I, a, b = 211.0, 0.3, 0.1
    p = W.base_problem(1, [3], 0.0, 0.05, q_lo=0.535, q_hi=0.735, info=I, effect="paper", paper_a=a,
                       paper_b=b, paper_events=1e18, alpha_rule=rule, alpha_fixed=(0.01, a2))
    r = O.make_design(p, O.grid_point(p, 1)[0])["r"]
    m, d = O.eval_grid_dalpha(p, [1], 64)
    hh = 1e-6
    ref = (_point_mass_power(0.01 + hh, r, I, a, b, rule, a2) - _point_mass_power(0.01 - hh, r, I, a, b, rule, a2)) / (2 * hh)
    assert abs(m[0] - _point_mass_power(0.01, r, I, a, b, rule, a2)) < 1e-7
    assert abs(d[0] - ref) <= 1e-6 * max(abs(ref), 1.0), (d[0], ref)


def test_dalpha_one_test_closed_form_appendix_a3():
    """Appendix A.3's one-test form: with the second test off, dP/d alpha =
    E[phi(z - mu1)] / phi(z); under Formula 10 mu1 ~ N(sqrt(I) theta_1, I/20)
    (E = 80), so E[phi(z - mu1)] = phi((z - m)/s)/s with s^2 = 1 + I/20.  The
    estimate over 2e5 draws is within 6 standard errors (from 10 blocks)."""
    I, a, b = 211.0, 0.3, 0.1
    p = W.base_problem(1, [3], 0.0, 0.05, info=I, effect="paper", paper_a=a, paper_b=b, paper_events=80.0,
                       alpha_rule="fixed", alpha_fixed=(0.01, 0.0))
    z = -ndtri(0.01)
    m1 = math.sqrt(I) * -math.log(1 - (a - b))
    s = math.sqrt(1 + I / 20.0)
    pdf = lambda x: math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)  # noqa: E731
    closed = pdf((z - m1) / s) / (s * pdf(z))
    blocks = [O.eval_grid_dalpha(p, [1], 20_000, k0=20_000 * i)[1][0] for i in range(10)]
    se = np.std(blocks, ddof=1) / math.sqrt(len(blocks))
    assert abs(np.mean(blocks) - closed) < 6 * se, (np.mean(blocks), closed, se)
    assert se < 0.02 * closed


def test_dalpha_split_rule_converges_to_closed_form():
    """Under the split rule and Formula 10 (condition (b), r = 0.365) the
    estimate's derivative converges to the derivative of the closed-form power
    (scipy, central differences): within 6 standard errors over 2e5 draws."""
    p = W.base_problem(1, [3], 0.0, 0.05, q_lo=0.535, q_hi=0.735, info=211.0, effect="paper", paper_a=0.3,
                       paper_b=0.1, paper_events=80.0, alpha_rule="split", alpha_fixed=(0.008, 0.0))
    r = O.make_design(p, O.grid_point(p, 1)[0])["r"]
    hh = 1e-6
    ref = (_alpha_power_scipy(0.008 + hh, r) - _alpha_power_scipy(0.008 - hh, r)) / (2 * hh)
    blocks = [O.eval_grid_dalpha(p, [1], 20_000, k0=20_000 * i)[1][0] for i in range(10)]
    se = np.std(blocks, ddof=1) / math.sqrt(len(blocks))
    assert abs(np.mean(blocks) - ref) < 6 * se, (np.mean(blocks), ref, se)
    assert se < 0.05 * abs(ref)


def test_newton_level_search_finds_the_derivative_root():
    """The oracle's false-position search on fixed draws: where it stops
    inside the range the estimate's derivative is zero to 1e-6 (the probe with
    the largest estimate, which rounding picks among a few equal ones) and the level
    beats its neighbours at +-1e-4; it agrees with the golden-section search's
    maximum (80 steps) to 1e-12 in power; a design whose derivative keeps one
    sign over the range ends at that end."""
    spec = W.base_problem(2, [5, 4], 0.3, 0.05)
    g = np.arange(20)
    M = 300
    best, x = O.optimize_levels_newton(spec, g, M, 0.001, 0.024, 40, 1e-12)
    gb, gx = O.optimize_levels(spec, g, M, 0.001, 0.024, 80)
    assert np.all(np.abs(best - gb) <= 1e-12 * np.maximum(1.0, np.abs(gb)))
    inside = (x > 0.001) & (x < 0.024)
    assert inside.sum() >= 5
    for i in np.nonzero(inside)[0][:6]:
        sp = dict(spec, alpha_rule="split", alpha_fixed=(float(x[i]), 0.0))
        m, d = O.eval_grid_dalpha(sp, [g[i]], M)
        assert abs(m[0] - best[i]) <= 1e-15 and abs(d[0]) < 1e-6, (i, d[0])
        for dx in (-1e-4, 1e-4):
            mn, _ = O.eval_grid(dict(sp, alpha_fixed=(float(x[i]) + dx, 0.0)), [g[i]], M)
            assert mn[0] < best[i]
        assert abs(x[i] - gx[i]) < 1e-5
    for i in np.nonzero(~inside)[0]:
        assert abs(x[i] - gx[i]) < 1e-9


# ---------------------------------------------------------------- two cutoffs on one biomarker
# Three nested populations cut from one biomarker (n = 3 in the cutoff design
# space): all, x > Phi^-1(q_1), x > Phi^-1(q_2).

@pytest.mark.parametrize("r2,r3", [(0.8, 0.5), (0.6, 0.15), (0.9, 0.85), (0.3, 0.1)])
def test_nested3_zstar_on_fwer_boundary(r2, r3):
    z = O.zstar3(r2, r3)
    fwer = 1.0 - _tvn_scipy([z, z, z], math.sqrt(r2), math.sqrt(r3), math.sqrt(r3 / r2))
    assert abs(fwer - 0.025) < 2e-8, (r2, r3, z, fwer)
    assert -ndtri(0.025) < z < -ndtri(0.025 / 3)


def test_nested3_designs_and_null_prior():
    """Designs exist only for q_1 < q_2 within the partial-correlation bound;
    under a null prior (no effect) every existing design rejects with
    probability alpha0 exactly (FWER-equal rule) or 1 - Phi_3 at the
    Bonferroni value (scipy)."""
    spec = W.nested3_design(6, mu_b0=0.0, sd_b0=0.0, mu_b1=0.0, sd_b1=0.0)
    G = O.grid_size(spec)
    m, _ = O.eval_grid(spec, np.arange(G), 20)
    n_ok = 0
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        r2, r3 = 1 - q[0], 1 - q[1]
        exists = q[0] < q[1] and r3 * (1 - r2) <= 0.975 ** 2 * r2 * (1 - r3)
        assert np.isnan(m[g]) == (not exists), (g, q)
        if exists:
            n_ok += 1
            assert abs(m[g] - 0.025) < 1e-9, (g, m[g])
    assert n_ok >= 10
    bon = dict(spec, alpha_rule="bonferroni")
    mb, _ = O.eval_grid(bon, np.arange(G), 5)
    g = 3   # q = (0.1, 0.74)
    q, _ = O.grid_point(bon, g)
    zb = -ndtri(0.025 / 3)
    ref = 1.0 - _tvn_scipy([zb] * 3, math.sqrt(1 - q[0]), math.sqrt(1 - q[1]), math.sqrt((1 - q[1]) / (1 - q[0])))
    assert abs(mb[g] - ref) < 2e-8, (mb[g], ref)


def test_nested3_one_draw_against_a_simulated_trial():
    """One draw (no prior spread, the true cutoff fixed) computed from the
    definitions by simulation: the responders inside each population from 4e6
    simulated biomarker values, the drifts sqrt(r_i I) Delta_i, and the
    rejection probability P(some Z_i > z*) from 4e6 draws of the three
    statistics with the nested correlations; the oracle's summand is within 5
    standard errors."""
    tau = 0.35
    spec = W.nested3_design(5, mu_b0=0.05, sd_b0=0.0, mu_b1=0.45, sd_b1=0.0, tau_lo=tau, tau_hi=tau)
    g = 1 * 5 + 3   # q = (0.3, 0.7)
    q, _ = O.grid_point(spec, g)
    m, _ = O.eval_grid(spec, [g], 3)
    ds = O.make_design(spec, q)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(4_000_000)
    resp = x > ndtri(tau)
    I = spec["info"]
    mu, r = [], []
    for c in (None, ndtri(q[0]), ndtri(q[1])):
        inside = np.ones_like(x, dtype=bool) if c is None else x > c
        ri = inside.mean()
        delta = 0.05 + 0.45 * (resp & inside).mean() / ri
        mu.append(math.sqrt(ri * I) * delta)
        r.append(ri)
    R = np.array([[1, math.sqrt(r[1]), math.sqrt(r[2])], [math.sqrt(r[1]), 1, math.sqrt(r[2] / r[1])],
                  [math.sqrt(r[2]), math.sqrt(r[2] / r[1]), 1]])
    Z = rng.multivariate_normal(mu, R, size=4_000_000)
    hit = (Z > ds["z1"]).any(axis=1)
    p, se = hit.mean(), hit.std() / math.sqrt(hit.size)
    assert abs(m[0] - p) < 5 * se + 2e-4, (m[0], p, se)


# ---------------------------------------------------------------- two-layer estimator
# Formula 7 (the inner layer of Formula 6) and its variance, Appendix A.2
# corrected: the inner draws are shared by every outer draw, so the estimate's
# variance keeps the covariance terms A.2 drops.

def _two_layer_brute(spec, g, N1, N2, A, B):
    """Formula 7 restated with the scalar primitives: outer normals from
    make_draw, inner normals from Philox counters (l, 0, scenario, 2^31 | b)
    and the quantile, the nested chain, the thresholds, the block counts."""
    n = {"alpha3": 3, "alpha4": 4}.get(spec.get("design"), 2)
    ds = O.make_design(spec, O.grid_point(spec, g)[0])
    r = [1.0, ds["r"], ds["r3"], ds["r4"]][:n]
    z = [ds["z1"], ds["z2"], ds["z3"], ds["z4"]][:n]
    key = [spec["seed"] & 0xFFFFFFFF, spec["seed"] >> 32]
    x = np.zeros((N2, n))
    for l in range(N2):
        w = np.concatenate([O.philox([l, 0, spec["scenario"], 0x80000000 | b], key) for b in range(2)])
        for i in range(n):
            e = O.Phiinv(O.uniform52(w[2 * i], w[2 * i + 1]))
            x[l, i] = e if i == 0 else math.sqrt(r[i] / r[i - 1]) * x[l, i - 1] + math.sqrt(1 - r[i] / r[i - 1]) * e
    cnt = np.zeros((A, B), dtype=np.int64)
    for k in range(N1):
        dr = O.make_draw(spec, k)
        e = [dr["e1"], dr["e2"], dr["e3"], dr["e4"]]
        Y, b = [], []
        for i in range(n):
            Y.append(e[0] if i == 0 else math.sqrt(r[i] / r[i - 1]) * Y[i - 1] + math.sqrt(1 - r[i] / r[i - 1]) * e[i])
            th = -math.log1p(-(spec["paper_a"] - spec["paper_b"] * r[i]))
            sg = 1.0 / math.sqrt(spec["paper_events"] * r[i] / 4.0)
            b.append(z[i] - math.sqrt(r[i] * spec["info"]) * (th + sg * Y[i]))
        below = np.all(x <= np.array(b), axis=1)
        for bb in range(B):
            cnt[k // (N1 // A), bb] += int(below[bb * (N2 // B):(bb + 1) * (N2 // B)].sum())
    return cnt


@pytest.mark.parametrize("which", ["alpha", "alpha3", "alpha4"])
def test_two_layer_counts_restated(which):
    spec = {"alpha": W.alpha_design(5), "alpha3": W.alpha3_design(3), "alpha4": W.alpha4_design(2)}[which]
    g = 1 if which != "alpha4" else 0
    N1, N2, A, B = 24, 96, 4, 2
    m, v, blk = O.eval_grid_two_layer(spec, [g], N1, N2, A, B)
    cnt = _two_layer_brute(spec, g, N1, N2, A, B)
    assert np.array_equal(blk[0].astype(np.int64), cnt)
    assert m[0] == 1.0 - cnt.sum() / (N1 * N2)
    assert 0 < cnt.sum() < N1 * N2


def _one_test_parts(I, E, a, z):
    """One test under Formula 10 (second test off): h = [x <= z - mu],
    mu ~ N(m, s^2), x ~ N(0, 1).  theta = E h = Phi(w), w = (z - m)/sqrt(1 + s^2);
    Var_mu E_x h = Phi_2(w, w; s^2/(1 + s^2)) - theta^2;
    Var_x E_mu h = Phi_2(w, w; 1/(1 + s^2)) - theta^2."""
    m = math.sqrt(I) * -math.log(1 - a)
    s2 = I * 4.0 / E
    w = (z - m) / math.sqrt(1 + s2)
    th = ndtr(w)
    return th, _bvn_owen(w, w, s2 / (1 + s2)) - th * th, _bvn_owen(w, w, 1 / (1 + s2)) - th * th


def test_two_layer_variance_closed_form():
    """The one-test case has the Hoeffding parts in closed form, so the
    variance of Formula 7's estimate is s1/N1 + s2/N2 + (theta(1-theta) - s1 -
    s2)/(N1 N2) exactly.  Over 40 independent replications (seeds) the
    oracle's block estimate of that variance averages to it within 4 standard
    errors, the replications' own spread matches it (chi-square 99.9%), and
    their mean matches 1 - theta; at the paper's N1 = 10240, N2 = 20480 the
    exact variance exceeds Appendix A.2's bound 1/(4 N1 N2) by orders of
    magnitude."""
    from scipy.stats import chi2
    I, E, a, a1 = 211.0, 80.0, 0.3, 0.01
    spec = W.base_problem(1, [3], 0.0, 0.05, info=I, effect="paper", paper_a=a, paper_b=0.0, paper_events=E,
                          alpha_rule="fixed", alpha_fixed=(a1, 0.0))
    z = -ndtri(a1)
    th, s1, s2 = _one_test_parts(I, E, a, z)
    N1, N2, A, B, R = 256, 512, 8, 8, 40
    exact = s1 / N1 + s2 / N2 + (th * (1 - th) - s1 - s2) / (N1 * N2)
    means, vars_ = [], []
    for sd in range(R):
        m, v, _ = O.eval_grid_two_layer(dict(spec, seed=1000 + sd), [1], N1, N2, A, B)
        means.append(m[0])
        vars_.append(v[0])
    means, vars_ = np.array(means), np.array(vars_)
    assert abs(vars_.mean() - exact) < 4 * vars_.std(ddof=1) / math.sqrt(R), (vars_.mean(), exact)
    ratio = means.var(ddof=1) / exact
    assert chi2.ppf(0.0005, R - 1) / (R - 1) < ratio < chi2.ppf(0.9995, R - 1) / (R - 1), ratio
    assert abs(means.mean() - (1 - th)) < 4 * math.sqrt(exact / R)
    big = s1 / 10240 + s2 / 20480
    assert big > 1000 * 1 / (4 * 10240 * 20480)


@pytest.mark.parametrize("which", ["alpha", "alpha3", "alpha4"])
def test_two_layer_converges_to_formula5(which):
    """On the same outer draws the inner layer averages to Phi_Sigma (Formula 6
    is unbiased for it), so Formula 7 minus Formula 5 is the inner draws'
    error: within 5 of its standard errors from the inner groups' spread (the
    groups are independent replicates of the inner layer given the outer
    draws)."""
    spec = {"alpha": W.alpha_design(5), "alpha3": W.alpha3_design(3), "alpha4": W.alpha4_design(2)}[which]
    g = 1 if which != "alpha4" else 0
    N1, N2, A, B = 256, 16384, 4, 16
    m, v, blk = O.eval_grid_two_layer(spec, [g], N1, N2, A, B)
    det, _ = O.eval_grid(spec, [g], N1)
    colmeans = 1 - blk[0].sum(axis=0) / (N1 * N2 / B)
    se = colmeans.std(ddof=1) / math.sqrt(B)
    assert abs(m[0] - det[0]) < 5 * se, (m[0], det[0], se)
    assert 0 < se < 0.01


# ---------------------------------------------------------------- continuous refinement

def test_refinement_reaches_the_maximiser_of_a_deterministic_objective():
    """With a point-mass prior (sd 0, fixed true cutoff) every draw is the same,
    so the objective is one deterministic function of the cutoff; the refinement
    from the grid's edge must reach the maximiser scipy finds on that function."""
    from scipy.optimize import minimize_scalar
    p = W.base_problem(1, None, 0.0, 0.05, width=0.02, sd_b0=0.0, sd_b1=0.0, tau_lo=0.55, tau_hi=0.55,
                       mu_b1=0.6)
    f = lambda x: float(O.eval_points(p, np.array([[x]]), 1, want_var=False)[0])  # noqa: E731
    res = minimize_scalar(lambda x: -f(x), bounds=(0.05, 0.95), method="bounded", options={"xatol": 1e-8})
    q, fq, it = O.refine_design(p, [0.2], 4, max_iter=200, tol=1e-9)
    assert 1 <= it < 200
    assert abs(q[0] - res.x) < 2e-5, (q, res.x)
    assert fq >= -res.fun - 1e-10
    # the objective's gradient vanishes there (interior maximum)
    _, g, _ = O.grad_points(p, q[None, :], 1)
    assert abs(g[0, 0]) < 1e-3


def test_refinement_climbs_and_stays_in_the_box():
    p = W.base_problem(2, None, 0.3, 0.05, width=0.01)
    M = 600
    q0 = np.array([0.15, 0.85])
    f0 = float(O.grad_points(p, q0[None, :], M)[0][0])
    q, fq, it = O.refine_design(p, q0, M, max_iter=30, tol=1e-7)
    assert it >= 1 and fq > f0
    assert np.all(q >= 0.05) and np.all(q <= 0.95)
    # a start on the box edge with the gradient pointing out stays on the edge
    qe, _, _ = O.refine_design(dict(p, q_hi=0.5), np.array([0.5, 0.5]), M, max_iter=5)
    assert np.all(qe <= 0.5)


# ---------------------------------------------------------------- optimal level split (f2)

def test_split_rule_at_the_equal_split_is_the_fwer_equal_rule():
    p = W.base_problem(1, [3], 0.0, 0.05, q_lo=0.5, q_hi=0.7)
    r = 0.4
    z = O.zstar(r)
    ps = dict(p, alpha_rule="split", alpha_fixed=(float(ndtr(-z)), 0.0))
    ds = O.make_design(ps, [0.6])
    assert abs(ds["r"] - r) < 1e-15 and abs(ds["z1"] - z) < 1e-12 and abs(ds["z2"] - z) < 1e-9
    m_eq, _ = O.eval_grid(p, np.array([1]), 3000)
    m_sp, _ = O.eval_grid(ps, np.array([1]), 3000)
    assert abs(m_eq[0] - m_sp[0]) < 1e-9


def test_level_surface_matches_closed_form_under_point_mass_prior():
    """Point-mass step prior (no Monte Carlo noise): at q = 0.6 with true cutoff
    0.3 the drifts are sqrt(I) b1 P(R) and sqrt(r I) b1 P(R and S)/r, and the
    power for each level split is 1 - Phi_2(z1 - mu1, z2 - mu2; sqrt r) with z2
    from scipy's FWER root; the level surface is its maximum over the list."""
    p = W.base_problem(1, [3], 0.0, 0.05, q_lo=0.5, q_hi=0.7, sd_b0=0.0, sd_b1=0.0, tau_lo=0.3, tau_hi=0.3)
    r, I = 0.4, 100.0
    mu1 = math.sqrt(I) * 0.5 * 0.7
    mu2 = math.sqrt(r * I) * 0.5 * 0.4 / r
    alphas = np.linspace(0.001, 0.024, 47)
    power = []
    for a1 in alphas:
        z1 = -ndtri(a1)
        z2 = _z2_scipy(z1, r)
        power.append(1.0 - _bvn_owen(z1 - mu1, z2 - mu2, math.sqrt(r)))
    best, k = O.eval_grid_levels(p, np.array([1]), 2, alphas)
    assert abs(best[0] - max(power)) < 1e-12
    assert k[0] == int(np.argmax(power))
    # an interior optimum: both tests keep part of the level
    assert 0 < k[0] < len(alphas) - 1


def test_level_search_reaches_scipy_optimum_under_point_mass_prior():
    """Per-design search of the level split (Sec. 2.4's optimal power at each
    design) under the point-mass prior of the level-surface pin: the searched
    level and power agree with scipy's bounded maximiser of the closed form, and
    the searched power is at least the best of a fine level grid."""
    from scipy.optimize import minimize_scalar
    p = W.base_problem(1, [3], 0.0, 0.05, q_lo=0.5, q_hi=0.7, sd_b0=0.0, sd_b1=0.0, tau_lo=0.3, tau_hi=0.3)
    r, I = 0.4, 100.0
    mu1 = math.sqrt(I) * 0.5 * 0.7
    mu2 = math.sqrt(r * I) * 0.5 * 0.4 / r

    def power(a1):
        z1 = -ndtri(a1)
        return 1.0 - _bvn_owen(z1 - mu1, _z2_scipy(z1, r) - mu2, math.sqrt(r))

    res = minimize_scalar(lambda x: -power(x), bounds=(0.001, 0.024), method="bounded", options={"xatol": 1e-10})
    best, x = O.optimize_levels(p, np.array([1]), 2, 0.001, 0.024, 30)
    assert abs(x[0] - res.x) < 2e-6, (x[0], res.x)
    assert abs(best[0] + res.fun) < 1e-11
    grid_best, _ = O.eval_grid_levels(p, np.array([1]), 2, np.linspace(0.001, 0.024, 47))
    assert best[0] >= grid_best[0] - 1e-15
    # a boundary optimum: with the search range cut below the interior optimum
    # the search ends exactly at the range's upper end
    b2, x2 = O.optimize_levels(p, np.array([1]), 2, 0.001, 0.5 * res.x, 30)
    assert x2[0] == 0.5 * res.x and abs(b2[0] - power(x2[0])) < 1e-12


# ---------------------------------------------------------------- three nested populations

def _tvn_scipy(h, r12, r13, r23):
    cov = np.array([[1.0, r12, r13], [r12, 1.0, r23], [r13, r23, 1.0]])
    return stats.multivariate_normal.cdf(np.asarray(h, dtype=float), mean=np.zeros(3), cov=cov,
                                         abseps=1e-11, releps=1e-11, maxpts=20_000_000)


def test_trivariate_cdf_against_scipy_and_closed_forms():
    for h, r in [((0.3, -0.5, 1.2), (0.6, 0.4, 0.67)), ((2.0, 1.5, 1.8), (0.8, 0.5, 0.62)),
                 ((-1.0, 0.7, 0.2), (0.3, -0.2, 0.1)), ((1.96, 2.2, 2.4), (0.67, 0.41, 0.61))]:
        assert abs(O.tvn(*h, *r) - _tvn_scipy(h, *r)) < 2e-8, (h, r)
    # independent coordinates: a product
    h = (0.4, -0.3, 1.1)
    assert abs(O.tvn(*h, 0.0, 0.0, 0.0) - ndtr(0.4) * ndtr(-0.3) * ndtr(1.1)) < 1e-14
    # an infinite bound drops a coordinate: the bivariate CDF (Owen's T)
    assert abs(O.tvn(0.5, -0.2, math.inf, 0.45, 0.3, 0.2) - _bvn_owen(0.5, -0.2, 0.45)) < 1e-14
    # equicorrelated orthant: 1/8 + 3 asin(rho) / (4 pi)
    for rho in (0.2, 0.5, 0.8):
        assert abs(O.tvn(0.0, 0.0, 0.0, rho, rho, rho) - (0.125 + 3 * math.asin(rho) / (4 * math.pi))) < 1e-13


def test_paper_case_c_printed_power():
    """Condition (c) of Sec. 3 at its printed optimum (three populations,
    printed levels): the Formula 10 closed form through the trivariate CDF
    reproduces the printed best power 0.977."""
    r = [1.0, 0.446, 0.168]
    a = [0.00194, 0.0135, 0.0133]
    I = 211.0
    s = math.sqrt(1 + I / 20.0)
    h = [(-ndtri(a[i]) - math.sqrt(r[i] * I) * (-math.log(1 - (0.8 - 0.6 * r[i])))) / s for i in range(3)]
    R = (math.sqrt(r[1]), math.sqrt(r[2]), math.sqrt(r[2] / r[1]))
    p = 1.0 - O.tvn(*h, *R)
    assert abs(p - (1.0 - _tvn_scipy(h, *R))) < 2e-8
    rows = {row[0]: row for row in _golden("paper_values.txt")}
    printed, tol = float(rows["case_c_best_power"][1]), float(rows["case_c_best_power"][2])
    assert abs(p - printed) <= tol


def _alpha3(**kw):
    p = W.base_problem(2, [5, 5], 0.0, 0.002, design="alpha3", q_lo=0.001, q_hi=0.02, info=211.0,
                       effect="paper", paper_a=0.8, paper_b=0.6, paper_events=80.0)
    p.update(r_lo=0.446, r_hi=0.168)
    p.update(kw)
    return p


def test_alpha3_third_level_on_fwer_boundary():
    p = _alpha3()
    r2, r3 = 0.446, 0.168
    R = (math.sqrt(r2), math.sqrt(r3), math.sqrt(r3 / r2))
    for a1, a2 in [(0.002, 0.013), (0.01, 0.005), (0.0005, 0.0005)]:
        ds = O.make_design(p, [a1, a2])
        assert ds["r"] == r2 and ds["r3"] == r3
        z = (ds["z1"], ds["z2"], ds["z3"])
        assert abs(z[0] + ndtri(a1)) < 1e-12 and abs(z[1] + ndtri(a2)) < 1e-12
        assert abs((1.0 - _tvn_scipy(z, *R)) - 0.025) < 2e-8
    # the first two levels already spend alpha0: no valid third level
    assert math.isnan(O.make_design(p, [0.02, 0.01])["z3"])


def test_alpha3_draws_and_monte_carlo():
    p = _alpha3()
    p2 = W.alpha_design(5)
    for k in (0, 7, 12345):
        d3, d2 = O.make_draw(p, k), O.make_draw(p2, k)
        assert d3["e1"] == d2["e1"] and d3["e2"] == d2["e2"]   # same first two normals
        assert abs(d3["e3"] - ndtri(d3["u"][2])) < 1e-12
    M = 20000
    q = np.array([[0.002, 0.013], [0.008, 0.008], [0.001, 0.002]])
    m, v = O.eval_points(p, q, M)
    for i in range(len(q)):
        ex = O.exact_paper(p, q[i])
        assert abs(m[i] - ex) < 4 * math.sqrt(v[i] / M), (q[i], m[i], ex)


def _masked_surface(spec, seed):
    G = O.grid_size(spec)
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.2, 0.9, G)
    m = spec["m"]
    idx = np.array([O.grid_point(spec, g)[1] for g in range(G)])
    f[idx[:, 0] + idx[:, 1] >= m[0] + m[1] - 4] = np.nan   # a corner without values, as infeasible levels give
    return f


def test_masked_smoother_pins():
    """NaN-masked smoothing over the designs that have a value (Sec. 2.3's fit
    over the evaluated points): pinned to the separable smoother through the
    ratio of smoothed values and smoothed indicator, to the identity as the
    bandwidth vanishes, to constants, to the mean of the valid values as the
    bandwidth grows, and to the unmasked smoother without NaN."""
    spec = W.alpha3_design(7)
    spec["bandwidth"] = [0.004, 0.006]
    f = _masked_surface(spec, 3)
    nan = np.isnan(f)
    assert 0 < nan.sum() < f.size
    out = O.smooth_masked(spec, f)
    assert np.array_equal(np.isnan(out), nan)
    f0, v = np.where(nan, 0.0, f), (~nan).astype(float)
    ratio = O.smooth_separable(spec, f0) / O.smooth_separable(spec, v)
    assert np.max(np.abs(out[~nan] - ratio[~nan])) < 1e-13
    # constants on the valid designs stay constant
    c = np.where(nan, np.nan, 0.37)
    assert np.max(np.abs(O.smooth_masked(spec, c)[~nan] - 0.37)) < 1e-15
    # vanishing bandwidth: the identity
    tiny = dict(spec, bandwidth=[1e-6, 1e-6])
    assert np.max(np.abs(O.smooth_masked(tiny, f)[~nan] - f[~nan])) < 1e-15
    # huge bandwidth: the mean over the valid designs
    wide = dict(spec, bandwidth=[1e5, 1e5])
    assert np.max(np.abs(O.smooth_masked(wide, f)[~nan] - np.mean(f[~nan]))) < 1e-12
    # without NaN it is the plain smoother
    g = np.where(nan, 0.5, f)
    assert np.max(np.abs(O.smooth_masked(spec, g) - O.smooth_direct(spec, g))) < 1e-15


# ---------------------------------------------------------------- four nested populations

def _qvn_scipy(h, R):
    """scipy's four-variate normal CDF: a randomised quasi-Monte Carlo estimate
    (Genz), seeded so that the pins are deterministic; over seeds its error at
    4e6 points spreads with a standard deviation near 1e-7, so the pins that
    use it compare at 5e-7."""
    f = stats.multivariate_normal(mean=np.zeros(4), cov=np.asarray(R), seed=20200521)
    f.maxpts, f.abseps, f.releps = 4_000_000, 1e-9, 1e-9
    return f.cdf(np.asarray(h, dtype=float))


def _nested_R(r):
    return np.array([[math.sqrt(min(a, b) / max(a, b)) for b in r] for a in r])


def test_four_variate_cdf_against_scipy_and_closed_forms():
    """or_qvn (conditioning on the first coordinate through Phi_3, any
    correlation matrix) against scipy's MVN CDF and closed forms; the
    nested-population form or_qvn_nested (two 1-D integrals over the chain's
    middle statistics) against or_qvn and scipy."""
    rng = np.random.default_rng(11)
    A = rng.normal(size=(4, 6))
    C = A @ A.T
    R = C / np.sqrt(np.outer(np.diag(C), np.diag(C)))
    h = rng.normal(0.5, 1.0, 4)
    assert abs(O.qvn(h, R) - _qvn_scipy(h, R)) < 5e-7, (h, R)
    # equicorrelated orthant at rho = 1/2: 1/(n + 1)
    R = np.full((4, 4), 0.5)
    np.fill_diagonal(R, 1.0)
    assert abs(O.qvn(np.zeros(4), R) - 0.2) < 1e-13
    # equicorrelated, any bounds: the one-factor identity
    rho = 0.3
    R = np.full((4, 4), rho)
    np.fill_diagonal(R, 1.0)
    h = np.array([0.3, -0.5, 1.1, 0.2])
    f = lambda z: math.exp(-z * z / 2) / math.sqrt(2 * math.pi) * np.prod(ndtr((h - math.sqrt(rho) * z) / math.sqrt(1 - rho)))
    ref = integrate.quad(f, -np.inf, np.inf, epsabs=1e-14, epsrel=1e-14)[0]
    assert abs(O.qvn(h, R) - ref) < 1e-13
    # two independent pairs: a product of bivariate CDFs (Owen's T)
    R = np.eye(4)
    R[0, 1] = R[1, 0] = 0.6
    R[2, 3] = R[3, 2] = -0.4
    h = np.array([0.2, 1.0, -0.3, 0.8])
    assert abs(O.qvn(h, R) - _bvn_owen(0.2, 1.0, 0.6) * _bvn_owen(-0.3, 0.8, -0.4)) < 1e-13
    # an infinite bound drops a coordinate: the trivariate CDF
    r = [1.0, 0.6, 0.35, 0.2]
    Rn = _nested_R(r)
    h = np.array([0.4, 0.9, math.inf, -0.2])
    assert abs(O.qvn(h, Rn) - O.tvn(0.4, 0.9, -0.2, Rn[0, 1], Rn[0, 3], Rn[1, 3])) < 1e-13
    # nested chain form against the generic one and scipy, with finite and
    # infinite middle bounds
    for r, h in (([1.0, 0.6, 0.35, 0.2], [0.9, 1.4, 0.2, 1.7]), ([1.0, 0.9, 0.5, 0.45], [1.9, 0.1, 0.8, 0.6]),
                 ([1.0, 0.2, 0.05, 0.01], [-0.4, 2.1, 1.0, 0.3])):
        h = np.array(h)
        Rn = _nested_R(r)
        g = O.qvn(h, Rn)
        assert abs(O.qvn_nested(h, np.array(r)) - g) < 1e-13, (r, h)
        assert abs(g - _qvn_scipy(h, Rn)) < 5e-7
    r = np.array([1.0, 0.6, 0.35, 0.2])
    for j in (1, 2):
        h = np.array([0.4, 0.9, 0.1, -0.2])
        h[j] = math.inf
        assert abs(O.qvn_nested(h, r) - O.qvn(h, _nested_R(r))) < 1e-13


def _alpha4(**kw):
    p = W.alpha4_design(5)
    p.update(kw)
    return p


def test_alpha4_fourth_level_on_fwer_boundary():
    p = _alpha4()
    r = [1.0, p["r_lo"], p["r_hi"], p["r_4"]]
    R = _nested_R(r)
    for n, a in enumerate([(0.002, 0.004, 0.006), (0.008, 0.003, 0.001), (0.0005, 0.0005, 0.0005)]):
        ds = O.make_design(p, list(a))
        assert ds["r"] == r[1] and ds["r3"] == r[2] and ds["r4"] == r[3]
        z = (ds["z1"], ds["z2"], ds["z3"], ds["z4"])
        for i in range(3):
            assert abs(z[i] + ndtri(a[i])) < 1e-12
        assert abs((1.0 - _qvn_scipy(z, R)) - 0.025) < 5e-7
        if n == 0:   # through the generic CDF too (it takes seconds)
            assert abs((1.0 - O.qvn(np.array(z), R)) - 0.025) < 1e-12
    # the first three levels already spend alpha0: no valid fourth level
    assert math.isnan(O.make_design(p, [0.02, 0.015, 0.01])["z4"])


def test_alpha4_draws_and_monte_carlo():
    """The first three normals are the three-population draws; the estimate
    of Formula 5 stays within 4 CLT sd of the Formula 10 closed form."""
    p = _alpha4()
    p3 = W.alpha3_design(5)
    for k in (0, 7, 12345):
        d4, d3 = O.make_draw(p, k), O.make_draw(p3, k)
        assert d4["e1"] == d3["e1"] and d4["e2"] == d3["e2"] and d4["e3"] == d3["e3"]
        assert abs(d4["e4"] - ndtri(d4["u"][3])) < 1e-12
    M = 3000
    q = np.array([[0.002, 0.004, 0.006], [0.006, 0.006, 0.002]])
    m, v = O.eval_points(p, q, M)
    for i in range(len(q)):
        ex = O.exact_paper(p, q[i])
        assert abs(m[i] - ex) < 4 * math.sqrt(v[i] / M), (q[i], m[i], ex)


def test_alpha4_closed_form_against_scipy():
    """The Formula 10 closed form for four populations, 1 - Phi_4 at the
    standardised critical values, against scipy's MVN CDF."""
    p = _alpha4()
    r = [1.0, p["r_lo"], p["r_hi"], p["r_4"]]
    I = p["info"]
    s = math.sqrt(1 + 4 * I / p["paper_events"])
    for a in [(0.002, 0.004, 0.006), (0.006, 0.006, 0.002)]:
        ds = O.make_design(p, list(a))
        z = [ds["z1"], ds["z2"], ds["z3"], ds["z4"]]
        h = [(z[i] - math.sqrt(r[i] * I) * (-math.log(1 - (0.8 - 0.6 * r[i])))) / s for i in range(4)]
        assert abs(O.exact_paper(p, np.array(a)) - (1.0 - _qvn_scipy(h, _nested_R(r)))) < 5e-7


def test_smoothed_surface_at_continuous_designs():
    """The oracle's Nadaraya-Watson sum at a continuous design: at grid designs
    it is the masked smoother's value (and the direct one without NaN), a
    constant stays constant, a huge bandwidth gives the mean of the valid
    values, and swapping the axes of a symmetric surface and point leaves it."""
    spec = W.base_problem(2, [9, 9], 0.3, 0.08)
    f = W.noisy_surface([9, 9], seed=2)
    f[:3] = np.nan
    sm = O.smooth_masked(spec, f)
    for g in (10, 40, 80):
        q, _ = O.grid_point(spec, g)
        assert abs(O.smooth_at(spec, f, q) - sm[g]) < 1e-14
    c = np.where(np.isnan(f), np.nan, 0.42)
    assert abs(O.smooth_at(spec, c, [0.33, 0.71]) - 0.42) < 1e-15
    wide = dict(spec, bandwidth=[1e5, 1e5])
    assert abs(O.smooth_at(wide, f, [0.2, 0.6]) - np.nanmean(f)) < 1e-12
    s = W.noisy_surface([9, 9], seed=3).reshape(9, 9)
    s = (s + s.T).ravel()
    assert abs(O.smooth_at(spec, s, [0.3, 0.6]) - O.smooth_at(spec, s, [0.6, 0.3])) < 1e-14


# ------------------------------------------------------------ thin-plate spline (Sec. 2.3)

_TPS_KERNEL = {1: "cubic", 2: "thin_plate_spline", 3: "linear"}   # scipy's names for r^3, r^2 log r, -r


@pytest.mark.parametrize("d,m", [(1, [40]), (2, [12, 9]), (3, [6, 5, 7])])
@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.1])
def test_tps_matches_scipy_rbf(d, m, lam):
    """The oracle's spline against scipy's radial-basis interpolator with the
    same kernel, a linear polynomial and the same smoothing (it adds lam to the
    kernel matrix's diagonal), on the unit-box coordinates."""
    from scipy.interpolate import RBFInterpolator
    spec = W.base_problem(d, m, 0.3, 0.05)
    f = W.noisy_surface(m, seed=3)
    fit = O.tps_fit(spec, f, lam)
    q = O.grid_points(spec, np.arange(O.grid_size(spec)))
    u = O.tps_unit(spec, q)
    rng = np.random.default_rng(5)
    qx = spec["q_lo"] + (spec["q_hi"] - spec["q_lo"]) * rng.random((50, d))
    rbf = RBFInterpolator(u, f, kernel=_TPS_KERNEL[d], smoothing=lam, degree=1)
    assert np.max(np.abs(O.tps_value(spec, fit, q) - rbf(u))) < 1e-10
    assert np.max(np.abs(O.tps_value(spec, fit, qx) - rbf(O.tps_unit(spec, qx)))) < 1e-10


@pytest.mark.parametrize("d,m", [(1, [30]), (2, [9, 11]), (3, [5, 6, 4])])
def test_tps_interpolation_planes_and_least_squares(d, m):
    """lam = 0 interpolates; a plane is reproduced exactly for any lam (the
    polynomial part carries it, c = 0); a huge lam leaves the least-squares
    plane."""
    spec = W.base_problem(d, m, 0.3, 0.05)
    G = O.grid_size(spec)
    q = O.grid_points(spec, np.arange(G))
    f = W.noisy_surface(m, seed=4)
    assert np.max(np.abs(O.smooth_tps(spec, f, 0.0) - f)) < 1e-9
    plane = 0.3 + q @ np.linspace(0.5, -0.7, d)
    for lam in (0.0, 0.05, 10.0):
        fit = O.tps_fit(spec, plane, lam)
        assert np.max(np.abs(fit[1])) < 1e-9
        assert np.max(np.abs(O.tps_value(spec, fit, q) - plane)) < 1e-12
    u = O.tps_unit(spec, q)
    X = np.hstack([np.ones((G, 1)), u])
    ls = X @ np.linalg.lstsq(X, f, rcond=None)[0]
    assert np.max(np.abs(O.smooth_tps(spec, f, 1e9) - ls)) < 1e-6


def test_tps_skips_designs_without_a_value():
    """Designs whose value is NaN stay NaN and do not enter the fit: the fit
    equals scipy's on the designs that have a value."""
    from scipy.interpolate import RBFInterpolator
    spec = W.base_problem(2, [10, 12], 0.3, 0.05)
    f = W.noisy_surface([10, 12], seed=6, nan_corner=5)
    s = O.smooth_tps(spec, f, 0.01)
    nan = np.isnan(f)
    assert np.array_equal(np.isnan(s), nan) and nan.sum() > 0
    u = O.tps_unit(spec, O.grid_points(spec, np.arange(f.size)))
    rbf = RBFInterpolator(u[~nan], f[~nan], kernel="thin_plate_spline", smoothing=0.01, degree=1)
    assert np.max(np.abs(s[~nan] - rbf(u[~nan]))) < 1e-10


@pytest.mark.parametrize("d,m", [(1, [25]), (2, [9, 8]), (3, [5, 4, 6])])
def test_tps_derivatives_by_central_differences(d, m):
    """Gradient and Hessian in design coordinates against central differences
    of the (scipy-pinned) value, away from the centres."""
    spec = W.base_problem(d, m, 0.3, 0.05)
    f = W.noisy_surface(m, seed=7)
    fit = O.tps_fit(spec, f, 1e-3)
    rng = np.random.default_rng(8)
    w = spec["q_hi"] - spec["q_lo"]
    for _ in range(5):
        q = spec["q_lo"] + w * (0.1 + 0.8 * rng.random(d))
        v, g, H = O.tps_derivatives(spec, fit, q)
        assert abs(v - O.tps_value(spec, fit, q[None, :])[0]) < 1e-13
        h = 1e-5 * w
        for j in range(d):
            e = np.zeros(d)
            e[j] = h
            vp = O.tps_derivatives(spec, fit, q + e)
            vm = O.tps_derivatives(spec, fit, q - e)
            assert abs((vp[0] - vm[0]) / (2 * h) - g[j]) < 1e-6 * max(1.0, np.abs(g).max())
            assert np.max(np.abs((vp[1] - vm[1]) / (2 * h) - H[j])) < 1e-4 * max(1.0, np.abs(H).max())


# ------------------------------------------------------------ three cutoffs on one biomarker (n = 4)

@pytest.mark.parametrize("r", [(0.7, 0.45, 0.2), (0.85, 0.5, 0.3), (0.5, 0.3, 0.12)])
def test_nested4_zstar_on_fwer_boundary(r):
    """z* against scipy's four-variate normal CDF of the nested correlations:
    the FWER at alpha0 within the seeded estimator's accuracy, inside the
    one-test and Bonferroni bounds."""
    z = O.zstar4(*r)
    rr = [1.0, *r]
    fwer = 1.0 - _qvn_scipy([z] * 4, _nested_R(rr))
    assert abs(fwer - 0.025) < 5e-7, (r, z, fwer)
    assert -ndtri(0.025) < z < -ndtri(0.025 / 4)


def test_nested4_designs_and_null_prior():
    """Designs exist only for q_1 < q_2 < q_3 within the partial-correlation
    and fraction bounds; under a null prior every existing design rejects with
    probability alpha0 (FWER-equal rule), and at the Bonferroni value with
    scipy's 1 - Phi_4."""
    spec = W.nested4_design(5, mu_b0=0.0, sd_b0=0.0, mu_b1=0.0, sd_b1=0.0)
    G = O.grid_size(spec)
    m, _ = O.eval_grid(spec, np.arange(G), 4)
    n_ok = 0
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        r2, r3, r4 = 1 - q[0], 1 - q[1], 1 - q[2]
        exists = (q[0] < q[1] < q[2] and r3 * (1 - r2) <= 0.975 ** 2 * r2 * (1 - r3)
                  and r4 * (r2 - r3) <= 0.975 ** 2 * r3 * (r2 - r4) and r3 <= 0.95 * r2)
        assert np.isnan(m[g]) == (not exists), (g, q)
        if exists:
            n_ok += 1
            assert abs(m[g] - 0.025) < 1e-9, (g, m[g])
    assert n_ok >= 4
    bon = dict(spec, alpha_rule="bonferroni")
    g = int(np.nonzero(~np.isnan(m))[0][0])
    mb, _ = O.eval_grid(bon, [g], 2)
    q, _ = O.grid_point(bon, g)
    zb = -ndtri(0.025 / 4)
    ref = 1.0 - _qvn_scipy([zb] * 4, _nested_R([1.0, 1 - q[0], 1 - q[1], 1 - q[2]]))
    assert abs(mb[0] - ref) < 5e-7, (mb[0], ref)


def test_nested4_one_draw_against_a_simulated_trial():
    """One draw (fixed effects and true cutoff) from the definitions by
    simulation: each population's fraction and responders from 4e6 biomarker
    values, the drifts sqrt(r_i I) Delta_i, and P(some Z_i > z*) from 4e6 draws
    of the four statistics with the nested correlations; the oracle's summand
    is within 5 standard errors."""
    tau = 0.45
    spec = W.nested4_design(5, mu_b0=0.05, sd_b0=0.0, mu_b1=0.45, sd_b1=0.0, tau_lo=tau, tau_hi=tau)
    G = O.grid_size(spec)
    cand = [g for g in range(G) if np.allclose(O.grid_point(spec, g)[0], [0.1, 0.5, 0.7])]
    g = cand[0]
    q, _ = O.grid_point(spec, g)
    m, _ = O.eval_grid(spec, [g], 2)
    ds = O.make_design(spec, q)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(4_000_000)
    resp = x > ndtri(tau)
    I = spec["info"]
    mu, r = [], []
    for c in (None, ndtri(q[0]), ndtri(q[1]), ndtri(q[2])):
        inside = np.ones_like(x, dtype=bool) if c is None else x > c
        ri = inside.mean()
        mu.append(math.sqrt(ri * I) * (0.05 + 0.45 * (resp & inside).mean() / ri))
        r.append(ri)
    R = _nested_R(r)
    Z = rng.multivariate_normal(mu, R, size=4_000_000)
    hit = (Z > ds["z4"]).any(axis=1)
    p, se = hit.mean(), hit.std() / math.sqrt(hit.size)
    assert abs(m[0] - p) < 5 * se + 2e-4, (m[0], p, se)
