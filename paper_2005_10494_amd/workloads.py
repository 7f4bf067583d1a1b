"""Seeded synthetic workloads: problem descriptors and input generators.

This module holds only inputs (problem settings, seeds, design points drawn for
the continuous form, the batch of scenarios).  It contains none of the method's
arithmetic, so both the HIP path and the CPU oracle may use it.

The paper measures on no dataset; its experiments are simulation settings
(Sec. 3).  The workloads below mirror those settings for a biomarker-cutoff
design: a 1-D cutoff grid, a 3-D grid of three correlated biomarkers, a 5-D
grid, a continuous 5-D design batch for gradients, and a batch of uneven
scenarios.  Priors: baseline effect ~ N(0, 0.1^2), extra responder effect ~
N(0.5, 0.2^2), true cutoff quantile ~ U(0.2, 0.8); n = 200 patients per arm,
so I = n/2 = 100 information units (the paper's I_3 is a quarter of the total
events, Sec. 2.1; with 400 patients all having events I_3 = 100).
"""
from __future__ import annotations

import numpy as np

STEP_PRIOR = dict(mu_b0=0.0, sd_b0=0.1, mu_b1=0.5, sd_b1=0.2, tau_lo=0.2, tau_hi=0.8)

#: grid points per axis used by the batch scenarios, indexed by d - 1
BATCH_M = (201, 64, 40, 24, 14, 10)


def base_problem(d: int, m, rho_b: float, bandwidth: float, **kw) -> dict:
    p = dict(d=d, m=list(m) if m is not None else None, q_lo=0.05, q_hi=0.95, rho_b=rho_b,
             info=100.0, alpha0=0.025, alpha_rule="fwer", alpha_fixed=(0.0, 0.0),
             effect="step", paper_a=0.0, paper_b=0.0, paper_events=80.0, width=0.0,
             bandwidth=[bandwidth] * d, gh_nodes=0, seed=0, scenario=0)
    p.update(STEP_PRIOR)
    p.update(kw)
    return p


def plain_1d() -> dict:
    """One biomarker, 201-point cutoff grid, M = 10,000 draws, bandwidth 0.02."""
    p = base_problem(1, [201], 0.0, 0.02)
    p["n_draws"] = 10_000
    return p


def plain_3d() -> dict:
    """Three biomarkers (correlation 0.3), 64^3 grid, M = 100,000, bandwidth 0.03."""
    p = base_problem(3, [64, 64, 64], 0.3, 0.03)
    p["n_draws"] = 100_000
    return p


def precision_5d() -> dict:
    """Five biomarkers (correlation 0.3), 24^5 grid, M = 200,000, bandwidth 0.03."""
    p = base_problem(5, [24] * 5, 0.3, 0.03)
    p["n_draws"] = 200_000
    return p


def grad_5d() -> dict:
    """Continuous 5-D designs, logistic indicator width 0.01, M = 1,000,000."""
    p = base_problem(5, None, 0.3, 0.03, width=0.01)
    p["n_draws"] = 1_000_000
    p["n_points"] = 4096
    return p


def alpha_design(m_alpha: int, r=0.365, m_r: int = 0, r_range=(0.05, 0.95), n_draws: int = 10_240,
                 bandwidth=(0.05, 0.0015)) -> dict:
    """The paper's own design variables for n = 2 nested populations (Sec. 3,
    condition (b): drug effect D0(r) = 0.3 - 0.1 r, I_3 = 211, Formula 10 prior
    with E = 80): the first test's level alpha_1 on an ``m_alpha``-point grid over
    [0.0005, 0.0245] (alpha_2 from the FWER boundary), at subgroup fraction
    ``r`` (m_r = 0), or on an (r_2, alpha_1) grid with ``m_r`` points of r_2 over
    ``r_range``.  M defaults to the paper's N1 = 10,240 outer draws."""
    d = 2 if m_r else 1
    p = base_problem(d, [m_r, m_alpha] if m_r else [m_alpha], 0.0, 0.0, design="alpha",
                     q_lo=0.0005, q_hi=0.0245, info=211.0, effect="paper", paper_a=0.3,
                     paper_b=0.1, paper_events=80.0)
    p["bandwidth"] = list(bandwidth) if m_r else [bandwidth[-1]]
    p["r_lo"], p["r_hi"] = (float(r_range[0]), float(r_range[1])) if m_r else (float(r), float(r))
    p["n_draws"] = n_draws
    return p


def alpha_grid() -> dict:
    """Sec. 3's two-population experiment under condition (b) as a design grid:
    r_2 over [0.05, 0.95] in steps of 0.005 (181 points) times alpha_1 over
    [0.0005, 0.0245] in steps of 0.0001 (241 points), M = 1,000,000 draws;
    smoothing sd 0.02 in r_2 and 0.0005 in alpha_1."""
    return alpha_design(241, m_r=181, r_range=(0.05, 0.95), n_draws=1_000_000, bandwidth=(0.02, 0.0005))


def alpha3_design(m: int, r2: float = 0.446, r3: float = 0.168, q_range=(0.0005, 0.0245),
                  n_draws: int = 10_240, bandwidth: float = 0.0015) -> dict:
    """Three nested populations (Sec. 3, condition (c): drug effect
    D0(r) = 0.8 - 0.6 r, I_3 = 211, Formula 10 prior with E = 80, subgroup
    fractions r_2 = 0.446 and r_3 = 0.168): an m x m grid of the first two
    levels (alpha_1, alpha_2) over ``q_range``, alpha_3 from the FWER boundary.
    Designs whose first two levels already spend alpha0 have no third level."""
    p = base_problem(2, [m, m], 0.0, bandwidth, design="alpha3", q_lo=float(q_range[0]),
                     q_hi=float(q_range[1]), info=211.0, effect="paper", paper_a=0.8, paper_b=0.6,
                     paper_events=80.0)
    p["r_lo"], p["r_hi"] = float(r2), float(r3)
    p["n_draws"] = n_draws
    return p


def alpha3_grid() -> dict:
    """Condition (c) of Sec. 3 as a design grid: alpha_1 and alpha_2 each over
    [0.0005, 0.0245] in steps of 0.00025 (97 x 97), M = 100,000 draws."""
    return alpha3_design(97, n_draws=100_000)


def alpha4_design(m: int, r2: float = 0.7, r3: float = 0.446, r4: float = 0.168, q_range=(0.0005, 0.0245),
                  n_draws: int = 10_240, bandwidth: float = 0.0015) -> dict:
    """Four nested populations (the three-threshold designs of Sec. 3) under
    condition (c)'s effects D0(r) = 0.8 - 0.6 r, I_3 = 211, Formula 10 prior
    with E = 80; fractions r = (1, 0.7, 0.446, 0.168) (condition (c)'s two
    subgroups with a wider one in front): an m x m x m grid of the first three
    levels over ``q_range``, alpha_4 from the FWER boundary.  Designs whose
    first three levels already spend alpha0 have no fourth level."""
    p = base_problem(3, [m, m, m], 0.0, bandwidth, design="alpha4", q_lo=float(q_range[0]),
                     q_hi=float(q_range[1]), info=211.0, effect="paper", paper_a=0.8, paper_b=0.6,
                     paper_events=80.0)
    p["r_lo"], p["r_hi"], p["r_4"] = float(r2), float(r3), float(r4)
    p["n_draws"] = n_draws
    return p


def alpha4_grid() -> dict:
    """Four populations as a design grid: alpha_1, alpha_2, alpha_3 each over
    [0.0005, 0.0245] in steps of 0.001 (25^3), M = 100,000 draws."""
    return alpha4_design(25, n_draws=100_000)


def nested3_design(m, q_range=(0.1, 0.9), rule: str = "fwer", n_draws: int = 100_000, bandwidth: float = 0.03,
                   **kw) -> dict:
    """Three nested populations cut from one biomarker by two cutoffs: an
    m x m grid (or m = (m0, m1)) of cutoff quantiles (q_1, q_2) over
    ``q_range``, populations all, x > Phi^-1(q_1), x > Phi^-1(q_2); the step
    prior of ``STEP_PRIOR`` with one true cutoff; designs with q_1 >= q_2 do
    not exist."""
    mm = [m, m] if np.isscalar(m) else list(m)
    p = base_problem(2, mm, 0.0, bandwidth, design="nested3", q_lo=float(q_range[0]), q_hi=float(q_range[1]),
                     alpha_rule=rule)
    p.update(kw)
    p["n_draws"] = n_draws
    return p


def nested4_design(m, q_range=(0.1, 0.9), rule: str = "fwer", n_draws: int = 100_000, bandwidth: float = 0.05,
                   **kw) -> dict:
    """Four nested populations cut from one biomarker by three cutoffs: an
    m^3 grid (or m = (m0, m1, m2)) of cutoff quantiles (q_1, q_2, q_3) over
    ``q_range``; the step prior of ``STEP_PRIOR`` with one true cutoff;
    designs outside q_1 < q_2 < q_3 (or beyond the partial-correlation and
    fraction bounds) do not exist."""
    mm = [m, m, m] if np.isscalar(m) else list(m)
    p = base_problem(3, mm, 0.0, bandwidth, design="nested4", q_lo=float(q_range[0]), q_hi=float(q_range[1]),
                     alpha_rule=rule)
    p.update(kw)
    p["n_draws"] = n_draws
    return p


def nested4_grid() -> dict:
    """Three cutoffs on one biomarker, 24^3 grid over [0.1, 0.9], M = 1e5."""
    return nested4_design(24)


def nested3_grid() -> dict:
    """Two cutoffs on one biomarker, 64 x 64 grid over [0.1, 0.9], M = 1e5."""
    return nested3_design(64)


def noisy_surface(m, seed: int = 0, nan_corner: int = 0) -> np.ndarray:
    """A seeded stand-in for an estimated grid surface (row-major over the
    axes m, axis 0 slowest): a smooth bump plus N(0, 0.02^2) noise.  With
    ``nan_corner`` = c > 0 the designs whose axis indices sum to at least
    sum(m) - c are NaN, as designs without a valid level split are."""
    m = [int(x) for x in m]
    rng = np.random.default_rng(seed)
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in m], indexing="ij"), -1).reshape(-1, len(m))
    x = idx / np.maximum(np.asarray(m) - 1, 1)
    f = 0.3 + 0.4 * np.exp(-np.sum((x - 0.6) ** 2, axis=1) / 0.1) + 0.02 * rng.standard_normal(len(x))
    if nan_corner > 0:
        f[idx.sum(axis=1) >= sum(m) - nan_corner] = np.nan
    return f


def design_points(n: int, d: int, seed: int = 1, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """Continuous design points, iid U(lo, hi)^d (cutoff quantiles)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, d))


def batch_scenarios(n: int = 256, seed: int = 2, m_scale: float = 1.0,
                    m_draws=(1e4, 1e6)) -> list:
    """Uneven scenarios: d ~ U{1..6}, per-axis grid from ``BATCH_M`` (optionally
    scaled down for tests), M log-uniform in ``m_draws``, n per arm U{100..400},
    rho_b ~ U(0, 0.5), prior means (responder effect, centre of the true-cutoff
    interval) scaled by a factor in [0.8, 1.2].  Scenario i uses Philox
    counter word ``scenario = i``."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = np.log10(m_draws[0]), np.log10(m_draws[1])
    for i in range(n):
        d = int(rng.integers(1, 7))
        m = max(2, int(round(BATCH_M[d - 1] * m_scale)))
        n_arm = int(rng.integers(100, 401))
        rho_b = float(rng.uniform(0.0, 0.5))
        f1 = 1.0 + 0.4 * (float(rng.uniform()) - 0.5)
        f2 = 1.0 + 0.4 * (float(rng.uniform()) - 0.5)
        M = int(round(10 ** rng.uniform(lo, hi)))
        p = base_problem(d, [m] * d, rho_b, 0.03, info=n_arm / 2.0, scenario=i)
        p["mu_b1"] = STEP_PRIOR["mu_b1"] * f1
        centre = 0.5 * f2
        p["tau_lo"], p["tau_hi"] = centre - 0.3, centre + 0.3
        p["n_draws"] = M
        out.append(p)
    return out
