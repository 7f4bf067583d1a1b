"""The paper's own design variables on the GPU: for two nested populations
(Sec. 2.2-2.3), the first test's level alpha_1 with alpha_2 on the FWER
boundary of Formula 2, over alpha_1 alone or an (r_2, alpha_1) grid, under the
Formula 10 prior of Sec. 3's condition (b).  Through the C ABI against the
oracle on the same draws (bars as in test_gpu_parity: FP64 1e-9, FP32 1e-5,
relative to max(|f|, 1e-3); grid coordinates bit-exact; critical values
1e-12), and against the closed form of the prior within Monte Carlo error."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2005_10494_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2005_10494_amd as bmd  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(got, ref, prec, what):
    bound = TOL[prec] * np.maximum(np.abs(ref), 1e-3)
    err = np.abs(np.asarray(got) - ref)
    w = int(np.argmax(err / bound))
    assert np.all(err <= bound), f"{what} {prec}: index {w} got {got[w]!r} ref {ref[w]!r}"


@pytest.mark.parametrize("spec", [W.alpha_design(49), W.alpha_design(23, m_r=17)])
def test_alpha_designs_and_critical_values(spec):
    say(f"alpha designs d={spec['d']} m={spec['m']}")
    with bmd.Problem(spec) as p:
        G = p.G
        f = p.designs(0, G).cpu().numpy()
        assert bmd.sweep_kind(p) == "direct"
    d = spec["d"]
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        assert np.array_equal(f[g, :d], q), g
        ds = O.make_design(spec, q)
        assert f[g, 12] == ds["r"]
        assert abs(f[g, 14] - ds["z1"]) <= 1e-12, (g, f[g, 14], ds["z1"])
        assert abs(f[g, 15] - ds["z2"]) <= 1e-12, (g, f[g, 15], ds["z2"])


@pytest.mark.parametrize("M", [2000, 1037])
def test_alpha_grid_objective_matches_oracle(M):
    spec = W.alpha_design(23, m_r=17, n_draws=M)
    G = O.grid_size(spec)
    ref_mean, ref_var = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        say(f"alpha grid {spec['m']} M={M} {prec}")
        with bmd.Problem(spec) as p:
            mean, var = p.eval_grid(M, prec, want_var=True)
            torch.cuda.synchronize()
            mean, var = mean.cpu().numpy(), var.cpu().numpy()
        _check(mean, ref_mean, prec, "alpha-grid mean")
        assert np.allclose(var, ref_var, rtol=1e-6 if prec == "fp64" else 2e-3, atol=1e-9)


def test_alpha_smoothing_and_argmax_match_oracle():
    spec = W.alpha_design(23, m_r=17)
    raw_h = W.noisy_surface(spec["m"], seed=5)
    with bmd.Problem(spec) as p:
        raw = torch.tensor(raw_h, dtype=torch.float64, device="cuda")
        s64 = p.smooth(raw, "fp64")
        i64, v64, cell = p.argmax(s64)
        s64_h = s64.cpu().numpy()
    ref = O.smooth_separable(spec, raw_h)
    assert np.max(np.abs(s64_h - ref)) <= 1e-13
    assert np.max(np.abs(O.smooth_direct(spec, raw_h) - ref)) < 1e-13
    io = O.argmax(ref)
    assert i64 == io and v64 == pytest.approx(ref[io], abs=1e-13)
    _, idx = O.grid_point(spec, io)
    assert tuple(idx) == cell


def test_alpha_line_converges_to_closed_form():
    """At r_2 = 0.365 (condition (b)), 49 levels alpha_1, 10^6 draws: every GPU
    estimate is within 5 Monte Carlo standard errors of the closed form, and
    the estimated surface peaks within two grid steps of its maximiser."""
    spec = W.alpha_design(49, r=0.365)
    M = 1_000_000
    with bmd.Problem(spec) as p:
        mean, var = p.eval_grid(M, "fp32", want_var=True)
        torch.cuda.synchronize()
        mean, var = mean.cpu().numpy(), var.cpu().numpy()
    exact = np.array([O.exact_paper(spec, O.grid_point(spec, g)[0]) for g in range(49)])
    z = (mean - exact) / np.sqrt(var / M)
    assert np.max(np.abs(z)) < 5.0, z
    assert abs(int(np.argmax(mean)) - int(np.argmax(exact))) <= 2


def test_alpha_problem_in_a_batch():
    """An alpha-design problem batched with cutoff problems gives its one-problem sweep."""
    specs = [W.alpha_design(23, m_r=9), W.base_problem(2, [9, 7], 0.3, 0.05), W.plain_1d()]
    draws = [1500, 900, 700]
    probs = [bmd.Problem(s) for s in specs]
    try:
        means, _ = bmd.eval_batch(probs, draws, "fp32")
        for p, m, n in zip(probs, means, draws):
            ref = p.eval_grid(n, "fp32")
            torch.cuda.synchronize()
            assert (m - ref).abs().max().item() <= 1e-12
    finally:
        for p in probs:
            p.close()


def test_alpha_full_grid_sampled():
    """The benchmarked alpha grid (181 x 241 designs, M = 1e6, FP32 integrand):
    six designs, corners included, against the oracle on the same draws."""
    spec = W.alpha_grid()
    G, M = O.grid_size(spec), spec["n_draws"]
    rng = np.random.default_rng(11)
    gs = np.unique(np.concatenate([[0, G - 1, G // 2 + 17], rng.integers(0, G, 3)]))
    say(f"alpha full grid G={G} M={M}: oracle on {len(gs)} designs")
    ref, _ = O.eval_grid(spec, gs, M)
    with bmd.Problem(spec) as p:
        mean = p.eval_grid(M, "fp32").cpu().numpy()
    _check(mean[gs], ref, "fp32", "alpha full grid")
    assert np.all(np.isfinite(mean)) and mean.min() >= 0.0 and mean.max() <= 1.0
