"""Four nested populations on the GPU (n = 4 of Sec. 2.2, the three-threshold
designs of Sec. 3, Formula 10 prior with condition (c)'s effects): an
(alpha_1, alpha_2, alpha_3) grid with alpha_4 on the FWER boundary, through
the C ABI against the oracle on the same draws (bars as in test_gpu_parity:
FP64 1e-9, FP32 1e-5, relative to max(|f|, 1e-3); grid coordinates and
uniforms bit-exact; critical values 1e-10), and against the closed form of
the prior within Monte Carlo error.  Designs whose first three levels spend
alpha0 are NaN on both sides.  The oracle's Phi_4 takes milliseconds and its
fourth level a fraction of a second, so grids and draw counts here are small."""
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
    got = np.asarray(got)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan), f"{what} {prec}: NaN pattern differs"
    got, ref = got[~nan], ref[~nan]
    bound = TOL[prec] * np.maximum(np.abs(ref), 1e-3)
    err = np.abs(got - ref)
    w = int(np.argmax(err / bound))
    assert np.all(err <= bound), f"{what} {prec}: index {w} got {got[w]!r} ref {ref[w]!r}"


@pytest.mark.parametrize("spec", [W.alpha4_design(4), W.alpha4_design(3, r2=0.85, r3=0.5, r4=0.3),
                                  W.alpha4_design(3, r2=0.3, r3=0.1, r4=0.02, q_range=(0.001, 0.012))])
def test_alpha4_designs_and_critical_values(spec):
    say(f"alpha4 designs m={spec['m']} r=({spec['r_lo']}, {spec['r_hi']}, {spec['r_4']})")
    with bmd.Problem(spec) as p:
        G = p.G
        f = p.designs(0, G).cpu().numpy()
        assert bmd.sweep_kind(p) == "direct"
    n_nan = 0
    rng = np.random.default_rng(G)
    sample = np.unique(np.concatenate([[0, G - 1], rng.integers(0, G, 10)]))   # the oracle's root takes ~0.5 s
    for g in sample:
        q, _ = O.grid_point(spec, g)
        assert np.array_equal(f[g, :3], q), g
        ds = O.make_design(spec, q)
        assert f[g, 12] == ds["r"] == spec["r_lo"] and f[g, 6] == ds["r3"] == spec["r_hi"]
        assert f[g, 8] == ds["r4"] == spec["r_4"]
        assert abs(f[g, 14] - ds["z1"]) <= 1e-12 and abs(f[g, 15] - ds["z2"]) <= 1e-12, g
        assert abs(f[g, 7] - ds["z3"]) <= 1e-12, g
        if math.isnan(ds["z4"]):
            assert math.isnan(f[g, 9]), g
            n_nan += 1
        else:
            assert abs(f[g, 9] - ds["z4"]) <= 1e-10, (g, f[g, 9], ds["z4"])
    if spec["q_hi"] > 0.02:
        assert 0 < n_nan < sample.size


def test_alpha4_draws():
    spec = W.alpha4_design(3)
    spec.update(seed=0x5EED, scenario=3)
    k0, n = (1 << 32) - 20, 40
    with bmd.Problem(spec) as p:
        u, f = p.draws(k0, n)
        u, f = u.cpu().numpy(), f.cpu().numpy()
    for i in range(n):
        dr = O.make_draw(spec, k0 + i)
        assert np.array_equal(u[i, :4], dr["u"][:4]), i
        assert np.all(u[i, 4:] == 0.0)
        for j, e in ((3, dr["e1"]), (4, dr["e2"]), (5, dr["e3"]), (6, dr["e4"])):
            assert abs(f[i, j] - e) <= 4 * np.spacing(abs(e)) + 1e-17, (i, j, f[i, j], e)


@pytest.mark.parametrize("spec,M", [(W.alpha4_design(4), 48), (W.alpha4_design(3, r2=0.85, r3=0.5, r4=0.3), 37)])
def test_alpha4_grid_objective_matches_oracle(spec, M):
    G = O.grid_size(spec)
    say(f"alpha4 oracle m={spec['m']} M={M}")
    ref_mean, ref_var = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        say(f"alpha4 grid m={spec['m']} M={M} {prec}")
        with bmd.Problem(spec) as p:
            mean, var = p.eval_grid(M, prec, want_var=True)
            torch.cuda.synchronize()
            mean, var = mean.cpu().numpy(), var.cpu().numpy()
        _check(mean, ref_mean, prec, "alpha4 mean")
        ok = ~np.isnan(ref_var)
        assert np.allclose(var[ok], ref_var[ok], rtol=1e-6 if prec == "fp64" else 2e-3, atol=1e-9)


def test_alpha4_converges_to_closed_form():
    """3 x 3 x 3 levels, 4 * 10^5 draws: every feasible GPU estimate is within 5
    Monte Carlo standard errors of the Formula 10 closed form, and the argmax
    over feasible designs is the closed form's or within one grid step of it."""
    spec = W.alpha4_design(3, q_range=(0.001, 0.009))
    M = 400_000
    with bmd.Problem(spec) as p:
        mean, var = p.eval_grid(M, "fp32", want_var=True)
        torch.cuda.synchronize()
        i_gpu, v_gpu, cell = p.argmax(mean)
        mean, var = mean.cpu().numpy(), var.cpu().numpy()
    exact = np.array([O.exact_paper(spec, O.grid_point(spec, g)[0]) for g in range(27)])
    ok = ~np.isnan(exact)
    assert ok.sum() > 0 and np.array_equal(ok, ~np.isnan(mean))
    z = (mean[ok] - exact[ok]) / np.sqrt(var[ok] / M)
    assert np.max(np.abs(z)) < 5.0, z
    i_ex = int(np.nanargmax(exact))
    _, b = O.grid_point(spec, i_ex)
    assert max(abs(int(x) - int(y)) for x, y in zip(cell, b)) <= 1
    assert v_gpu == mean[i_gpu]


def test_alpha4_masked_smoothing_and_argmax_match_oracle():
    """Designs without a fourth level are NaN: the smoother sums over the others
    and keeps them NaN (FP64 1e-13, FP32 2e-6 of the surface's scale); the
    argmax skips them."""
    spec = W.alpha4_design(11)
    raw_h = W.noisy_surface(spec["m"], seed=4, nan_corner=9)
    nan = np.isnan(raw_h)
    assert 0 < nan.sum() < raw_h.size
    with bmd.Problem(spec) as p:
        raw = torch.tensor(raw_h, dtype=torch.float64, device="cuda")
        s64, s32 = p.smooth(raw, "fp64"), p.smooth(raw, "fp32")
        i64, v64, cell = p.argmax(s64)
        s64_h, s32_h = s64.cpu().numpy(), s32.cpu().numpy()
    ref = O.smooth_masked(spec, raw_h)
    for got in (s64_h, s32_h):
        assert np.array_equal(np.isnan(got), nan)
    assert np.max(np.abs(s64_h[~nan] - ref[~nan])) <= 1e-13
    assert np.max(np.abs(s32_h[~nan] - ref[~nan])) <= 2e-6 * np.max(np.abs(ref[~nan]))
    io = int(np.nanargmax(ref))
    assert i64 == io and v64 == pytest.approx(ref[io], abs=1e-13)
    _, idx = O.grid_point(spec, io)
    assert tuple(idx) == cell


@pytest.mark.parametrize("M", [1, 7])
def test_alpha4_few_draws(M):
    """One draw and a ragged handful: a single partial slice per design."""
    spec = W.alpha4_design(3)
    G = O.grid_size(spec)
    ref, _ = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        with bmd.Problem(spec) as p:
            mean = p.eval_grid(M, prec).cpu().numpy()
        _check(mean, ref, prec, f"alpha4 M={M}")


@pytest.mark.parametrize("m,M", [((5, 9, 6), 300), ((25, 25, 25), 500)])
def test_alpha4_block_mapping_sampled(m, M):
    """Wavefronts take the designs in the problem's order (those with a fourth
    level first): a ragged grid and the benchmarked 25^3 grid (the last
    wavefront partly past the end of the order) against the oracle
    at sampled designs, corners included; every design is written (finite or
    NaN as its fourth level says)."""
    spec = W.alpha4_design(5)
    spec["m"] = list(m)
    G = int(np.prod(m))
    rng = np.random.default_rng(m[0])
    gs = np.unique(np.concatenate([[0, m[2] - 1, G - m[2], G - 1], rng.integers(0, G, 4)]))
    say(f"alpha4 blocks m={m} M={M}: oracle on {gs.size} designs")
    ref, _ = O.eval_grid(spec, gs, M)
    for prec in ("fp64", "fp32"):
        say(f"alpha4 blocks m={m} M={M} {prec}")
        with bmd.Problem(spec) as p:
            mean = p.eval_grid(M, prec).cpu().numpy()
            z4 = p.designs(0, G).cpu().numpy()[:, 9]
        assert np.array_equal(np.isnan(mean), np.isnan(z4))
        _check(mean[gs], ref, prec, f"alpha4 blocks {m}")


def test_alpha4_full_grid_sampled():
    """The benchmarked four-population grid (25^3 designs): at the full
    M = 1e5 the FP32 surface is within 1e-5 of the FP64 one everywhere and NaN
    exactly where the fourth level is; at M = 256 four sampled designs match
    the oracle on the same draws in both precisions (the oracle's Phi_4 takes
    milliseconds a summand, too slow for 1e5 draws)."""
    spec = W.alpha4_grid()
    G, M = O.grid_size(spec), spec["n_draws"]
    with bmd.Problem(spec) as p:
        say(f"alpha4 full grid G={G} M={M}")
        m32 = p.eval_grid(M, "fp32").cpu().numpy()
        m64 = p.eval_grid(M, "fp64").cpu().numpy()
        z4 = p.designs(0, G).cpu().numpy()[:, 9]
    assert np.array_equal(np.isnan(m32), np.isnan(z4)) and np.array_equal(np.isnan(m64), np.isnan(z4))
    assert 0 < np.isnan(m32).sum() < G
    ok = ~np.isnan(m64)
    assert np.max(np.abs(m32[ok] - m64[ok]) / np.maximum(np.abs(m64[ok]), 1e-3)) <= 1e-5
    Ms = 256
    gs = np.array([0, (3 * 25 + 5) * 25 + 2, (10 * 25 + 2) * 25 + 7, 24 * 25])
    say(f"alpha4 full grid: oracle on {gs.size} designs at M={Ms}")
    ref, _ = O.eval_grid(spec, gs, Ms)
    assert not np.any(np.isnan(ref))
    for prec in ("fp64", "fp32"):
        with bmd.Problem(spec) as p:
            mean = p.eval_grid(Ms, prec).cpu().numpy()
        _check(mean[gs], ref, prec, "alpha4 full grid")


def test_alpha4_rejected_where_unsupported():
    spec = W.alpha4_design(3)
    with bmd.Problem(spec) as p, bmd.Problem(W.plain_1d()) as q:
        with pytest.raises(bmd.BmdError) as e:
            bmd.eval_batch([q, p], [100, 100], "fp32")
        assert e.value.status == -5
    bad = W.alpha4_design(3, r2=0.5, r3=0.49, r4=0.1)   # r_3 > 0.95 r_2
    with pytest.raises(bmd.BmdError) as e:
        bmd.Problem(bad)
    assert e.value.status == -2
