"""Three nested populations on the GPU (n = 3 of Sec. 2.2 with the Formula 10
prior of Sec. 3's condition (c)): an (alpha_1, alpha_2) grid with alpha_3 on
the FWER boundary, through the C ABI against the oracle on the same draws
(bars as in test_gpu_parity: FP64 1e-9, FP32 1e-5, relative to max(|f|, 1e-3);
grid coordinates and uniforms bit-exact; critical values 1e-10), and against
the closed form of the prior within Monte Carlo error.  Designs whose first two
levels spend alpha0 are NaN on both sides."""
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


@pytest.mark.parametrize("spec", [W.alpha3_design(7), W.alpha3_design(5, r2=0.85, r3=0.3),
                                  W.alpha3_design(4, r2=0.2, r3=0.02, q_range=(0.001, 0.012))])
def test_alpha3_designs_and_critical_values(spec):
    say(f"alpha3 designs m={spec['m']} r=({spec['r_lo']}, {spec['r_hi']})")
    with bmd.Problem(spec) as p:
        G = p.G
        f = p.designs(0, G).cpu().numpy()
        assert bmd.sweep_kind(p) == "direct"
    n_nan = 0
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        assert np.array_equal(f[g, :2], q), g
        ds = O.make_design(spec, q)
        assert f[g, 12] == ds["r"] == spec["r_lo"] and f[g, 6] == ds["r3"] == spec["r_hi"]
        assert abs(f[g, 14] - ds["z1"]) <= 1e-12 and abs(f[g, 15] - ds["z2"]) <= 1e-12, g
        if math.isnan(ds["z3"]):
            assert math.isnan(f[g, 7]), g
            n_nan += 1
        else:
            assert abs(f[g, 7] - ds["z3"]) <= 1e-10, (g, f[g, 7], ds["z3"])
    if spec["q_hi"] > 0.02:
        assert 0 < n_nan < G


def test_alpha3_draws():
    spec = W.alpha3_design(5)
    spec.update(seed=0x5EED, scenario=3)
    k0, n = (1 << 32) - 20, 40
    with bmd.Problem(spec) as p:
        u, f = p.draws(k0, n)
        u, f = u.cpu().numpy(), f.cpu().numpy()
    for i in range(n):
        dr = O.make_draw(spec, k0 + i)
        assert np.array_equal(u[i, :3], dr["u"][:3]), i
        assert np.all(u[i, 3:] == 0.0)
        for j, e in ((3, dr["e1"]), (4, dr["e2"]), (5, dr["e3"])):
            assert abs(f[i, j] - e) <= 4 * np.spacing(abs(e)) + 1e-17, (i, j, f[i, j], e)


@pytest.mark.parametrize("spec,M", [(W.alpha3_design(7), 1000), (W.alpha3_design(5, r2=0.85, r3=0.3), 703),
                                    (W.alpha3_design(4, r2=0.9, r3=0.5, q_range=(0.001, 0.02)), 515)])
def test_alpha3_grid_objective_matches_oracle(spec, M):
    G = O.grid_size(spec)
    say(f"alpha3 oracle m={spec['m']} M={M}")
    ref_mean, ref_var = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        say(f"alpha3 grid m={spec['m']} M={M} {prec}")
        with bmd.Problem(spec) as p:
            mean, var = p.eval_grid(M, prec, want_var=True)
            torch.cuda.synchronize()
            mean, var = mean.cpu().numpy(), var.cpu().numpy()
        _check(mean, ref_mean, prec, "alpha3 mean")
        ok = ~np.isnan(ref_var)
        assert np.allclose(var[ok], ref_var[ok], rtol=1e-6 if prec == "fp64" else 2e-3, atol=1e-9)


def test_alpha3_converges_to_closed_form():
    """5 x 5 levels around condition (c)'s printed optimum, 4 * 10^5 draws: every
    feasible GPU estimate is within 5 Monte Carlo standard errors of the closed
    form, and the argmax over feasible designs is the closed form's or within
    one grid step of it."""
    spec = W.alpha3_design(5, q_range=(0.0005, 0.0185))
    M = 400_000
    with bmd.Problem(spec) as p:
        mean, var = p.eval_grid(M, "fp32", want_var=True)
        torch.cuda.synchronize()
        i_gpu, v_gpu, cell = p.argmax(mean)
        mean, var = mean.cpu().numpy(), var.cpu().numpy()
    exact = np.array([O.exact_paper(spec, O.grid_point(spec, g)[0]) for g in range(25)])
    ok = ~np.isnan(exact)
    assert np.array_equal(ok, ~np.isnan(mean))
    z = (mean[ok] - exact[ok]) / np.sqrt(var[ok] / M)
    assert np.max(np.abs(z)) < 5.0, z
    i_ex = int(np.nanargmax(exact))
    _, b = O.grid_point(spec, i_ex)
    assert max(abs(int(x) - int(y)) for x, y in zip(cell, b)) <= 1
    assert v_gpu == mean[i_gpu]


@pytest.mark.parametrize("m,corner", [(9, 5), (23, 12)])
def test_alpha3_masked_smoothing_and_argmax_match_oracle(m, corner):
    """Designs without a third level are NaN: the smoother sums over the others
    and keeps them NaN (FP64 1e-13, FP32 2e-6 of the surface's scale); the
    argmax skips them."""
    spec = W.alpha3_design(m)
    raw_h = W.noisy_surface(spec["m"], seed=m, nan_corner=corner)
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


def test_alpha3_grid_without_any_third_level():
    """Levels that always spend alpha0 in the first two tests: every design is
    NaN on both sides, smoothing keeps them NaN and the argmax reports NaN."""
    spec = W.alpha3_design(4, q_range=(0.02, 0.024))
    assert all(math.isnan(O.make_design(spec, O.grid_point(spec, g)[0])["z3"]) for g in range(16))
    with bmd.Problem(spec) as p:
        mean = p.eval_grid(300, "fp32")
        s = p.smooth(mean, "fp32")
        i, v, cell = p.argmax(s)
        assert torch.isnan(mean).all().item() and torch.isnan(s).all().item()
    assert i == 0 and math.isnan(v) and tuple(cell) == (0, 0)


def test_alpha3_not_batched():
    spec = W.alpha3_design(5)
    with bmd.Problem(spec) as p, bmd.Problem(W.plain_1d()) as q:
        with pytest.raises(bmd.BmdError) as e:
            bmd.eval_batch([q, p], [100, 100], "fp32")
        assert e.value.status == -5


@pytest.mark.parametrize("M", [1, 7])
def test_alpha3_few_draws(M):
    """One draw and a ragged handful: a single partial slice per design."""
    spec = W.alpha3_design(5)
    G = O.grid_size(spec)
    ref, _ = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        with bmd.Problem(spec) as p:
            mean = p.eval_grid(M, prec).cpu().numpy()
        _check(mean, ref, prec, f"alpha3 M={M}")


@pytest.mark.parametrize("m,M", [((13, 21), 900), ((211, 211), 2000)])
def test_alpha3_block_mapping_sampled(m, M):
    """Wavefronts take the designs in the problem's order (those with a third
    level first): a ragged non-square grid and a large one (the last
    wavefront partly past the end of the order) against the
    oracle at sampled designs, corners and designs without a third level
    included; every design is written (finite or NaN as the oracle says)."""
    spec = W.alpha3_design(5)
    spec["m"] = list(m)
    spec["bandwidth"] = [0.0015, 0.0015]
    G = m[0] * m[1]
    rng = np.random.default_rng(m[0])
    gs = np.unique(np.concatenate([[0, m[1] - 1, G - m[1], G - 1], rng.integers(0, G, 6)]))
    ref, _ = O.eval_grid(spec, gs, M)
    feas = np.array([not math.isnan(O.make_design(spec, O.grid_point(spec, g)[0])["z3"]) for g in gs])
    for prec in ("fp64", "fp32"):
        say(f"alpha3 blocks m={m} M={M} {prec}")
        with bmd.Problem(spec) as p:
            mean = p.eval_grid(M, prec).cpu().numpy()
            z3 = p.designs(0, G).cpu().numpy()[:, 7]
        assert np.array_equal(np.isnan(mean), np.isnan(z3))
        assert np.array_equal(~np.isnan(mean[gs]), feas)
        _check(mean[gs], ref, prec, f"alpha3 blocks {m}")


def test_alpha3_full_grid_sampled():
    """The benchmarked three-population grid (97 x 97 designs, M = 1e5, FP32
    integrand): two feasible designs against the oracle on the same draws, and
    the NaN pattern of the whole surface is that of the designs' third levels."""
    spec = W.alpha3_grid()
    G, M = O.grid_size(spec), spec["n_draws"]
    gs = np.array([0, 52 * 97 + 20])
    say(f"alpha3 full grid G={G} M={M}: oracle on {len(gs)} designs")
    ref, _ = O.eval_grid(spec, gs, M)
    with bmd.Problem(spec) as p:
        mean = p.eval_grid(M, "fp32").cpu().numpy()
        z3 = p.designs(0, G).cpu().numpy()[:, 7]
    _check(mean[gs], ref, "fp32", "alpha3 full grid")
    assert np.array_equal(np.isnan(mean), np.isnan(z3)) and 0 < np.isnan(mean).sum() < G
