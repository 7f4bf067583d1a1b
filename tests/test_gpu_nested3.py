"""Three nested populations cut from one biomarker by two cutoffs (n = 3 in
the cutoff design space) on the GPU, through the C ABI against the oracle on
the same draws: critical values 1e-10 and the NaN pattern of designs that do
not exist; the one-biomarker draws (tau bit-exact); the Formula 5 estimate in
FP64 (1e-9) and FP32 (1e-5, relative to max(|f|, 1e-3)); masked smoothing and
the argmax."""
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
    bound = TOL[prec] * np.maximum(np.abs(ref[~nan]), 1e-3)
    err = np.abs(got[~nan] - ref[~nan])
    w = int(np.argmax(err / bound))
    assert np.all(err <= bound), f"{what} {prec}: index {w} got {got[~nan][w]!r} ref {ref[~nan][w]!r}"


@pytest.mark.parametrize("rule", ["fwer", "bonferroni"])
def test_nested3_designs(rule):
    spec = W.nested3_design((9, 13), rule=rule)
    G = O.grid_size(spec)
    with bmd.Problem(spec) as p:
        f = p.designs(0, G).cpu().numpy()
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        ds = O.make_design(spec, q)
        assert np.array_equal(f[g, :2], q), g
        assert f[g, 12] == ds["r"] and f[g, 6] == ds["r3"], g
        if np.isnan(ds["z1"]):
            assert np.isnan(f[g, 14]) and np.isnan(f[g, 7]), g
        else:
            assert abs(f[g, 14] - ds["z1"]) <= 1e-10 and f[g, 15] == f[g, 14] == f[g, 7], (g, f[g, 14], ds["z1"])


def test_nested3_draws():
    spec = W.nested3_design(5, seed=0x77, scenario=2)
    k0, n = (1 << 32) - 10, 24
    with bmd.Problem(spec) as p:
        u, f = p.draws(k0, n)
        u, f = u.cpu().numpy(), f.cpu().numpy()
    for i in range(n):
        dr = O.make_draw(spec, k0 + i)
        assert np.array_equal(u[i, :3], dr["u"][:3]) and np.all(u[i, 3:] == 0.0), i
        assert f[i, 5] == dr["tau"][0] and f[i, 2] == dr["PR"], i
        for j, v in ((0, dr["b0"]), (1, dr["b1"])):
            assert abs(f[i, j] - v) <= 4 * np.spacing(abs(v)) + 1e-17, (i, j)


@pytest.mark.parametrize("spec,M", [(W.nested3_design((9, 13)), 700), (W.nested3_design(6, rule="bonferroni"), 513),
                                    (W.nested3_design((7, 5), q_range=(0.2, 0.6)), 1), (W.nested3_design(5), 7)])
def test_nested3_matches_oracle(spec, M):
    G = O.grid_size(spec)
    say(f"nested3 m={spec['m']} M={M}")
    ref, ref_var = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        with bmd.Problem(spec) as p:
            mean, var = p.eval_grid(M, prec, want_var=True)
            torch.cuda.synchronize()
            mean, var = mean.cpu().numpy(), var.cpu().numpy()
        _check(mean, ref, prec, f"nested3 {spec['m']}")
        ok = ~np.isnan(ref)
        if M > 1:
            assert np.allclose(var[ok], ref_var[ok], rtol=1e-6 if prec == "fp64" else 2e-3, atol=1e-9)


def test_nested3_full_grid_sampled():
    """The benchmarked 64 x 64 grid at M = 1e5: the FP32 surface within 1e-5 of
    the FP64 one, NaN exactly for designs that do not exist; sampled designs
    against the oracle at M = 600 in both precisions."""
    spec = W.nested3_grid()
    G, M = O.grid_size(spec), spec["n_draws"]
    with bmd.Problem(spec) as p:
        say(f"nested3 full grid G={G} M={M}")
        m32 = p.eval_grid(M, "fp32").cpu().numpy()
        m64 = p.eval_grid(M, "fp64").cpu().numpy()
        z = p.designs(0, G).cpu().numpy()[:, 7]
        assert np.array_equal(np.isnan(m32), np.isnan(z)) and np.array_equal(np.isnan(m64), np.isnan(z))
        ok = ~np.isnan(m64)
        assert 0 < ok.sum() < G
        assert np.max(np.abs(m32[ok] - m64[ok]) / np.maximum(np.abs(m64[ok]), 1e-3)) <= 1e-5
        Ms = 600
        gs = np.nonzero(ok)[0][:: max(1, ok.sum() // 6)][:6]
        ref, _ = O.eval_grid(spec, gs, Ms)
        for prec in ("fp64", "fp32"):
            mean = p.eval_grid(Ms, prec).cpu().numpy()
            _check(mean[gs], ref, prec, "nested3 full grid")


def test_nested3_masked_smoothing_and_argmax():
    """The smoother sums over the designs that exist and keeps the others NaN
    (FP64 1e-13 against the oracle's masked smoother); the argmax skips NaN."""
    spec = W.nested3_design(12, bandwidth=0.06)
    G = O.grid_size(spec)
    with bmd.Problem(spec) as p:
        raw = p.eval_grid(400, "fp64")
        raw_h = raw.cpu().numpy()
        s64 = p.smooth(raw, "fp64")
        i64, v64, cell = p.argmax(s64)
        s64 = s64.cpu().numpy()
    ref = O.smooth_masked(spec, raw_h)
    nan = np.isnan(raw_h)
    assert np.array_equal(np.isnan(s64), nan) and 0 < nan.sum() < G
    assert np.max(np.abs(s64[~nan] - ref[~nan])) <= 1e-13
    io = int(np.nanargmax(ref))
    assert i64 == io and v64 == pytest.approx(ref[io], abs=1e-13)


def test_nested3_rejected_where_undefined():
    for bad, status in ((dict(effect="paper"), -1), (dict(q_lo=0.05), -2), (dict(width=0.01), -2),
                        (dict(m=[4096, 4097]), -2),
                        (dict(alpha_rule="fixed", alpha_fixed=(0.01, 0.01)), -1)):
        with pytest.raises(bmd.BmdError) as e:
            bmd.Problem(dict(W.nested3_design(5), **bad))
        assert e.value.status == status, bad
    with bmd.Problem(W.nested3_design(5)) as p, bmd.Problem(W.plain_1d()) as q:
        with pytest.raises(bmd.BmdError) as e:
            bmd.eval_batch([q, p], [100, 100], "fp32")
        assert e.value.status == -5
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid_two_layer(1024, 4096)
        assert e.value.status == -5
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid_dalpha(100, "fp32")
        assert e.value.status == -6
        with pytest.raises(bmd.BmdError) as e:
            p.grad_design(torch.full((1, 2), 0.5, dtype=torch.float64, device="cuda"), 100, "fp32")
        assert e.value.status == -5


def test_nested3_noalloc_matches():
    """The allocation-free entry point on the two-cutoff space, twice in a row
    (the second on a smaller problem), against bmd_eval_grid."""
    for m, M in (((9, 13), 900), (5, 300)):
        with bmd.Problem(W.nested3_design(m)) as p:
            a, va = p.eval_grid(M, "fp32", want_var=True)
            b, vb = p.eval_grid(M, "fp32", want_var=True, noalloc=True)
            a, b, va, vb = (t.cpu().numpy() for t in (a, b, va, vb))
        assert np.array_equal(np.isnan(a), np.isnan(b))
        ok = ~np.isnan(a)
        assert np.array_equal(a[ok], b[ok]) and np.array_equal(va[ok], vb[ok])
