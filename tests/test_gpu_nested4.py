"""Four nested populations cut from one biomarker by three cutoffs on the
GPU, through the C ABI against the oracle on the same draws: critical values
(1e-10) and the NaN pattern of designs that do not exist, the one-biomarker
draws, the Formula 5 estimate in FP64 (1e-9) and FP32 (1e-5, relative to
max(|f|, 1e-3)), the full 24^3 grid sampled, masked smoothing, rejections.
The oracle's four-variate CDF takes milliseconds, so its grids are small."""
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
    assert np.all(err <= bound), f"{what} {prec}: max err {err.max()!r}"


@pytest.mark.parametrize("rule", ["fwer", "bonferroni"])
def test_nested4_designs(rule):
    spec = W.nested4_design(5, rule=rule)
    G = O.grid_size(spec)
    with bmd.Problem(spec) as p:
        f = p.designs(0, G).cpu().numpy()
    n_ok = 0
    for g in range(G):
        q, _ = O.grid_point(spec, g)
        ds = O.make_design(spec, q)
        assert np.array_equal(f[g, :3], q), g
        assert f[g, 12] == ds["r"] and f[g, 6] == ds["r3"] and f[g, 8] == ds["r4"], g
        if np.isnan(ds["z4"]):
            assert np.isnan(f[g, 14]) and np.isnan(f[g, 9]), g
        else:
            n_ok += 1
            assert abs(f[g, 14] - ds["z4"]) <= 1e-10, (g, f[g, 14], ds["z4"])
            assert f[g, 15] == f[g, 14] == f[g, 7] == f[g, 9], g
    assert n_ok >= 4


def test_nested4_draws():
    spec = W.nested4_design(4, seed=0x99, scenario=5)
    k0, n = (1 << 32) - 7, 16
    with bmd.Problem(spec) as p:
        u, f = p.draws(k0, n)
        u, f = u.cpu().numpy(), f.cpu().numpy()
    for i in range(n):
        dr = O.make_draw(spec, k0 + i)
        assert np.array_equal(u[i, :3], dr["u"][:3]) and np.all(u[i, 3:] == 0.0), i
        assert f[i, 5] == dr["tau"][0] and f[i, 2] == dr["PR"], i


@pytest.mark.parametrize("spec,M", [(W.nested4_design(5), 40), (W.nested4_design((4, 6, 5), rule="bonferroni"), 7),
                                    (W.nested4_design(5, q_range=(0.15, 0.85)), 1)])
def test_nested4_matches_oracle(spec, M):
    G = O.grid_size(spec)
    say(f"nested4 m={spec['m']} M={M}")
    ref, ref_var = O.eval_grid(spec, np.arange(G), M)
    for prec in ("fp64", "fp32"):
        with bmd.Problem(spec) as p:
            mean, var = p.eval_grid(M, prec, want_var=True)
            mean, var = mean.cpu().numpy(), var.cpu().numpy()
        _check(mean, ref, prec, f"nested4 {spec['m']}")
        ok = ~np.isnan(ref)
        if M > 1:
            assert np.allclose(var[ok], ref_var[ok], rtol=1e-6 if prec == "fp64" else 2e-3, atol=1e-9)


def test_nested4_full_grid_sampled():
    """The benchmarked 24^3 grid at M = 1e5: FP32 within 1e-5 of FP64, NaN
    exactly where designs do not exist; four designs against the oracle at
    M = 60 in both precisions."""
    spec = W.nested4_grid()
    G, M = O.grid_size(spec), spec["n_draws"]
    with bmd.Problem(spec) as p:
        say(f"nested4 full grid G={G} M={M}")
        m32 = p.eval_grid(M, "fp32").cpu().numpy()
        m64 = p.eval_grid(M, "fp64").cpu().numpy()
        z = p.designs(0, G).cpu().numpy()[:, 9]
        assert np.array_equal(np.isnan(m32), np.isnan(z)) and np.array_equal(np.isnan(m64), np.isnan(z))
        ok = ~np.isnan(m64)
        assert 0 < ok.sum() < G
        assert np.max(np.abs(m32[ok] - m64[ok]) / np.maximum(np.abs(m64[ok]), 1e-3)) <= 1e-5
        gs = np.nonzero(ok)[0][:: max(1, ok.sum() // 4)][:4]
        Ms = 60
        ref, _ = O.eval_grid(spec, gs, Ms)
        for prec in ("fp64", "fp32"):
            mean = p.eval_grid(Ms, prec).cpu().numpy()
            _check(mean[gs], ref, prec, "nested4 full grid")


def test_nested4_masked_smoothing_and_argmax():
    spec = W.nested4_design(9, bandwidth=0.08)
    G = O.grid_size(spec)
    with bmd.Problem(spec) as p:
        raw = p.eval_grid(300, "fp64")
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


def test_nested4_rejected_where_undefined():
    for bad, status in ((dict(effect="paper"), -1), (dict(q_lo=0.05), -2), (dict(width=0.01), -2),
                        (dict(alpha_rule="fixed", alpha_fixed=(0.01, 0.01)), -1)):
        with pytest.raises(bmd.BmdError) as e:
            bmd.Problem(dict(W.nested4_design(4), **bad))
        assert e.value.status == status, bad
    with pytest.raises(bmd.BmdError) as e:
        bmd.Problem(dict(W.nested4_design(4), d=2, m=[4, 4], bandwidth=[0.05, 0.05]))
    assert e.value.status == -2
    with bmd.Problem(W.nested4_design(4)) as p, bmd.Problem(W.plain_1d()) as q:
        with pytest.raises(bmd.BmdError) as e:
            bmd.eval_batch([q, p], [100, 100], "fp32")
        assert e.value.status == -5
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid_two_layer(1024, 4096)
        assert e.value.status == -5
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid_dalpha(100, "fp32")
        assert e.value.status == -6


def test_nested4_noalloc_matches():
    for m, M in ((6, 700), (4, 200)):
        with bmd.Problem(W.nested4_design(m)) as p:
            a, va = p.eval_grid(M, "fp32", want_var=True)
            b, vb = p.eval_grid(M, "fp32", want_var=True, noalloc=True)
            a, b, va, vb = (t.cpu().numpy() for t in (a, b, va, vb))
        assert np.array_equal(np.isnan(a), np.isnan(b))
        ok = ~np.isnan(a)
        assert np.array_equal(a[ok], b[ok]) and np.array_equal(va[ok], vb[ok])
