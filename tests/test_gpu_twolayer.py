"""The two-layer sampling estimator of Formula 7 on the GPU (the inner layer
of Formula 6 with one set of inner draws for every outer draw) against the
oracle on the same draws: the comparison counts are integers, so in FP64 the
estimate equals the oracle's bit for bit and the block variance estimate to
1e-12 relative (the same formula over the same counts); in FP32 (both sides of
each comparison rounded) the estimate is within 1e-5 of max(|f|, 1e-3).
Designs without a valid level split are NaN on both sides."""
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _specs():
    return {
        "alpha_n2": W.alpha_design(9),
        "alpha_r_grid": W.alpha_design(7, m_r=5),
        "alpha3": W.alpha3_design(4),
        "alpha4": W.alpha4_design(3),
        "cutoff_fwer": W.base_problem(1, [11], 0.0, 0.05, info=211.0, effect="paper", paper_a=0.3, paper_b=0.1),
        "cutoff_one_test": W.base_problem(1, [7], 0.0, 0.05, info=211.0, effect="paper", paper_a=0.3, paper_b=0.1,
                                          alpha_rule="fixed", alpha_fixed=(0.01, 0.0)),
    }


def _check_fp64(got_m, got_v, ref_m, ref_v, what):
    nan = np.isnan(ref_m)
    assert np.array_equal(np.isnan(got_m), nan), what
    assert np.array_equal(got_m[~nan], ref_m[~nan]), (what, got_m, ref_m)
    assert np.allclose(got_v[~nan], ref_v[~nan], rtol=1e-12, atol=1e-18), (what, got_v, ref_v)


@pytest.mark.parametrize("name", list(_specs()))
def test_two_layer_matches_oracle(name):
    spec = _specs()[name]
    G = O.grid_size(spec)
    N1, N2, A, B = 1280, 4096, 16, 16
    say(f"two-layer {name} G={G} N1={N1} N2={N2}")
    ref_m, ref_v, _ = O.eval_grid_two_layer(spec, np.arange(G), N1, N2, A, B)
    with bmd.Problem(spec) as p:
        m64, v64 = (t.cpu().numpy() for t in p.eval_grid_two_layer(N1, N2, "fp64", (A, B)))
        m32, v32 = (t.cpu().numpy() for t in p.eval_grid_two_layer(N1, N2, "fp32", (A, B)))
    _check_fp64(m64, v64, ref_m, ref_v, name)
    ok = ~np.isnan(ref_m)
    assert np.array_equal(np.isnan(m32), ~ok)
    assert np.all(np.abs(m32[ok] - ref_m[ok]) <= 1e-5 * np.maximum(np.abs(ref_m[ok]), 1e-3)), name
    assert np.all(v64[ok] > 0)


def test_two_layer_full_size_sampled():
    """The paper's sizes N1 = 10,240 and N2 = 20,480 (Sec. 2.2) on the
    two-population level grid (241 levels at r_2 = 0.365) and the
    three-population 97 x 97 grid of condition (c): every design on the GPU,
    sampled designs against the oracle (2.1e8 comparisons each) bit for bit in
    FP64, every FP32 value within 1e-5 of FP64."""
    N1, N2 = 10240, 20480
    for spec, gs in ((W.alpha_design(241), [0, 120, 240]), (W.alpha3_grid(), [0, 48 * 97 + 13])):
        G = O.grid_size(spec)
        say(f"two-layer full size G={G}")
        with bmd.Problem(spec) as p:
            m64, v64 = (t.cpu().numpy() for t in p.eval_grid_two_layer(N1, N2, "fp64"))
            m32 = p.eval_grid_two_layer(N1, N2, "fp32", want_var=False)[0].cpu().numpy()
        ok = ~np.isnan(m64)
        assert ok.sum() > 0 and np.array_equal(np.isnan(m32), ~ok)
        assert np.max(np.abs(m32[ok] - m64[ok])) <= 1e-5
        say(f"  oracle on {len(gs)} designs")
        ref_m, ref_v, _ = O.eval_grid_two_layer(spec, np.array(gs), N1, N2, 16, 16)
        _check_fp64(m64[gs], v64[gs], ref_m, ref_v, "full size")


def test_two_layer_agrees_with_formula5_on_the_gpu():
    """On the same outer draws Formula 7 differs from the deterministic
    Formula 5 sweep only by the inner layer's error: within 5 of its standard
    errors estimated from the inner groups (each group an independent
    replicate of the inner layer given the outer draws) — the block variance
    with the outer part held fixed."""
    spec = W.alpha3_design(6)
    N1, N2, A, B = 2048, 65536, 4, 32
    with bmd.Problem(spec) as p:
        m2, _ = p.eval_grid_two_layer(N1, N2, "fp64", (A, B))
        det = p.eval_grid(N1, "fp64")
        m2, det = m2.cpu().numpy(), det.cpu().numpy()
    G = O.grid_size(spec)
    ok = ~np.isnan(det)
    gs = np.nonzero(ok)[0][:4]
    _, _, blk = O.eval_grid_two_layer(spec, gs, N1, N2, A, B)
    for i, g in enumerate(gs):
        col = 1 - blk[i].sum(axis=0) / (N1 * N2 / B)
        se = col.std(ddof=1) / math.sqrt(B)
        assert abs(m2[g] - det[g]) < 5 * se, (g, m2[g], det[g], se)
    assert np.array_equal(np.isnan(m2), ~ok) and G > len(gs)


def test_two_layer_rejected_where_undefined():
    with bmd.Problem(W.plain_1d()) as p:   # step prior
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid_two_layer(1024, 4096)
        assert e.value.status == -5
    with bmd.Problem(W.alpha_design(5)) as p:
        for n1, n2, blocks in ((1000, 4096, (16, 16)), (1024, 4000, (16, 16)), (1024, 4096, (1, 16)),
                               (1024, 4096, (16, 65)), (1024, 4096, (16, 32)), (1024, 3072, (16, 8))):
            with pytest.raises(bmd.BmdError) as e:
                p.eval_grid_two_layer(n1, n2, "fp64", blocks)
            assert e.value.status == -2, (n1, n2, blocks)
