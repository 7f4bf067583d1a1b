"""Batched form: many uneven grid problems in one graph-captured work-list
launch, checked against the single-problem sweep (same draws) and against the
oracle on sampled designs."""
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


def _scenarios(n, seed, m_scale, draws):
    sc = W.batch_scenarios(n, seed=seed, m_scale=m_scale, m_draws=draws)
    return sc


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_matches_single_problem_sweeps(prec):
    """Each work item of the batch runs the one-problem tile body on the same
    draws, so the batch matches the one-problem sweep up to the order of the
    FP64 slice sums."""
    sc = _scenarios(14, seed=4, m_scale=0.25, draws=(300, 3000))
    say(f"batch of {len(sc)} scenarios, d = {[s['d'] for s in sc]}, {prec}")
    probs = [bmd.Problem(s) for s in sc]
    try:
        means, wall = bmd.eval_batch(probs, [s["n_draws"] for s in sc], prec)
        torch.cuda.synchronize()
        for p, s, m in zip(probs, sc, means):
            ref = p.eval_grid(s["n_draws"], prec)
            torch.cuda.synchronize()
            err = (m - ref).abs().max().item()
            assert err <= 1e-12, (s["d"], s["m"], bmd.sweep_kind(p), err)
        assert np.all(wall > 0) and np.all(np.isfinite(wall))
        means2, _ = bmd.eval_batch(probs, [s["n_draws"] for s in sc], prec)
        for a, b in zip(means, means2):
            assert torch.equal(a, b)
    finally:
        for p in probs:
            p.close()


def test_batch_groups_under_a_memory_budget(monkeypatch):
    """A tiny draw budget puts every problem in a graph of its own; the results
    are those of one group."""
    sc = _scenarios(6, seed=7, m_scale=0.25, draws=(500, 2000))
    probs = [bmd.Problem(s) for s in sc]
    try:
        one, _ = bmd.eval_batch(probs, [s["n_draws"] for s in sc], "fp32")
        monkeypatch.setenv("BMD_BATCH_BUDGET", "1")
        many, wall = bmd.eval_batch(probs, [s["n_draws"] for s in sc], "fp32")
        monkeypatch.delenv("BMD_BATCH_BUDGET")
        for a, b in zip(one, many):
            assert (a - b).abs().max().item() <= 1e-12
        assert np.all(np.diff(np.sort(wall)) >= 0) and np.all(wall > 0)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_mixed_kernel_kinds(prec):
    """Problems that take the direct sweep at d >= 2 (logistic indicator,
    Formula 10 prior, alpha rules) next to matrix-core ones in one batch."""
    specs = []
    a = W.base_problem(2, [11, 9], 0.3, 0.05, scenario=1)
    a["width"] = 0.01
    b = W.base_problem(3, [6, 5, 7], 0.25, 0.05, scenario=2)
    b.update(effect="paper", paper_a=0.8, paper_b=0.6, paper_events=80.0, info=211.0)
    c = W.base_problem(3, [8, 6, 5], 0.4, 0.05, scenario=3, alpha_rule="bonferroni")
    e = W.base_problem(1, [33], 0.0, 0.05, scenario=4)
    e["width"] = 0.02
    specs = [a, b, c, e]
    draws = [700, 1100, 900, 1300]
    probs = [bmd.Problem(s) for s in specs]
    try:
        kinds = [bmd.sweep_kind(p) for p in probs]
        assert kinds == ["direct", "direct", "matrix", "direct"]
        means, wall = bmd.eval_batch(probs, draws, prec)
        for p, m, M in zip(probs, means, draws):
            ref = p.eval_grid(M, prec)
            assert (m - ref).abs().max().item() <= 1e-12
        assert np.all(wall > 0)
    finally:
        for p in probs:
            p.close()


def test_batch_matches_oracle_sampled():
    sc = _scenarios(8, seed=9, m_scale=0.2, draws=(200, 800))
    probs = [bmd.Problem(s) for s in sc]
    try:
        means, _ = bmd.eval_batch(probs, [s["n_draws"] for s in sc], "fp64")
        m32, _ = bmd.eval_batch(probs, [s["n_draws"] for s in sc], "fp32")
        rng = np.random.default_rng(0)
        for p, s, m, m3 in zip(probs, sc, means, m32):
            G = p.G
            gs = np.unique(np.concatenate([[0, G - 1], rng.integers(0, G, 3)]))
            ref, _ = O.eval_grid(s, gs, s["n_draws"])
            got = m.cpu().numpy()[gs]
            got32 = m3.cpu().numpy()[gs]
            assert np.all(np.abs(got - ref) <= 1e-9 * np.maximum(np.abs(ref), 1e-3)), (s["d"], got, ref)
            assert np.all(np.abs(got32 - ref) <= 1e-5 * np.maximum(np.abs(ref), 1e-3)), (s["d"], got32, ref)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_full_size_scenarios_sampled(prec):
    """Eight problems of the 256-problem batch at full size (grids up to 10^6
    designs, M up to 43,281), sampled designs against the oracle."""
    full = W.batch_scenarios()
    pick = [2, 3, 5, 9, 12, 16, 17, 36]
    sc = [full[i] for i in pick]
    probs = [bmd.Problem(s) for s in sc]
    try:
        means, _ = bmd.eval_batch(probs, [s["n_draws"] for s in sc], prec)
        rng = np.random.default_rng(1)
        for p, s, m in zip(probs, sc, means):
            G = p.G
            gs = np.unique(np.concatenate([[0, G - 1], rng.integers(0, G, 2)]))
            say(f"oracle check d={s['d']} G={G} M={s['n_draws']} {prec}")
            ref, _ = O.eval_grid(s, gs, s["n_draws"])
            got = m.cpu().numpy()[gs]
            tol = 1e-9 if prec == "fp64" else 1e-5
            assert np.all(np.abs(got - ref) <= tol * np.maximum(np.abs(ref), 1e-3)), (s["d"], got, ref)
    finally:
        for p in probs:
            p.close()


def test_batch_single_and_invalid():
    spec = W.base_problem(2, [9, 11], 0.3, 0.05)
    with bmd.Problem(spec) as p:
        (m,), wall = bmd.eval_batch([p], [1234], "fp32")
        ref = p.eval_grid(1234, "fp32")
        assert (m - ref).abs().max().item() <= 1e-12
        assert wall[0] > 0
        with pytest.raises(bmd.BmdError):
            bmd.eval_batch([p], [0], "fp32")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_autotuner_settings_and_fixed_settings(prec):
    """The autotuner picks, per launch kind, draws per LDS chunk, rounds of
    resident workgroups and a launch-bound variant from their candidate sets
    (timed on the device); later batches reuse them.  Tuned and fixed settings
    differ only in how the draws are sliced, so their means agree to the FP64
    summation order, and both agree with the one-problem sweeps."""
    sc = _scenarios(10, seed=11, m_scale=0.25, draws=(400, 4000))
    probs = [bmd.Problem(s) for s in sc]
    M = [s["n_draws"] for s in sc]
    try:
        bmd.batch_autotune(2)   # forget earlier tuning: this batch tunes
        tuned, _ = bmd.eval_batch(probs, M, prec)
        kinds = sorted({(p.d, 1 if bmd.sweep_kind(p) == "matrix" else 0) for p in probs})
        step = 8 if prec == "fp32" else 4
        for d, kind in kinds:
            st = bmd.batch_settings(prec, d, kind)
            assert st is not None, (d, kind)
            say(f"tuned {prec} d={d} kind={kind}: {st}")
            if kind == 1:
                assert st["chunk"] == 0 or (st["chunk"] % step == 0 and step <= st["chunk"] <= 32)
            else:
                assert st["chunk"] == 0
            assert st["rounds"] in (2, 4, 8, 16)
            assert st["variant"] in ((0, 1) if (prec == "fp32" and kind == 1) else (0,))
            assert st["calibration_us"] > 0
        again, _ = bmd.eval_batch(probs, M, prec)   # reuses the tuned settings
        for a, b in zip(tuned, again):
            assert torch.equal(a, b)
        bmd.batch_autotune(0)
        fixed, _ = bmd.eval_batch(probs, M, prec)
        for p, s, a, b in zip(probs, sc, tuned, fixed):
            ref = p.eval_grid(s["n_draws"], prec)
            torch.cuda.synchronize()
            assert (a - b).abs().max().item() <= 1e-13
            assert (a - ref).abs().max().item() <= 1e-12
    finally:
        bmd.batch_autotune(1)
        for p in probs:
            p.close()
