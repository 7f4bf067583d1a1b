"""Differentiation form on the GPU: objective and gradients at continuous
design points against the oracle's forward-mode gradients on the same draws,
and against central finite differences of the GPU's own FP64 objective."""
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
from paper_2005_10494_amd.autograd import objective  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_grad(spec, q, M, prec):
    say(f"grad d={spec['d']} B={len(q)} M={M} width={spec['width']} {prec}")
    with bmd.Problem(spec) as p:
        obj, gq, gmu = p.grad_design(torch.as_tensor(q, device="cuda"), M, prec)
        torch.cuda.synchronize()
        return obj.cpu().numpy(), gq.cpu().numpy(), gmu.cpu().numpy()


def rel_err(a, b, floor):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))


@pytest.mark.parametrize("d,width,B,M", [(1, 0.01, 37, 2000), (1, 0.0, 20, 2000), (2, 0.01, 30, 1000),
                                         (3, 0.0, 17, 600), (3, 0.01, 130, 200), (5, 0.01, 9, 400),
                                         (6, 0.02, 5, 200)])
def test_grad_matches_oracle(d, width, B, M):
    spec = W.base_problem(d, None, 0.3, 0.03, width=width)
    q = W.design_points(B, d, seed=3)
    o_obj, o_gq, o_gmu = O.grad_points(spec, q, M)
    for prec, tol_o, tol_g in (("fp64", 1e-9, 1e-7), ("fp32", 1e-5, 2e-4)):
        obj, gq, gmu = gpu_grad(spec, q, M, prec)
        assert rel_err(obj, o_obj, 1e-3) <= tol_o, prec
        assert rel_err(gq, o_gq, 1e-2) <= tol_g, (prec, rel_err(gq, o_gq, 1e-2))
        assert rel_err(gmu, o_gmu, 1e-2) <= tol_g, (prec, rel_err(gmu, o_gmu, 1e-2))


def test_grad_objective_equals_grid_sweep():
    spec = W.base_problem(3, [6, 5, 7], 0.3, 0.05)
    G = 210
    q = O.grid_points(spec, np.arange(G))
    with bmd.Problem(spec) as p:
        grid = p.eval_grid(500, "fp64").cpu().numpy()
        obj, _, _ = p.grad_design(torch.as_tensor(q, device="cuda"), 500, "fp64")
    assert np.max(np.abs(obj.cpu().numpy() - grid)) < 1e-12


def test_grad_central_differences_fp64():
    spec = W.base_problem(5, None, 0.3, 0.03, width=0.01)
    q = W.design_points(4, 5, seed=11)
    M, h = 3000, 1e-4
    _, gq, gmu = gpu_grad(spec, q, M, "fp64")
    for j in range(5):
        qp, qm = q.copy(), q.copy()
        qp[:, j] += h
        qm[:, j] -= h
        fd = (gpu_grad(spec, qp, M, "fp64")[0] - gpu_grad(spec, qm, M, "fp64")[0]) / (2 * h)
        assert np.all(np.abs(gq[:, j] - fd) <= 1e-4 * np.abs(fd) + 1e-6), (j, gq[:, j], fd)
    for i, key in enumerate(("mu_b0", "mu_b1")):
        sp, sm = dict(spec), dict(spec)
        sp[key] += h
        sm[key] -= h
        fd = (gpu_grad(sp, q, M, "fp64")[0] - gpu_grad(sm, q, M, "fp64")[0]) / (2 * h)
        assert np.all(np.abs(gmu[:, i] - fd) <= 1e-5 * np.abs(fd) + 1e-8)


def test_grad_null_prior_and_invalid_points():
    spec = W.base_problem(3, None, 0.3, 0.03, width=0.01)
    spec.update(mu_b0=0.0, sd_b0=0.0, mu_b1=0.0, sd_b1=0.0)
    q = np.array([[0.3, 0.5, 0.6], [0.2, 0.9, 0.4], [0.01, 0.5, 0.5]])   # last one outside [q_lo, q_hi]
    obj, gq, gmu = gpu_grad(spec, q, 100, "fp64")
    assert np.all(np.abs(obj[:2] - 0.025) < 1e-14)
    assert np.max(np.abs(gq[:2])) < 1e-12
    assert np.all(np.isnan(obj[2:])) and np.all(np.isnan(gq[2:]))


def test_autograd_function():
    spec = W.base_problem(2, None, 0.3, 0.03, width=0.01)
    q = torch.tensor(W.design_points(6, 2, seed=5), device="cuda", requires_grad=True)
    mu = torch.tensor([0.0, 0.5], dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.arange(1, 7, dtype=torch.float64, device="cuda")
    loss = (objective(q, mu, spec, 800, "fp64") * w).sum()
    loss.backward()
    obj, gq, gmu = gpu_grad(spec, q.detach().cpu().numpy(), 800, "fp64")
    wh = w.cpu().numpy()
    assert np.allclose(q.grad.cpu().numpy(), wh[:, None] * gq, rtol=1e-12, atol=1e-15)
    assert np.allclose(mu.grad.cpu().numpy(), (wh[:, None] * gmu).sum(0), rtol=1e-12)


def test_differentiation_config_full_size():
    """4,096 points of the continuous 5-D design, M = 1,000,000 draws, FP32
    adjoint as benchmarked: checked against the FP64 adjoint on every point;
    then the first 64 points against the oracle's forward-mode gradients on the
    first 2,000 draws, in both precisions."""
    spec = W.grad_5d()
    q = W.design_points(spec["n_points"], 5, seed=1)
    M = spec["n_draws"]
    obj32, gq32, gmu32 = gpu_grad(spec, q, M, "fp32")
    obj64, gq64, gmu64 = gpu_grad(spec, q, M, "fp64")
    assert rel_err(obj32, obj64, 1e-3) <= 1e-5
    assert rel_err(gq32, gq64, 1e-2) <= 1e-4
    assert rel_err(gmu32, gmu64, 1e-2) <= 1e-4
    Mo, n = 2000, 64
    say(f"oracle gradients: {n} points x {Mo} draws")
    o_obj, o_gq, o_gmu = O.grad_points(spec, q[:n], Mo)
    for prec, tol_o, tol_g in (("fp64", 1e-9, 1e-7), ("fp32", 1e-5, 2e-4)):
        obj, gq, gmu = gpu_grad(spec, q[:n], Mo, prec)
        assert rel_err(obj, o_obj, 1e-3) <= tol_o, prec
        assert rel_err(gq, o_gq, 1e-2) <= tol_g, (prec, rel_err(gq, o_gq, 1e-2))
        assert rel_err(gmu, o_gmu, 1e-2) <= tol_g, (prec, rel_err(gmu, o_gmu, 1e-2))


def test_differentiation_config_central_differences_fp32():
    """The FP32 adjoint at the differentiation configuration's M = 1e6 against
    central differences (step 1e-4) of the FP64 objective on four of its points:
    1e-4 relative (floor 1e-2 on the gradient's scale)."""
    spec = W.grad_5d()
    q = W.design_points(spec["n_points"], 5, seed=1)[:4]
    M, h = spec["n_draws"], 1e-4
    _, gq, gmu = gpu_grad(spec, q, M, "fp32")
    for j in range(5):
        qp, qm = q.copy(), q.copy()
        qp[:, j] += h
        qm[:, j] -= h
        fd = (gpu_grad(spec, qp, M, "fp64")[0] - gpu_grad(spec, qm, M, "fp64")[0]) / (2 * h)
        assert np.all(np.abs(gq[:, j] - fd) <= 1e-4 * np.maximum(np.abs(fd), 1e-2)), (j, gq[:, j], fd)
    for i, key in enumerate(("mu_b0", "mu_b1")):
        sp, sm = dict(spec), dict(spec)
        sp[key] += h
        sm[key] -= h
        fd = (gpu_grad(sp, q, M, "fp64")[0] - gpu_grad(sm, q, M, "fp64")[0]) / (2 * h)
        assert np.all(np.abs(gmu[:, i] - fd) <= 1e-4 * np.maximum(np.abs(fd), 1e-2)), (key, gmu[:, i], fd)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grad_draw_passes_are_exact(prec, monkeypatch):
    """Draws held in HBM in several passes (a tiny budget) give bit-identical
    sums: the slices and their draws do not change, only when they are made."""
    spec = W.base_problem(3, None, 0.3, 0.03, width=0.01)
    q = torch.tensor(W.design_points(200, 3, seed=5), dtype=torch.float64, device="cuda")
    with bmd.Problem(spec) as p:
        one = p.grad_design(q, 5000, prec)
        monkeypatch.setenv("BMD_GRAD_BUDGET", "1")
        many = p.grad_design(q, 5000, prec)
        monkeypatch.delenv("BMD_GRAD_BUDGET")
    for a, b in zip(one, many):
        assert torch.equal(a, b)

