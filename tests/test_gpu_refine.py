"""Continuous refinement on the GPU (Sec. 2.3's local step from the best grid
point): the native projected-gradient loop over the gradient kernels against
the oracle's loop on the same draws, and against scipy's maximiser of a
deterministic objective."""
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


@pytest.mark.parametrize("d,q0", [(2, [0.3, 0.7]), (3, [0.2, 0.5, 0.8])])
def test_refine_matches_oracle(d, q0):
    spec = W.base_problem(d, None, 0.3, 0.05, width=0.01)
    M = 1500
    qo, fo, io = O.refine_design(spec, q0, M, max_iter=25, tol=1e-7)
    with bmd.Problem(spec) as p:
        say(f"refine d={d} fp64")
        q64, f64, i64 = p.refine_design(q0, M, "fp64", max_iter=25, tol=1e-7)
        say(f"refine d={d} fp32")
        q32, f32, i32 = p.refine_design(q0, M, "fp32", max_iter=25, tol=1e-7)
    assert i64 == io and io >= 1
    assert np.max(np.abs(q64 - qo)) < 1e-8, (q64, qo)
    assert abs(f64 - fo) <= 1e-9 * max(abs(fo), 1e-3)
    # FP32 gradients steer a nearby path to the same neighbourhood
    assert abs(f32 - fo) <= 2e-4 and np.max(np.abs(q32 - qo)) < 0.02, (q32, qo, f32, fo)


def test_refine_reaches_scipy_maximiser_of_deterministic_objective():
    from scipy.optimize import minimize_scalar
    spec = W.base_problem(1, None, 0.0, 0.05, width=0.02, sd_b0=0.0, sd_b1=0.0, tau_lo=0.55, tau_hi=0.55,
                          mu_b1=0.6)
    f = lambda x: float(O.eval_points(spec, np.array([[x]]), 1, want_var=False)[0])  # noqa: E731
    res = minimize_scalar(lambda x: -f(x), bounds=(0.05, 0.95), method="bounded", options={"xatol": 1e-8})
    with bmd.Problem(spec) as p:
        q, fq, it = p.refine_design([0.2], 4, "fp64", max_iter=200, tol=1e-9)
    assert abs(q[0] - res.x) < 2e-5 and fq >= -res.fun - 1e-10 and it >= 1


def test_refine_improves_the_grid_argmax():
    """Grid sweep, argmax, then refinement from that cell on the same draws: the
    refined objective is at least the best grid value (both are the same
    estimate of Formula 5 at grid points)."""
    spec = W.base_problem(2, [9, 9], 0.3, 0.05, width=0.01)
    M = 2000
    with bmd.Problem(spec) as p:
        surf = p.eval_grid(M, "fp64")
        g, v, cell = p.argmax(surf)
        q0 = p.designs(g, 1).cpu().numpy()[0, :2]
        q, fq, it = p.refine_design(q0, M, "fp64", max_iter=30)
        ob, _, _ = p.grad_design(torch.tensor(q0[None, :]), M, "fp64")
        torch.cuda.synchronize()
    assert abs(ob.item() - v) <= 1e-12
    assert fq >= v - 1e-12 and np.all(q >= 0.05) and np.all(q <= 0.95)
