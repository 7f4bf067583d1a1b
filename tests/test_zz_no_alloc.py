"""bmd_eval_grid_noalloc, the sweep whose workspace is the library's fixed
device scratch, against bmd_eval_grid through the C ABI.

Both run the same kernels on the same draws with the same slicing, so the
means and variances must be equal bit for bit.  Two calls in a row on
different problems, the second smaller, show that the scratch's leftover
contents do not leak into a result; a sweep larger than the scratch is
rejected on the host before any launch.
"""
import sys

import numpy as np
import pytest

from paper_2005_10494_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2005_10494_amd as bmd  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _both(spec, M, prec, want_var):
    with bmd.Problem(spec) as p:
        say(f"noalloc d={spec['d']} G={p.G} M={M} {prec} var={want_var}")
        ref = p.eval_grid(M, prec, want_var=want_var)
        got = p.eval_grid(M, prec, want_var=want_var, noalloc=True)
        torch.cuda.synchronize()
    if want_var:
        return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got]
    return [ref.cpu().numpy()], [got.cpu().numpy()]


def test_noalloc_equals_eval_grid_two_calls():
    # first call: the 3-D configuration's grid (64^3) at 20,000 draws, FP32
    big = W.plain_3d()
    ref, got = _both(big, 20_000, "fp32", False)
    assert np.array_equal(ref[0], got[0])
    # second call, smaller: a 40 x 33 grid, 777 draws, FP64 with variances
    small = W.base_problem(2, [40, 33], 0.3, 0.05)
    ref, got = _both(small, 777, "fp64", True)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    assert np.all(np.isfinite(got[0])) and np.all(got[1] >= 0.0)


def test_noalloc_rejects_sweeps_beyond_the_scratch():
    spec = W.precision_5d()   # 24^5 designs: the partial sums alone exceed the scratch
    with bmd.Problem(spec) as p:
        out = torch.empty(p.G, dtype=torch.float64, device="cuda")
        with pytest.raises(bmd.BmdError) as e:
            p.eval_grid(200_000, "fp32", out=out, noalloc=True)
        assert e.value.status == -2 and "scratch" in str(e.value)
    # after the rejection the scratch still serves a sweep that fits
    small = W.plain_1d()
    with bmd.Problem(small) as p1:
        ref = p1.eval_grid(small["n_draws"], "fp64")
        got = p1.eval_grid(small["n_draws"], "fp64", noalloc=True)
        assert torch.equal(ref, got)
