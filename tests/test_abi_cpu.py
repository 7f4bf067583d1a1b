"""The C-ABI library without a GPU: it loads, exports every symbol that
include/bmd.h declares, its Python descriptor mirrors the C struct, and the
host-side validation rejects bad problems before any device call."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2005_10494_amd as bmd
from paper_2005_10494_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bmd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = bmd.library()
    names = _declared()
    assert "bmd_create_problem" in names and "bmd_grad_design" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(bmd.SIGNATURES), "binding and header disagree"
    out = subprocess.run(["nm", "-D", "--defined-only", bmd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (bmd_\w+)", out))
    assert set(names) <= exported
    assert lib.bmd_abi_version() == bmd.ABI_VERSION == 3


def test_descriptor_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    fields = [f[0] for f in bmd._Desc._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof(bmd_problem_desc, {f}));' for f in fields)
    src.write_text(f"""#include <stdio.h>
#include <stddef.h>
#include "bmd.h"
int main(void) {{ printf("%zu\\n", sizeof(bmd_problem_desc)); {body} return 0; }}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(bmd._Desc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(bmd._Desc, f).offset == off, f


def _create_status(spec):
    lib = bmd.library()
    desc = bmd.make_desc(spec)
    h = ctypes.c_void_p()
    st = lib.bmd_create_problem(ctypes.byref(desc), ctypes.byref(h), None)
    return st, lib.bmd_last_error().decode()


@pytest.mark.parametrize("change,status", [
    ({"d": 0}, -2), ({"d": 7}, -2), ({"q_lo": 0.6, "q_hi": 0.5}, -2), ({"q_lo": 0.0}, -2),
    ({"rho_b": 0.7}, -2), ({"info": -1.0}, -2), ({"alpha0": 0.0}, -2), ({"alpha_rule": 5}, -1),
    ({"effect": 3}, -1), ({"sd_b0": -0.1}, -2), ({"tau_lo": 0.9, "tau_hi": 0.1}, -2),
    ({"width": -1.0}, -2), ({"gh_nodes": 2}, -2), ({"gh_nodes": 6}, -2), ({"gh_nodes": 132}, -2), ({"bandwidth": [0.0]}, -2),
    ({"m": [1]}, -2), ({"q_lo": 0.01}, -2),   # r = 0.99 > 0.95: bivariate quadrature range
    ({"mu_b1": float("nan")}, -1),
    ({"alpha_rule": "split", "alpha_fixed": (0.0, 0.0)}, -2), ({"alpha_rule": "split", "alpha_fixed": (0.025, 0.0)}, -2),
])
def test_validation_rejects_before_any_launch(change, status):
    spec = W.plain_1d()
    spec.update(change)
    st, msg = _create_status(spec)
    assert st == status, msg
    assert msg


@pytest.mark.parametrize("change,status", [
    ({"effect": "step"}, -1), ({"alpha_rule": "bonferroni"}, -1),
    ({"q_hi": 0.025}, -2), ({"q_hi": 0.03}, -2), ({"r_lo": 0.0}, -2), ({"r_hi": 0.96}, -2),
    ({"r_lo": 0.6, "r_hi": 0.4}, -2), ({"d": 3, "m": [4, 4, 4], "bandwidth": [0.1] * 3}, -2),
    ({"m": [0, 0]}, -2),
])
def test_alpha_design_validation(change, status):
    """The alpha design space (Sec. 2.2 levels, n = 2) rejects what it does not cover."""
    spec = W.alpha_design(8, m_r=5)
    spec.update(change)
    st, msg = _create_status(spec)
    assert st == status, msg
    assert msg


def test_unknown_design_space():
    lib = bmd.library()
    desc = bmd.make_desc(W.alpha_design(8))
    desc.design_space = 7
    h = ctypes.c_void_p()
    assert lib.bmd_create_problem(ctypes.byref(desc), ctypes.byref(h), None) == -1
    assert lib.bmd_last_error()


def test_null_arguments():
    lib = bmd.library()
    assert lib.bmd_create_problem(None, None, None) == -1
    assert lib.bmd_eval_grid(None, 10, 0, None, None, None) == -1
    assert lib.bmd_smooth(None, None, None, 0, None) == -1
    assert lib.bmd_grid_size(None) == 0
    assert lib.bmd_sweep_kind(None) == -1
    assert lib.bmd_gh_nodes(None, 0) == -1
    assert lib.bmd_refine_design(None, None, 10, 0, 5, 1e-6, None, None, None, None) == -1
    assert lib.bmd_eval_grid_levels(None, 10, 0, None, 1, None, None, None) == -1
    assert lib.bmd_optimize_levels(None, 10, 0, 0.001, 0.02, 5, None, None, None) == -1
    assert lib.bmd_eval_grid_dalpha(None, 10, 0, None, None, None) == -1
    assert lib.bmd_eval_grid_two_layer(None, 1024, 4096, 0, 16, 16, None, None, None) == -1
    assert lib.bmd_optimize_levels_newton(None, 10, 0, 0.001, 0.02, 5, 1e-10, None, None, None) == -1
    assert lib.bmd_smooth_tps(None, None, 0.0, None, None, None) == -1
    assert lib.bmd_tps_at(None, None, None, None, None, None) == -1
    assert lib.bmd_refine_tps(None, None, 5, 1e-9, None, None, None, None) == -1
    lib.bmd_destroy_problem(None)  # NULL-safe


def test_workloads_are_inputs_only():
    # the shared input module must not import the oracle or the library
    src = open(W.__file__).read()
    assert "oracle" not in src.split('"""')[-1] and "ctypes" not in src
    assert W.plain_3d()["m"] == [64, 64, 64] and W.precision_5d()["n_draws"] == 200_000
    sc = W.batch_scenarios(16)
    assert all(1 <= s["d"] <= 6 and 1e4 <= s["n_draws"] <= 1e6 for s in sc)


@pytest.mark.parametrize("change,status", [
    ({"effect": "step"}, -1), ({"alpha_rule": "bonferroni"}, -1), ({"q_hi": 0.025}, -2),
    ({"r_lo": 0.1, "r_hi": 0.2}, -2), ({"r_lo": 0.95}, -2), ({"r_hi": 0.0}, -2),
    ({"r_lo": 0.9, "r_hi": 0.899}, -2),   # partial correlation above 0.975
    ({"d": 1, "m": [5], "bandwidth": [0.1]}, -2), ({"m": [0, 0]}, -2),
])
def test_alpha3_design_validation(change, status):
    """Three nested populations (Sec. 2.2, n = 3) reject what they do not cover."""
    spec = W.alpha3_design(5)
    spec.update(change)
    st, msg = _create_status(spec)
    assert st == status, msg
    assert msg


@pytest.mark.parametrize("change,status", [
    ({"effect": "step"}, -1), ({"alpha_rule": "bonferroni"}, -1), ({"q_hi": 0.025}, -2),
    ({"r_4": 0.0}, -2), ({"r_4": 0.5}, -2), ({"r_lo": 0.95}, -2), ({"r_lo": 0.4, "r_hi": 0.5}, -2),
    ({"r_lo": 0.9, "r_hi": 0.899}, -2),                 # third on second given first above 0.975
    ({"r_lo": 0.5, "r_hi": 0.49, "r_4": 0.1}, -2),      # r_3 above 0.95 r_2
    ({"r_lo": 0.9, "r_hi": 0.5, "r_4": 0.499}, -2),     # fourth and third given second above 0.975
    ({"d": 2, "m": [5, 5], "bandwidth": [0.1] * 2}, -2), ({"m": [0, 0, 0]}, -2),
])
def test_alpha4_design_validation(change, status):
    """Four nested populations (Sec. 2.2, n = 4) reject what they do not cover."""
    spec = W.alpha4_design(5)
    spec.update(change)
    st, msg = _create_status(spec)
    assert st == status, msg
    assert msg


def test_batch_tuning_calls_validate_on_the_host():
    lib = bmd.library()
    assert lib.bmd_batch_autotune(3) == -1 and lib.bmd_last_error()
    out = (ctypes.c_int32 * 5)()
    assert lib.bmd_batch_settings(0, 0, 1, out) == -2      # no d = 0
    assert lib.bmd_batch_settings(0, 1, 1, out) == -2      # one biomarker has no matrix-core kind
    assert lib.bmd_batch_settings(7, 2, 1, out) == -1      # unknown precision
    assert lib.bmd_batch_settings(0, 2, 1, None) == -1
    assert lib.bmd_batch_settings(1, 3, 1, out) == -6      # nothing tuned in this process
