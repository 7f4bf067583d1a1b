"""Host logic of bench.py: the one-GPU contract, the counter-summary reader
and its source digest, and the algorithmic flop count."""
import os
import shutil
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _copy_sources(tmp):
    for sub in ("include", os.path.join("paper_2005_10494_amd", "csrc")):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(tmp, sub),
                        ignore=shutil.ignore_patterns("*.o", "*.so", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "paper_2005_10494_amd", "build.py"), os.path.join(tmp, "paper_2005_10494_amd"))


def test_source_digest_follows_code_not_comments(tmp_path, monkeypatch):
    _copy_sources(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.source_digest()
    assert base == bench.source_digest()
    hdr = tmp_path / "paper_2005_10494_amd" / "csrc" / "device_math.hpp"
    text = hdr.read_text()
    hdr.write_text(text + "\n// a remark\n/* and a block\n   comment */\n")
    assert bench.source_digest() == base            # comments do not reach the code object
    hdr.write_text(text + "\nnamespace bmd { constexpr int kUnused = 1; }\n")
    assert bench.source_digest() != base            # code does
    hdr.write_text(text)
    grad = tmp_path / "paper_2005_10494_amd" / "csrc" / "kernels_grad.hip"
    grad.write_text(grad.read_text() + "\nnamespace bmd { constexpr int kOther = 2; }\n")
    assert bench.source_digest() == base            # not part of the sweep kernel's sources


def test_counter_summary_reader(tmp_path, monkeypatch):
    _copy_sources(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    row = "| `k_eval_mfma<float, 3, 12, false>` | 2.0e+08 | 3.0e+07 | 1 | 2 | 3.9e+10 | 0.945 | 101.0 | 99.7 |"
    good = f"source digest: `{bench.source_digest()}`\n\n| kernel | a | b | c | d | e | f | g | h |\n|---|\n{row}\n"
    (tmp_path / "profiles" / "s.md").write_text(good)
    c = bench.measured_counters("s.md", "k_eval_mfma<float, 3, 12, false>")
    assert c == {"traffic": 2.3e8, "valu_issue_fill": 0.945, "valu_busy_pct": 101.0}
    assert bench.measured_counters("s.md", "k_eval_mfma<double, 3, 24, false>") is None
    (tmp_path / "profiles" / "t.md").write_text(good.replace(bench.source_digest(), "0" * 64))
    assert bench.measured_counters("t.md", "k_eval_mfma<float, 3, 12, false>") is None   # stale counters
    assert bench.measured_counters("missing.md", "k_eval_mfma<float, 3, 12, false>") is None


def test_algorithmic_flops_one_biomarker():
    """d = 1: no overlap quadrature, so F = 23 + 6 n(rho_g) per evaluation."""
    spec = {"d": 1, "m": [4], "effect": "step", "q_lo": 0.05, "q_hi": 0.95}
    r = np.array([0.04, 0.2, 0.5, 0.8, 0.87, 0.93])   # rho = 0.2, 0.447, 0.707, 0.894, 0.933, 0.964
    tau = np.full((10, 1), 0.5)
    f32, o32 = bench.algorithmic_flops(spec, r, tau, "fp32", 4)
    f64, o64 = bench.algorithmic_flops(spec, r, tau, "fp64", 4)
    assert f32 == 10 * sum(23 + 6 * n for n in (4, 4, 6, 8, 10, 12))
    assert f64 == 10 * sum(23 + 6 * n for n in (6, 8, 12, 16, 20, 24))
    assert o32 == 0.0 and o64 == 0.0


def test_algorithmic_flops_overlap_counts_mixed_designs_only():
    """d = 2, one draw with tau = 0.5 on both axes: a design needs the
    quadrature only when its cutoffs sit on both sides of the drawn ones."""
    spec = {"d": 2, "m": [2, 2], "effect": "step", "q_lo": 0.25, "q_hi": 0.75}
    r = np.full(4, 0.01)                     # rho = 0.1: 4 FP32 nodes
    tau = np.array([[0.5, 0.5]])
    K = 8
    f, o = bench.algorithmic_flops(spec, r, tau, "fp32", K)
    # grid q in {0.25, 0.75}^2: (0.25, 0.75) and (0.75, 0.25) are mixed; their
    # overlap sums run on the matrix cores and are counted apart
    assert f == 4 * (23 + 6 * 4)
    assert o == 2 * 2 * K
