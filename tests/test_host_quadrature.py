"""Host construction of the Gauss rules used by the kernels (no GPU):
compiled from the library's own source into a tiny driver and compared with
numpy's Gauss-Hermite (probabilists') and Gauss-Legendre rules."""
import os
import subprocess

import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from numpy.polynomial.legendre import leggauss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_10494_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "bmd_internal.hpp"
int main() {
  for (int n : {4, 8, 16, 24, 32, 48, 64, 96, 128}) {
    std::vector<double> x(n), w(n); bmd::gauss_hermite_prob(n, x.data(), w.data());
    for (int i = 0; i < n; ++i) printf("H %d %d %.17g %.17g\n", n, i, x[i], w[i]); }
  for (int n : {4, 6, 8, 10, 12, 16, 20, 24}) {
    std::vector<double> x(n), w(n); bmd::gauss_legendre(n, x.data(), w.data());
    for (int i = 0; i < n; ++i) printf("L %d %d %.17g %.17g\n", n, i, x[i], w[i]); }
  std::vector<double> t(200); bmd::gl_table(t.data());
  for (double v : t) printf("T %.17g\n", v);
}
"""


def test_gauss_rules_match_numpy(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, str(src), os.path.join(CSRC, "quad_nodes.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    rows = [line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines()]
    table = [float(r[1]) for r in rows if r[0] == "T"]
    for kind, n, i, x, w in (r for r in rows if r[0] in "HL"):
        n, i, x, w = int(n), int(i), float(x), float(w)
        if kind == "H":
            xr, wr = hermegauss(n)
            wr = wr / np.sqrt(2 * np.pi)
        else:
            xr, wr = leggauss(n)
        assert abs(x - xr[i]) <= 1e-13 * max(1.0, abs(xr[i])), (kind, n, i)
        assert abs(w - wr[i]) <= 1e-12 * wr[i] + 1e-300, (kind, n, i)
    # packed table: rules 4, 6, 8, 10, 12, 16, 20, 24, nodes then weights
    off = 0
    for n in (4, 6, 8, 10, 12, 16, 20, 24):
        xr, wr = leggauss(n)
        assert np.allclose(table[off:off + n], xr, atol=1e-14) and np.allclose(table[off + n:off + 2 * n], wr, rtol=1e-12)
        off += 2 * n
    assert off == 200
