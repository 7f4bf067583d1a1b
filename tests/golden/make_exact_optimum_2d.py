"""Writes exact_optimum_2d.txt: the maximiser of the exactly integrated expected
power (Formula 4, no Monte Carlo; the oracle's exact mode) for two biomarkers
with logistic cutoff indicator width 0.01, correlation 0.3 and the default step
prior, along the diagonal q1 = q2 (the objective is symmetric under swapping
the axes, with their draws).  Calls only the oracle.

Run: python tests/golden/make_exact_optimum_2d.py   (a few minutes on 8 cores)
"""
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def spec():
    from paper_2005_10494_amd import workloads as W
    return W.base_problem(2, None, 0.3, 0.05, width=0.01)


def f(q):
    import oracle as O
    return O.exact_step(spec(), list(q))


def main():
    import numpy as np
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        lo, hi = 0.45, 0.8
        best = None
        for _ in range(3):   # three rounds of 16 diagonal points, each around the last best
            xs = np.linspace(lo, hi, 16)
            vals = pool.map(f, [(x, x) for x in xs])
            i = int(np.argmax(vals))
            # parabola through the best point and its neighbours
            j = min(max(i, 1), len(xs) - 2)
            a, b, c = vals[j - 1], vals[j], vals[j + 1]
            h = xs[1] - xs[0]
            den = a - 2 * b + c
            x = xs[j] + (0.5 * h * (a - c) / den if den < 0 else 0.0)
            best = (x, f((x, x)))
            lo, hi = x - 2 * h, x + 2 * h
        x, v = best
        d = 0.01   # off the diagonal: a maximum, not a saddle
        side = pool.map(f, [(x + d, x - d), (x - d, x + d)])
    assert max(side) < v, (side, v)
    with open(os.path.join(HERE, "exact_optimum_2d.txt"), "w") as fh:
        fh.write("# q* on the diagonal and f(q*) of the exact expected power, two biomarkers (rho_b 0.3),\n")
        fh.write("# logistic width 0.01, default step prior; written by make_exact_optimum_2d.py (oracle only)\n")
        fh.write(f"q_star {x:.6f}\nf_star {v:.12f}\nf_off_diagonal {max(side):.12f}\n")
    print(x, v, side)


if __name__ == "__main__":
    main()
