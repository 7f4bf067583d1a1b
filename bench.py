"""Benchmark of the design-objective hot path on one MI355X.

One step = the whole grid hot path on one synthetic problem: per-design
precompute (grid, subgroup fraction, critical values), prior draws, the
designs x draws sweep of the Formula 5 estimate, separable smoothing and the
argmax.  Workload (default): three correlated biomarkers (rho_b = 0.3), a 64^3
cutoff grid, M = 100,000 draws, bandwidth 0.03.  `value` is integrand
evaluations per second of the FP32+FP64-sum path over whole steps; the plain
FP64 path is timed the same way beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "integrand evals/sec and % VALU roofline, FP32+comp vs FP64, at |Δobj|≤1e-5"
PEAK_FP32_TFLOPS = 157.3          # published dense FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop x 2.4 GHz, unpacked FMA
PEAK_FP64_TFLOPS = 78.6
# The paper's two-layer estimator rate, derived from its reported total time (V100): at least
# 2,000 x 10,240 x 20,480 comparisons in 4.5 h / 513 problems.
PAPER_TWO_LAYER_RATE = 1.3e10
SWEEP_KERNEL = {"direct": "k_eval_direct<float,%d,12,false> (designs x draws sweep, one design per thread)",
                "matrix": "k_eval_mfma<float,%d,12,false> (designs x draws sweep, 16x16 design tiles, overlap on MFMA)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(unit: str = "kernels_eval.hip") -> str:
    """SHA-256 over the code a kernel is built from: the translation unit
    `unit` under csrc/ and every header it includes (transitively, local
    includes), comments and layout removed, plus the build script with its
    compiler flags."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2005_10494_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    seen, todo = [], [os.path.join(csrc, unit)]
    while todo:
        path = todo.pop()
        if path in seen or not os.path.exists(path):
            continue
        seen.append(path)
        for line in open(path):
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                for base in (os.path.dirname(path), csrc, inc):
                    cand = os.path.join(base, m.group(1))
                    if os.path.exists(cand):
                        todo.append(cand)
                        break
    seen.append(os.path.join(ROOT, "paper_2005_10494_amd", "build.py"))
    h = hashlib.sha256()
    for path in sorted(seen):
        h.update(os.path.relpath(path, ROOT).encode())
        text = open(path).read()
        if not path.endswith(".py"):   # code only: comments and layout do not reach the code object
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            text = " ".join(text.split())
        h.update(text.encode())
    return h.hexdigest()


def measured_counters(summary: str, kernel: str):
    """Counter figures of `kernel` from a committed counter summary: HBM bytes
    per launch (fetch + write), VALU issue fill and rocprofv3's VALUBusy; None
    when the summary is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source digest: `([0-9a-f]{64})`", text)
    if not m or m.group(1) != source_digest():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 9 and cells[0] == f"`{kernel}`":
            return {"traffic": float(cells[1]) + float(cells[2]), "valu_issue_fill": float(cells[6]),
                    "valu_busy_pct": float(cells[7])}
    return None


def workload(name: str) -> dict:
    from paper_2005_10494_amd import workloads as W
    return {"3d": W.plain_3d, "1d": W.plain_1d, "5d": W.precision_5d, "alpha": W.alpha_grid}[name]()


# --------------------------------------------------------------- algorithmic work
# Floating-point operations per (design, draw) evaluation, as the method needs
# them (transcendentals count as one operation each), split by the unit that
# executes them in the matrix-core sweep:
#   vector units (VALU):
#     drift and thresholds                    6
#     bivariate normal: 2 Phi (3 each) + h k, (h^2+k^2)/2 (4) + combine (3)  13
#       plus 6 per Gauss-Legendre node (exponent 3, exp 1, weighted sum 2)
#     summand and FP64 sums (1 - p, s1, s2)    4
#   matrix cores (MFMA): the responder-in-subgroup overlap O, only when the
#     design's cutoffs are on both sides of the drawn true cutoffs: d flops per
#     Gauss-Hermite node (the products over axes and the sum over nodes).
PEAK_MFMA_FP32_TFLOPS = 157.3     # published dense FP32 matrix-core peak


def bvn_nodes(rho: np.ndarray, prec: str) -> np.ndarray:
    if prec == "fp64":
        edges, counts = [0.3, 0.5, 0.75, 0.9, 0.95], [6, 8, 12, 16, 20, 24]
    else:
        edges, counts = [0.58, 0.8, 0.91, 0.95], [4, 6, 8, 10, 12]
    return np.asarray(counts)[np.searchsorted(edges, rho, side="right")]


def algorithmic_flops(spec: dict, r: np.ndarray, tau: np.ndarray, prec: str, K: int):
    """Flops of one sweep launch (all designs x all draws): (vector part,
    overlap part)."""
    M = tau.shape[0]
    n = bvn_nodes(np.sqrt(r), prec)
    per_design = 23.0 + 6.0 * n
    valu = float(per_design.sum()) * M
    overlap = 0.0
    d = spec["d"]
    if d >= 2 and spec["effect"] == "step":
        m = spec["m"]
        G = r.size
        # T_j(k) = number of grid cutoffs at or below the drawn tau_j
        T = np.zeros((M, d), dtype=np.int64)
        for j in range(d):
            i = np.arange(m[j])
            q = spec["q_lo"] + ((spec["q_hi"] - spec["q_lo"]) * i) / (m[j] - 1)
            T[:, j] = np.searchsorted(q, tau[:, j], side="right")
        above = np.prod(np.asarray(m)[None, :] - T, axis=1)   # all cutoffs above tau
        below = np.prod(T, axis=1)                             # all below
        mixed = G - above - below
        overlap = float(mixed.sum()) * d * K
    return valu, overlap


# --------------------------------------------------------------- GPU steps

def run_steps(spec, prec, steps, warmup):
    import torch
    import paper_2005_10494_amd as bmd
    M = spec["n_draws"]
    sweep_ms, phase = [], []
    t_total = 0.0
    result = None
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = bmd.Problem(spec)
        p.profile(True)
        mean = p.eval_grid(M, prec)
        smooth = p.smooth(mean, prec)
        idx, val, cell = p.argmax(smooth)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ph = p.profile_read()
        if it >= warmup:
            t_total += t1 - t0
            sweep_ms.append(ph["sweep"])
            phase.append(ph)
        if it == warmup + steps - 1:
            result = dict(mean=mean, smooth=smooth, idx=idx, val=val, cell=cell, problem=p)
        else:
            p.close()
        log(f"  {prec} step {it}{' (warmup)' if it < warmup else ''}: {1e3 * (t1 - t0):.1f} ms, "
            f"sweep {ph['sweep']:.1f} ms, draws {ph['draws']:.2f} ms, smooth {ph['smooth']:.3f} ms")
    avg_phase = {k: float(np.mean([p_[k] for p_ in phase])) for k in phase[0]}
    return t_total, float(np.mean(sweep_ms)), avg_phase, result


def cpu_baseline(spec, budget_s=15.0):
    """The oracle as it stands, on a bounded sample of the same workload:
    random designs of the grid against the workload's full set of draws, as
    many designs as a short calibration run says fit in about ``budget_s``."""
    import oracle as O
    rng = np.random.default_rng(0)
    G = int(np.prod(spec["m"]))
    M = int(spec["n_draws"])
    M_cal, n_cal = min(M, 5000), 16
    t0 = time.perf_counter()
    O.eval_grid(spec, np.sort(rng.choice(G, n_cal, replace=False)), M_cal)   # calibration
    per_eval = (time.perf_counter() - t0) / (M_cal * n_cal)
    n_designs = int(min(G, max(4, budget_s / (per_eval * M))))
    gs = np.sort(rng.choice(G, n_designs, replace=False))
    t0 = time.perf_counter()
    O.eval_grid(spec, gs, M)
    dt = time.perf_counter() - t0
    return {"value": n_designs * M / dt, "unit": "integrand evals/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{n_designs} random designs of the {'x'.join(map(str, spec['m']))} grid x all {M} draws"
                      f" ({n_designs * M} evaluations, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="3d", choices=["3d", "1d", "5d", "alpha", "alpha3", "alpha4", "levels", "grad",
                                                         "refine", "batch", "smooth", "twolayer", "nested3", "nested4", "tps"])
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="batch workload only: scale of the per-axis grids and of the draw range (1 = full size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (3 times): the reference "
                         "kernel that scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the designs or the "
              f"draws over several GPUs is not implemented here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_10494_amd as bmd
    if not os.path.exists(bmd.LIB_PATH):
        from paper_2005_10494_amd import build
        build.build()
    torch.cuda.set_device(0)
    if args.copy_bytes > 0:
        n = args.copy_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 3}), flush=True)
        return
    if args.workload == "grad":
        return bench_grad(args)
    if args.workload == "refine":
        return bench_refine(args)
    if args.workload == "alpha3":
        return bench_alpha3(args)
    if args.workload == "alpha4":
        return bench_alpha4(args)
    if args.workload == "levels":
        return bench_levels(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "smooth":
        return bench_smooth(args)
    if args.workload == "twolayer":
        return bench_two_layer(args)
    if args.workload == "nested3":
        return bench_nested3(args)
    if args.workload == "nested4":
        return bench_nested3(args, n=4)
    if args.workload == "tps":
        return bench_tps(args)
    spec = workload(args.workload)
    M, G = spec["n_draws"], int(np.prod(spec["m"]))
    log(f"workload {args.workload}: d={spec['d']} grid={spec['m']} G={G} M={M}")

    t32, sweep32, ph32, res32 = run_steps(spec, "fp32", args.steps, args.warmup)
    evals = G * M
    value = evals * args.steps / t32
    out = {"metric": METRIC, "value": value, "unit": "integrand evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t32 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": _describe(spec, M),
                      "d": spec["d"], "grid": spec["m"], "n_draws": M, "designs": G,
                      "gauss_hermite_nodes": _gh_nodes(res32["problem"], "fp32")}}

    # algorithmic work of the sweep launch
    p32 = res32["problem"]
    r = p32.designs(0, G)[:, 12].cpu().numpy()
    d = spec["d"]
    _, f = p32.draws(0, M)
    tau = f[:, 5:5 + d].cpu().numpy()
    valu32, over32 = algorithmic_flops(spec, r, tau, "fp32", _gh_nodes(p32, "fp32"))
    achieved = valu32 / (sweep32 * 1e-3) / 1e12
    kind = bmd.sweep_kind(p32)
    summary = f"k_eval_mfma_{d}d_{spec['m'][0]}cube_M{M // 1000}k_counters.md"
    kname = "k_eval_" + ("mfma" if kind == "matrix" else "direct") + "<%s, " + str(d) + ", %d, false>"
    cnt32 = measured_counters(summary, kname % ("float", 12)) or {}
    cnt64 = measured_counters(summary, kname % ("double", 24)) or {}
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP32_TFLOPS, "traffic": cnt32.get("traffic"),
                       "traffic_unit": "bytes per launch (HBM, counter-measured)",
                       "numerator": "vector-unit flops of the launch (bivariate normal, drifts, sums); the "
                                    "overlap sums run on the matrix cores and are reported under 'mfma'",
                       "valu_issue_fill": cnt32.get("valu_issue_fill"),
                       "valu_busy_pct": cnt32.get("valu_busy_pct"),
                       "kernel": SWEEP_KERNEL[kind] % d,
                       "sweep_ms": sweep32, "flops_per_launch": valu32,
                       "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                       "frac_unpacked": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                       "sweep_evals_per_s": evals / (sweep32 * 1e-3)}
    if kind == "matrix":
        mf = over32 / (sweep32 * 1e-3) / 1e12
        out["roofline"]["mfma"] = {"achieved": mf, "peak": PEAK_MFMA_FP32_TFLOPS, "unit": "TFLOP/s",
                                   "frac": mf / PEAK_MFMA_FP32_TFLOPS, "flops_per_launch": over32}
    out["phases_ms"] = ph32

    if not args.no_fp64:
        t64, sweep64, ph64, res64 = run_steps(spec, "fp64", args.steps, args.warmup)
        valu64, _ = algorithmic_flops(spec, r, tau, "fp64", _gh_nodes(res64["problem"], "fp64"))
        flops64 = valu64
        m32, m64 = res32["mean"], res64["mean"]
        s32, s64 = res32["smooth"], res64["smooth"]
        out["fp64"] = {"value": evals * args.steps / t64, "ms_per_step": 1e3 * t64 / args.steps,
                       "sweep_ms": sweep64, "achieved_tflops": flops64 / (sweep64 * 1e-3) / 1e12,
                       "frac_of_fp64_peak": flops64 / (sweep64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                       "valu_issue_fill": cnt64.get("valu_issue_fill"), "valu_busy_pct": cnt64.get("valu_busy_pct")}
        out["fp32_vs_fp64"] = {
            "speedup_step": (evals * args.steps / t32) / (evals * args.steps / t64),
            "speedup_sweep": sweep64 / sweep32,
            "max_abs_diff_objective": float((m32 - m64).abs().max()),
            "max_abs_diff_smoothed": float((s32 - s64).abs().max()),
            "max_rel_diff_smoothed": float(((s32 - s64).abs() / s64.abs().clamp_min(1e-3)).max()),
            "objective_max_fp32": res32["val"], "objective_max_fp64": res64["val"],
            "argmax_cell_fp32": list(res32["cell"]), "argmax_cell_fp64": list(res64["cell"])}
        res64["problem"].close()
    p32.close()

    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(out), flush=True)


def _describe(spec: dict, M: int) -> str:
    grid = "x".join(map(str, spec["m"]))
    if spec.get("design") == "alpha":
        return (f"two nested populations, (r_2, alpha_1) grid {grid} with alpha_2 on the FWER boundary, "
                f"Formula 10 prior D0(r) = {spec['paper_a']} - {spec['paper_b']} r, I_3 = {spec['info']:g}, "
                f"M={M} prior draws, FP32 integrand + FP64 sums, steps = precompute+draws+sweep+smooth+argmax")
    return (f"{spec['d']}-biomarker cutoff grid {grid}, M={M} prior draws, rho_b={spec['rho_b']}, "
            f"bandwidth {spec['bandwidth'][0]}, FP32 integrand + FP64 sums, "
            f"steps = precompute+draws+sweep+smooth+argmax")


def bench_grad(args):
    """Differentiation form: objective and its gradient (cutoffs and prior
    means) at 4,096 continuous 5-biomarker designs, M = 1e6 draws, logistic
    indicator width 0.01; FP32 integrand and FP64 timed the same way."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.grad_5d()
    B, M = spec["n_points"], spec["n_draws"]
    q = torch.tensor(W.design_points(B, spec["d"]), dtype=torch.float64, device="cuda")
    res = {}
    with bmd.Problem(spec) as p:
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                obj, gq, gmu = p.grad_design(q, M, prec)
                torch.cuda.synchronize()
                if it >= args.warmup:
                    ts.append(time.perf_counter() - t0)
                log(f"  grad {prec} step {it}: {1e3 * (time.perf_counter() - t0):.1f} ms")
            res[prec] = (float(np.mean(ts)), obj, gq, gmu)
    t32, o32, g32, m32 = res["fp32"]
    t64, o64, g64, m64 = res["fp64"]
    scale = torch.cat([g64.abs().flatten(), m64.abs().flatten()]).max().clamp_min(1e-12)
    # Algorithmic work per (point, draw): the overlap O and its d cutoff
    # derivatives, per Gauss-Hermite node d mixes b + s (a - b) (2 each), d
    # derivative factors, the product and its accumulation (d + 1) and the
    # prefix/suffix products of the derivatives (3 d): K (7 d + 1); the
    # bivariate normal and its three partials at the smallest FP32 rule
    # (4 nodes: 58), and the d + 3 sums.  A lower bound (larger rules cost more).
    d = spec["d"]
    with bmd.Problem(spec) as p:
        K = _gh_nodes(p, "fp32")
    flops = float(B) * M * (K * (7 * d + 1) + 58 + d + 3)
    achieved = flops / t32 / 1e12
    out = {"metric": "gradient evaluations (design point x draw, objective + d + 2 partials) per second",
           "value": B * M / t32, "unit": "point-draws/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"5-biomarker continuous designs, {B} points U(0.1, 0.9)^5, M={M} draws, "
                                  f"logistic indicator width {spec['width']}, rho_b={spec['rho_b']}",
                      "points": B, "n_draws": M},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                        "kernel": f"k_grad<float, {d}, 12, 2, ·> (one thread per point, draws staged per LDS chunk)",
                        "flops_per_call": flops, "gauss_hermite_nodes": K,
                        "numerator": "overlap and its cutoff derivatives K (7 d + 1), bivariate normal and "
                                     "partials at the 4-node rule (58), sums (d + 3): a lower bound"},
           "fp64": {"value": B * M / t64, "ms_per_step": 1e3 * t64},
           "fp32_vs_fp64": {"speedup": t64 / t32,
                            "max_abs_diff_objective": float((o32 - o64).abs().max()),
                            "max_abs_diff_grad_rel_to_max": float(max((g32 - g64).abs().max(),
                                                                      (m32 - m64).abs().max()) / scale)}}
    print(json.dumps(out), flush=True)


def bench_alpha3(args):
    """Three nested populations (Sec. 3, condition (c)): the 97 x 97 grid of
    levels (alpha_1, alpha_2), alpha_3 on the FWER boundary, M = 1e5 draws."""
    return bench_nested(args, 3)


def bench_alpha4(args):
    """Four nested populations (Sec. 3's three-threshold designs, condition
    (c)'s effects): the 25^3 grid of levels (alpha_1, alpha_2, alpha_3),
    alpha_4 on the FWER boundary, M = 1e5 draws."""
    return bench_nested(args, 4)


def bench_nested(args, n):
    """n nested populations: a step is problem set-up (critical values) +
    draws + sweep + smoothing over the designs that have a last level +
    argmax over them.  FP32 and FP64."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.alpha3_grid() if n == 3 else W.alpha4_grid()
    M, G = spec["n_draws"], int(np.prod(spec["m"]))
    res = {}
    for prec in ("fp32", "fp64"):
        ts, sw = [], []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with bmd.Problem(spec) as p:
                p.profile(True)
                mean = p.eval_grid(M, prec)
                smooth = p.smooth(mean, prec)
                idx, val, cell = p.argmax(smooth)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ph = p.profile_read()
            if it >= args.warmup:
                ts.append(dt)
                sw.append(ph["sweep"])
            log(f"  alpha{n} {prec} step {it}: {1e3 * dt:.1f} ms, sweep {ph['sweep']:.1f} ms")
        res[prec] = (float(np.mean(ts)), float(np.mean(sw)), mean, idx, val, cell)
    t32, s32, m32, i32, v32, c32 = res["fp32"]
    t64, s64, m64, i64, v64, _ = res["fp64"]
    feasible = int((~torch.isnan(m32)).sum().item())
    evals = feasible * M
    a_best = [spec["q_lo"] + (spec["q_hi"] - spec["q_lo"]) * c / (m - 1) for c, m in zip(c32, spec["m"])]
    r2, r3 = spec["r_lo"], spec["r_hi"]
    if n == 3:
        # Per summand: three means (12) and, per panel point, the point (2), the two
        # conditional arguments (6), the Gaussian factor (3), two Phi (3 each) and
        # the weighted product and sum (5): 22.
        scale = min(np.sqrt((1 - r2) / r2), np.sqrt((r2 - r3) / r3))
        npan = max(3, min(64, int(np.ceil(2.5 / scale))))   # FP32 panel rule
        per_point, nb = 22.0, 0
        flops = feasible * M * (12.0 + npan * 8 * per_point)
        kernel = (f"k_eval_three<float,false> (one design per thread, {npan} panels x 8 points "
                  f"of two univariate CDFs given the middle statistic)")
    else:
        # Per summand: four means (20) and, per panel point, the point (2), three
        # conditional arguments (9), the Gaussian factor (3), one Phi (3), the
        # bivariate normal of the last two given the second (13 + 6 per node)
        # and the weighted product and sum (5): 35 + 6 nb.
        r4 = spec["r_4"]
        scale = min(np.sqrt((1 - r2) / r2), np.sqrt((r2 - r3) / r3), np.sqrt((r2 - r4) / r4))
        npan = max(3, min(64, int(np.ceil(2.5 / scale))))
        rho = np.sqrt(r4 * (r2 - r3) / (r3 * (r2 - r4)))
        nb = int(bvn_nodes(np.array([rho]), "fp32")[0])
        per_point = 35.0 + 6.0 * nb
        flops = feasible * M * (20.0 + npan * 8 * per_point)
        kernel = (f"k_eval_four<float,false> (one design per thread, {npan} panels x 8 points of a univariate "
                  f"and a {nb}-node bivariate CDF given the second statistic)")
    achieved = flops / (1e-3 * s32) / 1e12
    levels = ", ".join(f"alpha_{i + 1}" for i in range(n - 1))
    rs = ", ".join(str(x) for x in [spec["r_lo"], spec["r_hi"]] + ([spec["r_4"]] if n == 4 else []))
    out = {"metric": f"{'three' if n == 3 else 'four'}-population alpha grid: integrand evals/s", "value": evals / t32,
           "unit": "integrand evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{'three' if n == 3 else 'four'} nested populations r = (1, {rs}), "
                                  f"({levels}) grid {'x'.join(str(m) for m in spec['m'])} over "
                                  f"[{spec['q_lo']}, {spec['q_hi']}], alpha_{n} on the FWER boundary, Formula 10 "
                                  f"prior D0(r) = {spec['paper_a']} - {spec['paper_b']} r, I_3 = {spec['info']:g}, "
                                  f"M={M}, smoothing sd {spec['bandwidth'][0]} on every axis, steps = precompute+draws+"
                                  f"sweep+smooth+argmax over feasible designs",
                      "designs": G, "feasible_designs": feasible, "n_draws": M},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                        "frac": achieved / 157.3, "traffic": None, "kernel": kernel, "flops_per_launch": flops},
           "sweep_ms": s32, "sweep_evals_per_s": evals / (1e-3 * s32),
           "result": {"best_alpha": a_best, "best_power_smoothed": v32,
                      "raw_power_at_best": float(m32[i32].item())},
           "fp64": {"ms_per_step": 1e3 * t64, "sweep_ms": s64},
           "fp32_vs_fp64": {"speedup_sweep": s64 / s32,
                            "max_abs_diff_objective": float(np.nanmax((m32 - m64).abs().cpu().numpy())),
                            "argmax_fp32": int(i32), "argmax_fp64": int(i64)}}
    print(json.dumps(out), flush=True)


def bench_nested3(args, n=3):
    """n = 3 (4) nested populations cut from one biomarker by two (three)
    cutoffs: the 64 x 64 (24^3) grid of cutoff quantiles over [0.1, 0.9], one
    z* on the FWER boundary per design, step prior, M = 1e5.  A step is
    problem set-up (critical values and launch order) + draws + sweep +
    smoothing over the designs that exist + argmax.  FP32 and FP64."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.nested3_grid() if n == 3 else W.nested4_grid()
    M, G = spec["n_draws"], int(np.prod(spec["m"]))
    res = {}
    for prec in ("fp32", "fp64"):
        ts, sw = [], []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with bmd.Problem(spec) as p:
                p.profile(True)
                mean = p.eval_grid(M, prec)
                smooth = p.smooth(mean, prec)
                idx, val, cell = p.argmax(smooth)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ph = p.profile_read()
            if it >= args.warmup:
                ts.append(dt)
                sw.append(ph["sweep"])
            log(f"  nested{n} {prec} step {it}: {1e3 * dt:.1f} ms, sweep {ph['sweep']:.1f} ms")
        res[prec] = (float(np.mean(ts)), float(np.mean(sw)), mean, idx, val, cell)
    t32, s32, m32, i32, v32, c32 = res["fp32"]
    t64, s64, m64, i64, v64, _ = res["fp64"]
    exists = ~np.isnan(m32.cpu().numpy())
    feasible = int(exists.sum())
    evals = feasible * M
    m0 = spec["m"][0]
    q = spec["q_lo"] + (spec["q_hi"] - spec["q_lo"]) * np.arange(m0) / (m0 - 1)
    qs = [a.ravel() for a in np.meshgrid(*([q] * (n - 1)), indexing="ij")]
    rr = [1.0 - qq[exists] for qq in qs]
    if n == 3:
        # Per summand: the three means and 1 - Phi_3 with the sums (22) and, per
        # panel point, 22 as for the three-population sweep; the panel count is
        # each design's own under the FP32 rule (the sweep runs a wavefront at
        # its largest count, which the launch order keeps close to every lane's).
        r2, r3 = rr
        scale = np.minimum(np.sqrt((1 - r2) / r2), np.sqrt((r2 - r3) / r3))
        npan = np.clip(np.ceil(2.5 / scale), 3, 64)
        flops = float(M * np.sum(22.0 + npan * 8 * 22.0))
        kern = f"k_eval_nested3<float,false> (one design per thread, {npan.min():.0f}..{npan.max():.0f} panels " \
               f"(mean {npan.mean():.2f}) x 8 points of two univariate CDFs given the middle statistic)"
    else:
        # Per summand: four means and the sums (28) and, per panel point,
        # 35 + 6 nb as for the four-population sweep, with each design's own
        # panel and bivariate node counts under the FP32 rules.
        r2, r3, r4 = rr
        scale = np.minimum(np.minimum(np.sqrt((1 - r2) / r2), np.sqrt((r2 - r3) / r3)), np.sqrt((r2 - r4) / r4))
        npan = np.clip(np.ceil(2.5 / scale), 3, 64)
        rho = np.sqrt(r4 * (r2 - r3) / (r3 * (r2 - r4)))
        nb = bvn_nodes(rho, "fp32")
        flops = float(M * np.sum(28.0 + npan * 8 * (35.0 + 6.0 * nb)))
        kern = f"k_eval_nested4<float,12,false> (one design per thread, {npan.min():.0f}..{npan.max():.0f} panels " \
               f"(mean {npan.mean():.2f}) x 8 points of a univariate and a {nb.min():.0f}..{nb.max():.0f}-node " \
               f"bivariate CDF given the second statistic)"
    achieved = flops / (1e-3 * s32) / 1e12
    cells = np.unravel_index(i32, spec["m"])
    best = [float(q[c]) for c in cells]
    names = "(q_1, q_2)" if n == 3 else "(q_1, q_2, q_3)"
    out = {"metric": f"{'two' if n == 3 else 'three'}-cutoff grid: integrand evals/s", "value": evals / t32,
           "unit": "integrand evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{'three' if n == 3 else 'four'} nested populations from {n - 1} cutoffs on "
                                  f"one biomarker, {names} grid {'x'.join(str(x) for x in spec['m'])} over "
                                  f"[{spec['q_lo']}, {spec['q_hi']}], one z* on the FWER boundary, "
                                  f"step prior b0 ~ N({spec['mu_b0']}, {spec['sd_b0']}^2), b1 ~ N({spec['mu_b1']}, "
                                  f"{spec['sd_b1']}^2), tau ~ U({spec['tau_lo']}, {spec['tau_hi']}), I = "
                                  f"{spec['info']:g}, M={M}, smoothing sd {spec['bandwidth'][0]} on every axis, "
                                  f"steps = precompute+order+draws+sweep+smooth+argmax over designs that exist",
                      "designs": G, "feasible_designs": feasible, "n_draws": M},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                        "frac": achieved / 157.3, "traffic": None,
                        "kernel": kern, "flops_per_launch": flops},
           "sweep_ms": s32, "sweep_evals_per_s": evals / (1e-3 * s32),
           "result": {"best_q": best, "best_power_smoothed": v32, "raw_power_at_best": float(m32[i32].item())},
           "fp64": {"ms_per_step": 1e3 * t64, "sweep_ms": s64},
           "fp32_vs_fp64": {"speedup_sweep": s64 / s32,
                            "max_abs_diff_objective": float(np.nanmax((m32 - m64).abs().cpu().numpy())),
                            "argmax_fp32": int(i32), "argmax_fp64": int(i64)}}
    print(json.dumps(out), flush=True)


def bench_tps(args):
    """Thin-plate spline smoothing as Sec. 2.3 uses it: the spline fitted to
    the estimates of the three-population 97 x 97 level grid of condition (c)
    (M = 1e5, FP32 integrand; 5,780 designs have a third level), lam = 1e-4
    on the unit box, then the fitted surface's grid argmax refined by Newton
    on the spline.  A step is fit + grid evaluation + argmax + refinement
    (the estimates themselves are computed once, untimed).  FP64."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.alpha3_grid()
    lam = 1e-4
    with bmd.Problem(spec) as p:
        raw = p.eval_grid(spec["n_draws"], "fp32")
        torch.cuda.synchronize()
        m0 = spec["m"][0]
        ts = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, n = p.smooth_tps(raw, lam)
            i, v, cell = p.argmax(s)
            q0 = [spec["q_lo"] + (spec["q_hi"] - spec["q_lo"]) * c / (m - 1) for c, m in zip(cell, spec["m"])]
            q, val, iters = p.refine_tps(q0, max_iter=50, tol=1e-10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if it >= args.warmup:
                ts.append(dt)
            log(f"  tps step {it}: {1e3 * dt:.1f} ms (n = {n}, refine {iters} steps)")
        t = float(np.mean(ts))
    d = spec["d"]
    n2 = n - d - 1
    # algorithmic flops: the Cholesky factorisation (n2^3 / 3 multiply-adds,
    # 2 flops each) and the two-sided reflections (d + 1 of them, 4 n^2 each)
    flops = 2.0 * n2 ** 3 / 3.0 + 4.0 * (d + 1) * n * n
    achieved = flops / t / 1e12
    out = {"metric": "thin-plate spline fit of the level grid: FP64 TFLOP/s", "value": achieved, "unit": "TFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"thin-plate spline (order 2, d = 2: r^2 log r) on the {m0}x{m0} (alpha_1, alpha_2) "
                                  f"grid of three nested populations r = (1, {spec['r_lo']}, {spec['r_hi']}), its "
                                  f"{n} designs with a third level, estimates at M={spec['n_draws']} (FP32), "
                                  f"lam = {lam} on the unit box; step = fit + grid evaluation + argmax + Newton "
                                  f"refinement on the spline", "designs_fitted": n, "lambda": lam},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6,
                        "traffic": None, "kernel": "the whole fit (k_chol_update does the O(n^3) work on the FP64 "
                                                   "matrix cores, 64 x 64 output tiles; priced against the "
                                                   "FP64 vector peak)", "flops_per_call": flops},
           "result": {"best_alpha_grid": [float(x) for x in q0], "best_alpha_refined": [float(x) for x in q],
                      "spline_at_grid_best": v, "spline_at_refined": val, "refine_steps": iters}}
    print(json.dumps(out), flush=True)


def bench_levels(args):
    """Optimal level split per design (Sec. 2.4's optimal power at each design):
    the 3-D bench grid swept at 8 first-test levels 0.0025..0.0200, second
    level on each design's FWER boundary, M = 1e5; FP32 and FP64."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.plain_3d()
    M, G = spec["n_draws"], int(np.prod(spec["m"]))
    alphas = np.linspace(0.0025, 0.02, 8)
    res = {}
    with bmd.Problem(spec) as p:
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                best, k = p.eval_grid_levels(M, alphas, prec)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if it >= args.warmup:
                    ts.append(dt)
                log(f"  levels {prec} step {it}: {1e3 * dt:.1f} ms")
            res[prec] = (float(np.mean(ts)), best, k)
        eq = p.eval_grid(M, "fp32")
        torch.cuda.synchronize()
        # per-design golden-section search of the first level over the same range
        n_iter = 10
        srch = {}
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sb, sa = p.optimize_levels(M, float(alphas[0]), float(alphas[-1]), n_iter, prec)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if it >= args.warmup:
                    ts.append(dt)
                log(f"  level search {prec} step {it}: {1e3 * dt:.1f} ms")
            srch[prec] = (float(np.mean(ts)), sb, sa)
        # per-design false-position search on the alpha_1 derivative, same range
        n_newton = 8
        nwt = {}
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                nb, na = p.optimize_levels_newton(M, float(alphas[0]), float(alphas[-1]), n_newton, 1e-9, prec)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if it >= args.warmup:
                    ts.append(dt)
                log(f"  derivative search {prec} step {it}: {1e3 * dt:.1f} ms")
            nwt[prec] = (float(np.mean(ts)), nb, na)
    # the derivative sweep alone (value and alpha_1 derivative per design) on
    # the split rule at the middle of the level range
    with bmd.Problem(dict(spec, alpha_rule="split", alpha_fixed=(float(np.median(alphas)), 0.0))) as q:
        ts = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q.eval_grid_dalpha(M, "fp32")
            torch.cuda.synchronize()
            if it >= args.warmup:
                ts.append(time.perf_counter() - t0)
        t_dsweep = float(np.mean(ts))
    t32, b32, k32 = res["fp32"]
    t64, b64, k64 = res["fp64"]
    evals = G * M * len(alphas)
    counts = np.bincount(k32.cpu().numpy(), minlength=len(alphas))
    out = {"metric": "optimal level split: integrand evals/s over all levels", "value": evals / t32,
           "unit": "integrand evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3-biomarker cutoff grid 64x64x64, M={M}, first levels "
                                  f"{', '.join(f'{a:.4g}' for a in alphas)}, second level on each design's "
                                  f"FWER boundary", "designs": G, "n_draws": M, "levels": len(alphas)},
           "result": {"best_level_counts": counts.tolist(), "max_best": float(b32.max()),
                      "max_equal_split": float(eq.max()),
                      "mean_gain_over_equal_split": float((b32 - eq).mean())},
           "fp64": {"ms_per_step": 1e3 * t64},
           "fp32_vs_fp64": {"speedup": t64 / t32, "max_abs_diff_best": float((b32 - b64).abs().max()),
                            "level_index_agreement": float((k32 == k64).double().mean())},
           "level_search": {"method": f"golden section per design over [{alphas[0]:.4g}, {alphas[-1]:.4g}], "
                                      f"{n_iter} steps and the two ends ({n_iter + 4} sweeps on shared draws)",
                            "ms_fp32": 1e3 * srch["fp32"][0], "ms_fp64": 1e3 * srch["fp64"][0],
                            "evals_per_s_fp32": G * M * (n_iter + 4) / srch["fp32"][0],
                            "max_best": float(srch["fp32"][1].max()),
                            "mean_gain_over_level_grid": float((srch["fp32"][1] - b32).mean()),
                            "share_above_level_grid": float((srch["fp32"][1] >= b32 - 1e-12).double().mean()),
                            "max_abs_diff_best_fp32_fp64": float((srch["fp32"][1] - srch["fp64"][1]).abs().max())},
           "derivative_search": {
               "method": f"false position on d P / d alpha_1 per design over [{alphas[0]:.4g}, {alphas[-1]:.4g}], "
                         f"{n_newton} steps after the two ends ({n_newton + 2} derivative sweeps on shared draws)",
               "ms_fp32": 1e3 * nwt["fp32"][0], "ms_fp64": 1e3 * nwt["fp64"][0],
               "derivative_sweep_ms_fp32": 1e3 * t_dsweep,
               "max_best": float(nwt["fp32"][1].max()),
               "mean_gain_over_golden": float((nwt["fp32"][1] - srch["fp32"][1]).mean()),
               "share_at_or_above_golden": float((nwt["fp32"][1] >= srch["fp32"][1] - 1e-12).double().mean()),
               "max_abs_diff_best_fp32_fp64": float((nwt["fp32"][1] - nwt["fp64"][1]).abs().max())}}
    print(json.dumps(out), flush=True)


def bench_smooth(args):
    """Smoothing of a grid surface (Sec. 2.3's fit of the noisy estimates): the
    separable Nadaraya-Watson smoother of the 5-biomarker 24^5 grid (bandwidth
    0.03) on a seeded synthetic surface, FP32 and FP64 matrix cores.  Each of
    the d axis passes reads and writes the FP64 surface once (16 G bytes), the
    bound is HBM; the matrix cores do 2 m G flops per pass.  Times are the
    smoothing kernels' device time (HIP events on the launch stream)."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.precision_5d()
    G, d, m = int(np.prod(spec["m"])), spec["d"], spec["m"][0]
    raw = torch.tensor(W.noisy_surface(spec["m"], seed=5), dtype=torch.float64, device="cuda")
    res = {}
    with bmd.Problem(spec) as p:
        p.profile(True)
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                out = p.smooth(raw, prec)
                torch.cuda.synchronize()
                ms = p.profile_read()["smooth"]
                if it >= args.warmup:
                    ts.append(ms)
                log(f"  smooth {prec} step {it}: {ms:.3f} ms")
            res[prec] = (float(np.mean(ts)), out)
    bytes_call = 16.0 * G * d
    flops_call = 2.0 * m * G * d
    t32, s32 = res["fp32"]
    t64, s64 = res["fp64"]
    gbs = bytes_call / (t32 * 1e-3) / 1e9
    out = {"metric": "surface smoothing: HBM GB/s", "value": gbs, "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t32, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"separable Nadaraya-Watson smoothing of a {d}-biomarker "
                                  f"{'x'.join(map(str, spec['m']))} grid surface (seeded synthetic), bandwidth "
                                  f"{spec['bandwidth'][0]}, {d} axis passes", "designs": G},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                        "traffic": None, "kernel": "k_smooth_mfma<float, 2, 2> (axes 0-3) and k_smooth_rows<float, 2, 2> (last axis through LDS), 32 columns x all row blocks per wavefront",
                        "bytes_per_call": bytes_call,
                        "mfma": {"achieved": flops_call / (t32 * 1e-3) / 1e12, "peak": PEAK_MFMA_FP32_TFLOPS,
                                 "unit": "TFLOP/s", "flops_per_call": flops_call}},
           "fp64": {"ms_per_step": t64, "gb_per_s": bytes_call / (t64 * 1e-3) / 1e9},
           "fp32_vs_fp64": {"max_abs_diff": float((s32 - s64).abs().max())}}
    print(json.dumps(out), flush=True)


def bench_two_layer(args):
    """The paper's own estimator (Formula 7 with Formula 6's inner layer) at
    its sizes N1 = 10,240 outer and N2 = 20,480 inner draws (Sec. 2.2) on
    the three-population level grid of condition (c) (97 x 97, alpha_3 on the
    FWER boundary): N1 x N2 comparisons of three coordinates per feasible
    design, counted in 16 x 16 blocks with the unbiased variance estimate.
    Roofline: a comparison of n coordinates costs n compares and one add per
    lane (the and of the masks is scalar), so the vector units can make at
    most 256 CUs x 64 lanes x 2.4 GHz / (n + 1) comparisons per second."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.alpha3_grid()
    N1, N2, n = 10240, 20480, 3
    G = int(np.prod(spec["m"]))
    res = {}
    with bmd.Problem(spec) as p:
        feas = int((~torch.isnan(p.designs(0, G)[:, 7])).sum())
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m, v = p.eval_grid_two_layer(N1, N2, prec)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if it >= args.warmup:
                    ts.append(dt)
                log(f"  two-layer {prec} step {it}: {1e3 * dt:.1f} ms")
            res[prec] = (float(np.mean(ts)), m, v)
        det = p.eval_grid(N1, "fp64")
        torch.cuda.synchronize()
    t32, m32, v32 = res["fp32"]
    t64, m64, v64 = res["fp64"]
    cmp_ = float(feas) * N1 * N2
    rate = cmp_ / t32
    peak = 256 * 64 * 2.4e9 / (n + 1)
    ok = ~torch.isnan(m64)
    sd = torch.sqrt(v64[ok].clamp_min(0))
    i_best = int(torch.nan_to_num(m64, nan=-1.0).argmax())
    out = {"metric": "two-layer estimator (Formula 7): indicator comparisons/s", "value": rate,
           "unit": "comparisons/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": rate / PAPER_TWO_LAYER_RATE,
           "baseline_note": "the paper's two-layer rate, at least 1.3e10 indicator comparisons/s on a V100, derived "
                            "from its 4.5 h for 513 three-population optimisations of 2,000 x 10,240 x 20,480 "
                            "comparisons each",
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"three nested populations r = (1, {spec['r_lo']}, {spec['r_hi']}), (alpha_1, "
                                  f"alpha_2) grid 97x97, alpha_3 on the FWER boundary, Formula 10 prior (condition "
                                  f"(c)), N1={N1} outer x N2={N2} inner draws, 16x16 variance blocks",
                      "designs": G, "feasible_designs": feas, "n_outer": N1, "n_inner": N2},
           "roofline": {"bound": "alu", "achieved": rate, "peak": peak, "unit": "comparisons/s",
                        "frac": rate / peak, "traffic": None,
                        "kernel": "k_two_layer<float, 3> (256 inner draws per workgroup, outer thresholds via LDS)",
                        "comparisons_per_call": cmp_},
           "fp64": {"ms_per_step": 1e3 * t64, "comparisons_per_s": cmp_ / t64},
           "result": {"max_abs_fp32_fp64": float((m32 - m64)[ok].abs().max()),
                      "max_abs_two_layer_minus_formula5": float((m64 - det)[ok].abs().max()),
                      "median_sd_estimate": float(sd.median()), "max_sd_estimate": float(sd.max()),
                      "appendix_a2_sd_bound": math.sqrt(1.0 / (4.0 * N1 * N2)),
                      "best_design": i_best, "best_power": float(m64[i_best])}}
    if not args.no_cpu_baseline:
        import oracle as O
        gs = [int(g) for g in torch.nonzero(ok).flatten()[:2].cpu()]
        t0 = time.perf_counter()
        O.eval_grid_two_layer(spec, gs, N1, N2, 16, 16)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(gs) * N1 * N2 / dt, "unit": "comparisons/s", "cores": 1,
                               "kind": "oracle", "sample": f"{len(gs)} feasible designs x {N1} x {N2} comparisons "
                                                           f"({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


def bench_refine(args):
    """Continuous refinement (Sec. 2.3's local step): projected gradient ascent
    on the 5-biomarker logistic-indicator objective from the centre of the
    design box, M = 1e6 draws, 8 trial points per iteration; FP32 and FP64.
    The value is gradient point-draws per second over the whole refinement."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    spec = W.grad_5d()
    M = spec["n_draws"]
    q0 = np.full(spec["d"], 0.5)
    res = {}
    with bmd.Problem(spec) as p:
        for prec in ("fp32", "fp64"):
            ts = []
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                q, f, n_it = p.refine_design(q0, M, prec, max_iter=40, tol=1e-5)
                dt = time.perf_counter() - t0
                if it >= args.warmup:
                    ts.append(dt)
                log(f"  refine {prec} step {it}: {1e3 * dt:.1f} ms, {n_it} iterations, objective {f:.6f}")
            res[prec] = (float(np.mean(ts)), q, f, n_it)
    t32, q32, f32, n32 = res["fp32"]
    t64, q64, f64, n64 = res["fp64"]
    pd32 = (1 + 8 * n32) * M   # start point and 8 trials per accepted step (a final rejected set not counted)
    out = {"metric": "refinement: gradient point-draws per second (objective + d + 2 partials)",
           "value": pd32 / t32, "unit": "point-draws/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"projected gradient ascent, 5-biomarker continuous design from q = 0.5, "
                                  f"M={M} draws, logistic indicator width {spec['width']}, 8 trials per iteration",
                      "n_draws": M, "iterations": n32},
           "result": {"q": q32.tolist(), "objective": f32},
           "fp64": {"ms_per_step": 1e3 * t64, "iterations": n64, "q": q64.tolist(), "objective": f64},
           "fp32_vs_fp64": {"speedup": t64 / t32, "max_abs_diff_q": float(np.max(np.abs(q32 - q64))),
                            "abs_diff_objective": abs(f32 - f64)}}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batching form: 256 uneven grid problems (d uniform on 1..6, grids
    201/64/40/24/14/10 per axis, M log-uniform in [1e4, 1e6]) in one call."""
    import torch
    import paper_2005_10494_amd as bmd
    from paper_2005_10494_amd import workloads as W
    s = args.batch_scale
    sc = W.batch_scenarios(256, m_scale=s, m_draws=(1e4 * s, 1e6 * s))
    evals = float(sum(int(np.prod(x["m"])) * x["n_draws"] for x in sc))
    log(f"batch: {len(sc)} problems, {evals:.3e} evaluations")
    probs = [bmd.Problem(x) for x in sc]
    kinds_of = [bmd.sweep_kind(p) for p in probs]
    ts, walls, warm_ms = [], None, 0.0
    try:
        bmd.batch_autotune(2)   # tune during the first (warmup) call
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            means, wall = bmd.eval_batch(probs, [x["n_draws"] for x in sc], "fp32")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if it >= args.warmup:
                ts.append(dt)
                walls = wall
            elif it == 0:
                warm_ms = 1e3 * dt
            log(f"  batch step {it}: {1e3 * dt:.1f} ms, last problem done at {wall.max():.1f} ms")
            del means
    except BaseException:
        for p in probs:
            p.close()
        raise
    t = float(np.mean(ts))
    # launch settings the autotuner chose during the warmup call, per launch kind
    kinds = sorted({(x["d"], 1 if k == "matrix" else 0) for x, k in zip(sc, kinds_of)})
    settings = {f"d{d}_{'matrix' if kind else 'direct'}": bmd.batch_settings("fp32", d, kind) for d, kind in kinds}
    # algorithmic work of the call: vector-unit and matrix-core flops of every problem
    valu = mfma = 0.0
    for x, p in zip(sc, probs):
        r = p.designs(0, p.G)[:, 12].cpu().numpy()
        _, f = p.draws(0, x["n_draws"])
        tau = f[:, 5:5 + x["d"]].cpu().numpy()
        v, o = algorithmic_flops(x, r, tau, "fp32", _gh_nodes(p, "fp32"))
        valu += v
        mfma += o
    for p in probs:
        p.close()
    out = {"metric": "aggregate integrand evals/s over a batch of uneven grid problems",
           "value": evals / t, "unit": "integrand evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(sc)} grid problems, d uniform on 1..6, per-axis grid "
                                  f"{'/'.join(str(max(2, round(m * s))) for m in W.BATCH_M)}, M log-uniform in "
                                  f"[{1e4 * s:.0f}, {1e6 * s:.0f}], FP32 integrand + FP64 sums",
                      "problems": len(sc), "evaluations": evals},
           "wall_ms_per_problem": {"p50": float(np.percentile(walls, 50)), "p99": float(np.percentile(walls, 99)),
                                   "max": float(walls.max())},
           "tuning_ms": warm_ms - 1e3 * t, "tuned_settings": settings,
           "roofline": {"bound": "alu", "achieved": valu / t / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": valu / t / 1e12 / PEAK_FP32_TFLOPS, "traffic": None,
                        "numerator": "vector-unit flops of every problem's sweep over the whole call",
                        "kernel": "k_batch<float, d, 12, kind, variant> (one launch per biomarker count and kernel kind)",
                        "flops_per_call": valu,
                        "mfma": {"achieved": mfma / t / 1e12, "peak": PEAK_MFMA_FP32_TFLOPS, "unit": "TFLOP/s",
                                 "frac": mfma / t / 1e12 / PEAK_MFMA_FP32_TFLOPS, "flops_per_call": mfma}}}
    print(json.dumps(out), flush=True)


def _gh_nodes(problem, prec) -> int:
    """Gauss-Hermite node count the library chose (read from its axis tables' size)."""
    import paper_2005_10494_amd as bmd
    return bmd.gh_nodes(problem, prec)


if __name__ == "__main__":
    main()
