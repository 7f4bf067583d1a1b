"""Python access to the plain CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` import this module.  The product library
never loads it, and it shares no code with the HIP path.

Problems are plain dicts with the keys of ``paper_2005_10494_amd.workloads``;
this module converts them to the oracle's own C struct.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-ffp-contract=off",
               "-fPIC", "-shared", _SRC, "-lm", "-o", _SO + ".tmp"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("m", ctypes.c_int32 * 6),
        ("q_lo", ctypes.c_double), ("q_hi", ctypes.c_double),
        ("rho_b", ctypes.c_double), ("info", ctypes.c_double), ("alpha0", ctypes.c_double),
        ("alpha_rule", ctypes.c_int32), ("alpha_fixed", ctypes.c_double * 2),
        ("effect", ctypes.c_int32),
        ("mu_b0", ctypes.c_double), ("sd_b0", ctypes.c_double),
        ("mu_b1", ctypes.c_double), ("sd_b1", ctypes.c_double),
        ("tau_lo", ctypes.c_double), ("tau_hi", ctypes.c_double),
        ("paper_a", ctypes.c_double), ("paper_b", ctypes.c_double),
        ("paper_events", ctypes.c_double),
        ("width", ctypes.c_double), ("bandwidth", ctypes.c_double * 6),
        ("seed", ctypes.c_uint64), ("scenario", ctypes.c_uint32),
        ("design_space", ctypes.c_int32), ("r_lo", ctypes.c_double), ("r_hi", ctypes.c_double),
        ("r_4", ctypes.c_double),
    ]


class _Design(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double * 6), ("c", ctypes.c_double * 6),
                ("r", ctypes.c_double), ("rho", ctypes.c_double),
                ("z1", ctypes.c_double), ("z2", ctypes.c_double),
                ("r3", ctypes.c_double), ("z3", ctypes.c_double),
                ("r4", ctypes.c_double), ("z4", ctypes.c_double)]


class _Draw(ctypes.Structure):
    _fields_ = [("u", ctypes.c_double * 8), ("b0", ctypes.c_double), ("b1", ctypes.c_double),
                ("tau", ctypes.c_double * 6), ("t", ctypes.c_double * 6),
                ("PR", ctypes.c_double), ("e1", ctypes.c_double), ("e2", ctypes.c_double),
                ("e3", ctypes.c_double), ("e4", ctypes.c_double)]


_ALPHA = {"fwer": 0, "fwer_equal": 0, "bonferroni": 1, "fixed": 2, "split": 3}
_EFFECT = {"step": 0, "paper": 1, "paper_gauss": 1}
_DESIGN = {"cutoffs": 0, "alpha": 1, "alpha3": 2, "alpha4": 3, "nested3": 4, "nested4": 5}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        D, P, I64, U64, U32 = ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        pp = ctypes.POINTER(_Problem)
        sig = {
            "or_Phi": (D, [D]), "or_phi": (D, [D]), "or_Phiinv": (D, [D]),
            "or_bvn": (D, [D, D, D]), "or_bvn_density": (D, [D, D, D]),
            "or_orthant": (D, [ctypes.c_int, P, D]), "or_zstar": (D, [D, D]), "or_z2_fwer": (D, [D, D, D]),
            "or_tvn": (D, [D, D, D, D, D, D]), "or_z3_fwer": (D, [D, D, D, D, D]), "or_zstar3": (D, [D, D, D]), "or_zstar4": (D, [D, D, D, D]),
            "or_qvn": (D, [P, P]), "or_qvn_nested": (D, [P, P]), "or_z4_fwer": (D, [D, D, D, D, D, D, D]),
            "or_info_units": (D, [D, D, D]),
            "or_philox4x32_10": (None, [P, P, P]), "or_uniform52": (D, [U32, U32]),
            "or_grid_point": (None, [pp, I64, P, P]), "or_grid_size": (I64, [pp]),
            "or_make_design": (None, [pp, P, ctypes.POINTER(_Design)]),
            "or_make_draw": (None, [pp, U64, ctypes.POINTER(_Draw)]),
            "or_overlap": (D, [pp, ctypes.POINTER(_Design), ctypes.POINTER(_Draw)]),
            "or_success": (D, [pp, ctypes.POINTER(_Design), ctypes.POINTER(_Draw)]),
            "or_eval_points": (None, [pp, I64, P, U64, U64, P, P]),
            "or_eval_grid": (None, [pp, I64, P, U64, U64, P, P]),
            "or_eval_grid_dalpha": (None, [pp, I64, P, U64, U64, P, P]),
            "or_eval_grid_two_layer": (None, [pp, I64, P, U64, U64, ctypes.c_int, ctypes.c_int, P, P, P]),
            "or_smooth_direct": (None, [pp, P, P]), "or_smooth_separable": (None, [pp, P, P]),
            "or_smooth_masked": (None, [pp, P, P]), "or_smooth_at": (D, [pp, P, P]),
            "or_argmax": (I64, [I64, P]),
            "or_grad_points": (None, [pp, I64, P, U64, U64, P, P, P]),
            "or_exact_step": (D, [pp, P]), "or_exact_paper": (D, [pp, P]),
            "or_num_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def problem_struct(prob: dict) -> _Problem:
    s = _Problem()
    d = int(prob["d"])
    s.d = d
    m = list(prob.get("m") or [2] * d)
    for j in range(6):
        s.m[j] = int(m[j]) if j < len(m) else 1
    s.q_lo = float(prob.get("q_lo", 0.05))
    s.q_hi = float(prob.get("q_hi", 0.95))
    s.rho_b = float(prob.get("rho_b", 0.0))
    s.info = float(prob["info"])
    s.alpha0 = float(prob.get("alpha0", 0.025))
    rule = prob.get("alpha_rule", "fwer")
    s.alpha_rule = _ALPHA[rule] if isinstance(rule, str) else int(rule)
    af = prob.get("alpha_fixed", (0.0, 0.0))
    s.alpha_fixed[0], s.alpha_fixed[1] = float(af[0]), float(af[1])
    eff = prob.get("effect", "step")
    s.effect = _EFFECT[eff] if isinstance(eff, str) else int(eff)
    for k in ("mu_b0", "sd_b0", "mu_b1", "sd_b1", "tau_lo", "tau_hi",
              "paper_a", "paper_b", "paper_events", "width"):
        setattr(s, k, float(prob.get(k, 0.0)))
    bw = list(prob.get("bandwidth") or [0.02] * d)
    for j in range(6):
        s.bandwidth[j] = float(bw[j]) if j < len(bw) else 1.0
    s.seed = int(prob.get("seed", 0))
    s.scenario = int(prob.get("scenario", 0))
    s.design_space = _DESIGN[prob.get("design", "cutoffs")]
    s.r_lo = float(prob.get("r_lo", 0.0))
    s.r_hi = float(prob.get("r_hi", 0.0))
    s.r_4 = float(prob.get("r_4", 0.0))
    return s


# ---- primitives -------------------------------------------------------------

def Phi(x): return lib().or_Phi(float(x))
def phi(x): return lib().or_phi(float(x))
def Phiinv(p): return lib().or_Phiinv(float(p))
def bvn(h, k, rho): return lib().or_bvn(float(h), float(k), float(rho))
def bvn_density(h, k, rho): return lib().or_bvn_density(float(h), float(k), float(rho))
def zstar(r, alpha0=0.025): return lib().or_zstar(float(r), float(alpha0))
def z2_fwer(z1, r, alpha0=0.025): return lib().or_z2_fwer(float(z1), float(r), float(alpha0))
def tvn(h1, h2, h3, r12, r13, r23): return lib().or_tvn(*map(float, (h1, h2, h3, r12, r13, r23)))
def z3_fwer(z1, z2, r2, r3, alpha0=0.025): return lib().or_z3_fwer(*map(float, (z1, z2, r2, r3, alpha0)))
def zstar3(r2, r3, alpha0=0.025): return lib().or_zstar3(float(r2), float(r3), float(alpha0))
def zstar4(r2, r3, r4, alpha0=0.025): return lib().or_zstar4(float(r2), float(r3), float(r4), float(alpha0))


def qvn(h, R):
    """P(X_i <= h_i, i < 4) for a standard normal X with correlation matrix R (4 x 4)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    assert h.shape == (4,) and R.shape == (4, 4)
    return lib().or_qvn(_ptr(h), _ptr(R))


def qvn_nested(h, r):
    """P(X_i <= h_i, i < 4) for the null correlations of nested populations
    with fractions r = (1, r2, r3, r4)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    assert h.shape == (4,) and r.shape == (4,)
    return lib().or_qvn_nested(_ptr(h), _ptr(r))


def z4_fwer(z1, z2, z3, r2, r3, r4, alpha0=0.025):
    return lib().or_z4_fwer(*map(float, (z1, z2, z3, r2, r3, r4, alpha0)))
def info_units(alpha, beta, delta): return lib().or_info_units(float(alpha), float(beta), float(delta))
def uniform52(wa, wb): return lib().or_uniform52(int(wa), int(wb))


def orthant(v, rho_b):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_orthant(int(v.size), _ptr(v), float(rho_b))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


# ---- model ------------------------------------------------------------------

def grid_size(prob):
    return int(np.prod([int(x) for x in prob["m"][: int(prob["d"])]]))


def grid_point(prob, g):
    s = problem_struct(prob)
    q = np.zeros(6)
    idx = np.zeros(6, dtype=np.int32)
    lib().or_grid_point(ctypes.byref(s), int(g), _ptr(q), _ptr(idx))
    d = s.d
    return q[:d].copy(), idx[:d].copy()


def grid_points(prob, g_list):
    d = int(prob["d"])
    return np.array([grid_point(prob, g)[0] for g in g_list]).reshape(len(g_list), d)


def make_design(prob, q):
    s = problem_struct(prob)
    qq = np.zeros(6)
    qq[: s.d] = q
    ds = _Design()
    lib().or_make_design(ctypes.byref(s), _ptr(qq), ctypes.byref(ds))
    d = s.d
    return {"q": np.array(ds.q[:d]), "c": np.array(ds.c[:d]), "r": ds.r, "rho": ds.rho,
            "z1": ds.z1, "z2": ds.z2, "r3": ds.r3, "z3": ds.z3, "r4": ds.r4, "z4": ds.z4}


def make_draw(prob, k):
    s = problem_struct(prob)
    dr = _Draw()
    lib().or_make_draw(ctypes.byref(s), int(k), ctypes.byref(dr))
    d = s.d
    return {"u": np.array(dr.u[:]), "b0": dr.b0, "b1": dr.b1, "tau": np.array(dr.tau[:d]),
            "t": np.array(dr.t[:d]), "PR": dr.PR, "e1": dr.e1, "e2": dr.e2, "e3": dr.e3, "e4": dr.e4}


def _design_draw(prob, q, k):
    s = problem_struct(prob)
    qq = np.zeros(6)
    qq[: s.d] = q
    ds = _Design()
    dr = _Draw()
    lib().or_make_design(ctypes.byref(s), _ptr(qq), ctypes.byref(ds))
    lib().or_make_draw(ctypes.byref(s), int(k), ctypes.byref(dr))
    return s, ds, dr


def overlap(prob, q, k):
    s, ds, dr = _design_draw(prob, q, k)
    return lib().or_overlap(ctypes.byref(s), ctypes.byref(ds), ctypes.byref(dr))


def success(prob, q, k):
    s, ds, dr = _design_draw(prob, q, k)
    return lib().or_success(ctypes.byref(s), ctypes.byref(ds), ctypes.byref(dr))


def eval_points(prob, q, M, k0=0, want_var=True):
    s = problem_struct(prob)
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, s.d))
    n = q.shape[0]
    mean = np.zeros(n)
    var = np.zeros(n)
    lib().or_eval_points(ctypes.byref(s), n, _ptr(q), int(k0), int(M), _ptr(mean),
                         _ptr(var) if want_var else None)
    return (mean, var) if want_var else mean


def eval_grid(prob, g_list, M, k0=0):
    s = problem_struct(prob)
    g = np.ascontiguousarray(g_list, dtype=np.int64)
    mean = np.zeros(g.size)
    var = np.zeros(g.size)
    lib().or_eval_grid(ctypes.byref(s), g.size, _ptr(g), int(k0), int(M), _ptr(mean), _ptr(var))
    return mean, var


def eval_grid_dalpha(prob, g_list, M, k0=0):
    """Formula 5 estimate and its derivative in the first level alpha_1 at grid
    designs (Appendix A.3's differentiation under the integral, for the nested
    pair with rule "split" or "fixed"); returns (mean, dmean)."""
    s = problem_struct(prob)
    g = np.ascontiguousarray(g_list, dtype=np.int64)
    mean = np.zeros(g.size)
    dmean = np.zeros(g.size)
    lib().or_eval_grid_dalpha(ctypes.byref(s), g.size, _ptr(g), int(k0), int(M), _ptr(mean), _ptr(dmean))
    return mean, dmean


def eval_grid_two_layer(prob, g_list, N1, N2, A=16, B=16):
    """Formula 7, the two-layer sampling estimate (inner layer of Formula 6),
    at grid designs under the Formula 10 prior: outer draws 0..N1-1, inner
    draws 0..N2-1; returns (mean, var, blocks) with the unbiased variance
    estimate from the A x B block counts."""
    s = problem_struct(prob)
    g = np.ascontiguousarray(g_list, dtype=np.int64)
    mean = np.zeros(g.size)
    var = np.zeros(g.size)
    blocks = np.zeros((g.size, A, B), dtype=np.uint32)
    lib().or_eval_grid_two_layer(ctypes.byref(s), g.size, _ptr(g), int(N1), int(N2), int(A), int(B), _ptr(mean),
                                 _ptr(var), _ptr(blocks))
    return mean, var, blocks


def smooth_direct(prob, f):
    s = problem_struct(prob)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().or_smooth_direct(ctypes.byref(s), _ptr(f), _ptr(out))
    return out


def smooth_separable(prob, f):
    s = problem_struct(prob)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().or_smooth_separable(ctypes.byref(s), _ptr(f), _ptr(out))
    return out


def smooth_masked(prob, f):
    s = problem_struct(prob)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().or_smooth_masked(ctypes.byref(s), _ptr(f), _ptr(out))
    return out


def smooth_at(prob, f, q):
    """The Nadaraya-Watson surface of the grid values f at a continuous design q."""
    s = problem_struct(prob)
    f = np.ascontiguousarray(f, dtype=np.float64)
    qq = np.zeros(6)
    qq[: s.d] = q
    return lib().or_smooth_at(ctypes.byref(s), _ptr(f), _ptr(qq))


def argmax(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return int(lib().or_argmax(v.size, _ptr(v)))


def grad_points(prob, q, M, k0=0):
    s = problem_struct(prob)
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, s.d))
    n = q.shape[0]
    obj = np.zeros(n)
    gq = np.zeros((n, s.d))
    gmu = np.zeros((n, 2))
    lib().or_grad_points(ctypes.byref(s), n, _ptr(q), int(k0), int(M), _ptr(obj), _ptr(gq), _ptr(gmu))
    return obj, gq, gmu


def exact_step(prob, q):
    s = problem_struct(prob)
    qq = np.zeros(6)
    qq[: s.d] = q
    return lib().or_exact_step(ctypes.byref(s), _ptr(qq))


def exact_paper(prob, q):
    s = problem_struct(prob)
    qq = np.zeros(6)
    qq[: s.d] = q
    return lib().or_exact_paper(ctypes.byref(s), _ptr(qq))


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_num_threads())


def success_with_draw(prob, q, draw: dict):
    """Success probability for design q and an explicitly given draw."""
    s = problem_struct(prob)
    qq = np.zeros(6)
    qq[: s.d] = q
    ds = _Design()
    lib().or_make_design(ctypes.byref(s), _ptr(qq), ctypes.byref(ds))
    dr = _Draw()
    for j, v in enumerate(draw.get("u", [])):
        dr.u[j] = v
    dr.b0, dr.b1, dr.PR = draw["b0"], draw["b1"], draw["PR"]
    dr.e1, dr.e2 = draw.get("e1", 0.0), draw.get("e2", 0.0)
    for j in range(s.d):
        dr.tau[j] = draw["tau"][j]
        dr.t[j] = draw["t"][j]
    return lib().or_success(ctypes.byref(s), ctypes.byref(ds), ctypes.byref(dr))


# ---- continuous refinement ----------------------------------------------------

REFINE_TRIALS = 8        # step sizes tried per iteration: s, s/2, ..., s/128
REFINE_FIRST_STEP = 0.05  # largest coordinate move of the first trial (quantile units)
REFINE_MAX_STEP = 0.1
REFINE_ARMIJO = 1e-4


def refine_design(prob, q0, M, max_iter=50, tol=1e-6):
    """Local maximiser of the Monte Carlo objective from a start point (Sec. 2.3:
    the grid's best point refined by a gradient method).  Projected gradient
    ascent inside the box [q_lo, q_hi]^d on the objective and gradient of
    grad_points (draws 0..M-1 throughout, so the objective is one deterministic
    function of q).  Each iteration tries the steps q + t_j g / max|g| with
    t_j = s 2^-j, j = 0..7, clipped to the box, and accepts the first that
    gains at least 1e-4 g.(q_j - q) (Armijo); the next s is twice the accepted
    t_j, at most 0.1.  Stops when no trial gains, when the accepted move is
    below tol in every coordinate, or after max_iter iterations.  Returns
    (q, objective at q, iterations)."""
    lo, hi = float(prob["q_lo"]), float(prob["q_hi"])
    q = np.clip(np.asarray(q0, dtype=np.float64), lo, hi)
    f, g, _ = grad_points(prob, q[None, :], M)
    f, g = float(f[0]), g[0]
    s = REFINE_FIRST_STEP
    it = 0
    while it < max_iter:
        gn = float(np.max(np.abs(g)))
        if gn == 0.0:
            break
        t = s * 0.5 ** np.arange(REFINE_TRIALS)
        trials = np.clip(q[None, :] + (t[:, None] / gn) * g[None, :], lo, hi)
        ft, gt, _ = grad_points(prob, trials, M)
        ok = [j for j in range(REFINE_TRIALS) if ft[j] >= f + REFINE_ARMIJO * float(np.dot(g, trials[j] - q))]
        if not ok:
            break
        j = ok[0]
        it += 1
        move = float(np.max(np.abs(trials[j] - q)))
        q, f, g = trials[j].copy(), float(ft[j]), gt[j].copy()
        s = min(2.0 * t[j], REFINE_MAX_STEP)
        if move < tol:
            break
    return q, f, it


# ---- optimal level split per design ----------------------------------------------

def optimize_levels(prob, g_list, M, a_lo, a_hi, n_iter):
    """Sec. 2.4's optimal power at each design found by search: for n = 2 nested
    tests, golden-section search of the first level alpha_1 over [a_lo, a_hi]
    per design, the second level on the design's FWER boundary, on the Formula 5
    estimate with draws 0..M-1 (the same draws for every level, so each design's
    estimate is one deterministic function of alpha_1).  The two interior points
    split the bracket by the golden ratio; the side whose point is lower is
    dropped (ties keep the left part), and one new point is evaluated per step.
    The two ends of the range are evaluated last (a_lo, then a_hi), so a
    maximum at an end is found exactly.  Returns the largest estimate seen per
    design and its level (the first one seen on ties)."""
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    g_list = np.asarray(g_list, dtype=np.int64)
    n = len(g_list)

    def f(levels):
        out = np.empty(n)
        for i in range(n):
            pk = dict(prob, alpha_rule="split", alpha_fixed=(float(levels[i]), 0.0))
            out[i] = eval_grid(pk, g_list[i:i + 1], M)[0][0]
        return out

    a, b = np.full(n, float(a_lo)), np.full(n, float(a_hi))
    x1, x2 = b - gr * (b - a), a + gr * (b - a)
    f1 = f(x1)
    f2 = f(x2)
    best, best_x = f1.copy(), x1.copy()
    up = f2 > best
    best[up], best_x[up] = f2[up], x2[up]
    for _ in range(int(n_iter)):
        left = f1 >= f2
        probe = np.empty(n)
        for i in range(n):
            if left[i]:   # the maximum lies in [a, x2]
                b[i], x2[i], f2[i] = x2[i], x1[i], f1[i]
                x1[i] = b[i] - gr * (b[i] - a[i])
                probe[i] = x1[i]
            else:         # in [x1, b]
                a[i], x1[i], f1[i] = x1[i], x2[i], f2[i]
                x2[i] = a[i] + gr * (b[i] - a[i])
                probe[i] = x2[i]
        fp = f(probe)
        for i in range(n):
            if left[i]:
                f1[i] = fp[i]
            else:
                f2[i] = fp[i]
            if fp[i] > best[i]:
                best[i], best_x[i] = fp[i], probe[i]
    for end in (float(a_lo), float(a_hi)):
        fe = f(np.full(n, end))
        up = fe > best
        best[up], best_x[up] = fe[up], end
    return best, best_x


def optimize_levels_newton(prob, g_list, M, a_lo, a_hi, n_iter, tol):
    """Sec. 2.4's optimal power at each design for n = 2 nested tests, found from
    the derivative (Sec. 2.3 asks for a derivative-driven search; Appendix A.3
    gives the derivative): per design, the root of dP/d alpha_1 in [a_lo, a_hi]
    by the Illinois variant of false position, on the Formula 5 estimate with
    draws 0..M-1 and the second level on the FWER boundary.  Each probe yields
    (P, dP/d alpha_1); the largest P seen and its level are kept (the first one
    on ties after the a_lo probe).  The ends are probed first: a derivative <= 0
    at a_lo or >= 0 at a_hi puts the maximum at that end and the search stops
    there.  Otherwise each of the n_iter steps probes the secant root of the
    bracket's end derivatives (the bracket midpoint if that root is not strictly
    inside), keeps the end whose derivative has the same sign as at the probe on
    the other side, and halves the kept end's derivative when the same end was
    kept twice in a row; a zero derivative or a bracket narrower than tol stops
    the design.  Returns (best, best_alpha1)."""
    g_list = np.asarray(g_list, dtype=np.int64)
    best = np.empty(g_list.size)
    best_x = np.empty(g_list.size)

    def probe(g, a1):
        pk = dict(prob, alpha_rule="split", alpha_fixed=(float(a1), 0.0))
        m, d = eval_grid_dalpha(pk, [g], M)
        return m[0], d[0]

    for i, g in enumerate(g_list):
        lo, hi = float(a_lo), float(a_hi)
        f_lo, g_lo = probe(g, lo)
        f_hi, g_hi = probe(g, hi)
        bf, bx = f_lo, lo
        if f_hi > bf:
            bf, bx = f_hi, hi
        if g_lo > 0.0 and g_hi < 0.0:
            kept = 0   # +1: lo kept last, -1: hi kept last
            for _ in range(int(n_iter)):
                x = (lo * g_hi - hi * g_lo) / (g_hi - g_lo)
                if not (lo < x < hi):
                    x = 0.5 * (lo + hi)
                f, d = probe(g, x)
                if f > bf:
                    bf, bx = f, x
                if d > 0.0:        # the root is above x
                    lo, g_lo = x, d
                    if kept == -1:
                        g_hi *= 0.5
                    kept = -1
                else:
                    hi, g_hi = x, d
                    if kept == 1:
                        g_lo *= 0.5
                    kept = 1
                if d == 0.0 or hi - lo <= tol:
                    break
        best[i], best_x[i] = bf, bx
    return best, best_x


def eval_grid_levels(prob, g_list, M, alphas):
    """Sec. 2.4's optimal power at each design for n = 2 nested tests, over a list
    of first-test levels: for each alpha_1 the second level goes on the FWER
    boundary of the design (its r), Formula 5 is estimated on draws 0..M-1, and
    the largest estimate and the index of its level (ties: the lowest) are kept."""
    best, best_k = None, None
    for k, a1 in enumerate(alphas):
        pk = dict(prob, alpha_rule="split", alpha_fixed=(float(a1), 0.0))
        m, _ = eval_grid(pk, g_list, M)
        if best is None:
            best, best_k = m.copy(), np.zeros(len(m), dtype=np.int64)
        else:
            up = m > best
            best[up] = m[up]
            best_k[up] = k
    return best, best_k


# ---------------------------------------------------------------------------
# Thin-plate spline fit of a grid surface (Sec. 2.3 fits a thin-plate spline
# to the noisy estimates and maximises the fitted surface).  The spline of
# order 2 in d dimensions (Duchon): f(u) = sum_i c_i phi(|u - u_i|) + a_0 +
# sum_j a_j u_j, phi(r) = r^3 (d = 1), r^2 log r (d = 2), -r (d = 3), with the
# coefficients of the smoothing system
#   (Phi + lam I) c + P a = y,   P^T c = 0,   P = [1, u],
# on the designs with a value (not NaN), their coordinates mapped to the unit
# box of the grid (u_j = (q_j - lo_j) / (hi_j - lo_j)).  lam = 0 interpolates.
# The system is solved as written, in one dense solve.
# ---------------------------------------------------------------------------

def _axis_range(prob, j):
    if prob.get("design", "cutoffs") == "alpha" and int(prob["d"]) == 2 and j == 0:
        return float(prob["r_lo"]), float(prob["r_hi"])
    return float(prob["q_lo"]), float(prob["q_hi"])


def tps_phi(d, r):
    r = np.asarray(r, dtype=np.float64)
    if d == 1:
        return r ** 3
    if d == 2:
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(r > 0.0, r * r * np.log(np.where(r > 0.0, r, 1.0)), 0.0)
    if d == 3:
        return -r
    raise ValueError("thin-plate splines are defined here for d = 1, 2, 3")


def tps_unit(prob, q):
    """Design coordinates q [n, d] mapped to the grid's unit box."""
    d = int(prob["d"])
    q = np.asarray(q, dtype=np.float64).reshape(-1, d)
    lo = np.array([_axis_range(prob, j)[0] for j in range(d)])
    hi = np.array([_axis_range(prob, j)[1] for j in range(d)])
    return (q - lo) / (hi - lo)


def tps_fit(prob, f, lam):
    """Fit to the grid values f (NaN: no value); returns (centres [N, d] in
    unit coordinates, c [N], a [d + 1])."""
    d = int(prob["d"])
    f = np.asarray(f, dtype=np.float64)
    g = np.nonzero(~np.isnan(f))[0]
    u = tps_unit(prob, grid_points(prob, g))
    y = f[g]
    n = len(g)
    R = np.sqrt(((u[:, None, :] - u[None, :, :]) ** 2).sum(-1))
    A = np.zeros((n + d + 1, n + d + 1))
    A[:n, :n] = tps_phi(d, R) + lam * np.eye(n)
    P = np.hstack([np.ones((n, 1)), u])
    A[:n, n:] = P
    A[n:, :n] = P.T
    rhs = np.concatenate([y, np.zeros(d + 1)])
    sol = np.linalg.solve(A, rhs)
    return u, sol[:n], sol[n:]


def tps_value(prob, fit, q):
    """Fitted surface at design coordinates q [n, d] (in chunks of 512 points)."""
    u0, c, a = fit
    d = int(prob["d"])
    u = tps_unit(prob, q)
    out = np.empty(len(u))
    for s in range(0, len(u), 512):
        us = u[s:s + 512]
        R = np.sqrt(((us[:, None, :] - u0[None, :, :]) ** 2).sum(-1))
        out[s:s + 512] = tps_phi(d, R) @ c + a[0] + us @ a[1:]
    return out


def tps_derivatives(prob, fit, q):
    """Value, gradient [d] and Hessian [d, d] in design coordinates at one q,
    from phi's derivatives: with s = u - u_i, r = |s|, the gradient of
    phi(r) is phi'(r) s / r and its Hessian phi'(r)/r I + (phi''(r) - phi'(r)/r)
    s s^T / r^2; chain rule for u_j = (q_j - lo_j) / w_j.  Pinned by central
    differences of tps_value, which scipy's interpolator pins."""
    u0, c, a = fit
    d = int(prob["d"])
    w = np.array([_axis_range(prob, j)[1] - _axis_range(prob, j)[0] for j in range(d)])
    u = tps_unit(prob, q)[0]
    val = a[0] + u @ a[1:]
    gu = a[1:].copy()
    Hu = np.zeros((d, d))
    for ci, ui in zip(c, u0):
        s = u - ui
        r = math.sqrt(float(s @ s))
        val += ci * float(tps_phi(d, r))
        if r == 0.0:   # at a centre its own term adds no derivative (r^2 log r's Hessian diverges, -r has a kink)
            continue
        if d == 1:
            p1, p2 = 3 * r * r, 6 * r
        elif d == 2:
            p1, p2 = r * (2 * math.log(r) + 1), 2 * math.log(r) + 3
        else:
            p1, p2 = -1.0, 0.0
        gu += ci * p1 * s / r
        Hu += ci * (p1 / r * np.eye(d) + (p2 - p1 / r) * np.outer(s, s) / (r * r))
    return float(val), gu / w, Hu / np.outer(w, w)


def smooth_tps(prob, f, lam):
    """The fitted surface at every grid design; NaN where f has no value."""
    f = np.asarray(f, dtype=np.float64)
    fit = tps_fit(prob, f, lam)
    G = f.size
    out = tps_value(prob, fit, grid_points(prob, np.arange(G)))
    out[np.isnan(f)] = np.nan
    return out
