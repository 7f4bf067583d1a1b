"""MI355X-native hot path for optimal biomarker-cutoff trial designs.

Thin Python binding over ``libbmd.so`` (see ``include/bmd.h``): argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; PyTorch provides device memory and streams.  Importing works without
a GPU; creating a problem needs the built library and a GPU.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["BmdError", "Problem", "library", "FP64", "FP32_COMP", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbmd.so")

FP64, FP32_COMP = 0, 1
_PREC = {"fp64": FP64, "f64": FP64, "fp32": FP32_COMP, "fp32_comp": FP32_COMP, "f32": FP32_COMP}
_ALPHA = {"fwer": 0, "fwer_equal": 0, "bonferroni": 1, "fixed": 2, "split": 3}
_EFFECT = {"step": 0, "paper": 1, "paper_gauss": 1}
_DESIGN = {"cutoffs": 0, "alpha": 1, "alpha3": 2, "alpha4": 3, "nested3": 4, "nested4": 5}
DRAW_FIELDS = 17
DESIGN_FIELDS = 16

_STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EDEVICE", -5: "ENOTSUP", -6: "ESTATE"}


class BmdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bmd {_STATUS.get(status, status)}: {message}")
        self.status = status


class _Desc(ctypes.Structure):
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
        ("paper_events", ctypes.c_double), ("indicator_width", ctypes.c_double),
        ("bandwidth", ctypes.c_double * 6), ("gh_nodes", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("scenario_id", ctypes.c_uint32),
        ("design_space", ctypes.c_int32), ("r_lo", ctypes.c_double), ("r_hi", ctypes.c_double),
        ("r_4", ctypes.c_double),
    ]


_lib = None

#: version of include/bmd.h this binding marshals (its descriptor layout)
ABI_VERSION = 3

#: every entry point declared in include/bmd.h, with (restype, argtypes)
SIGNATURES = {
    "bmd_abi_version": (ctypes.c_int32, []),
    "bmd_last_error": (ctypes.c_char_p, []),
    "bmd_create_problem": (ctypes.c_int, [ctypes.POINTER(_Desc), ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "bmd_destroy_problem": (None, [ctypes.c_void_p]),
    "bmd_grid_size": (ctypes.c_int64, [ctypes.c_void_p]),
    "bmd_gh_nodes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "bmd_sweep_kind": (ctypes.c_int32, [ctypes.c_void_p]),
    "bmd_eval_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_eval_grid_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_smooth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "bmd_argmax": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_grad_design": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "bmd_eval_grid_levels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_optimize_levels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "bmd_eval_grid_two_layer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "bmd_eval_grid_dalpha": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_optimize_levels_newton": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_refine_design": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_eval_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_smooth_at": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_refine_smoothed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "bmd_smooth_tps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_tps_at": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_refine_tps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_batch_autotune": (ctypes.c_int, [ctypes.c_int32]),
    "bmd_batch_settings": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "bmd_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "bmd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_draws": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]),
    "bmd_designs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p]),
}


def library():
    """Load libbmd.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_10494_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.bmd_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI {L.bmd_abi_version()}, this binding needs {ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        msg = library().bmd_last_error()
        raise BmdError(status, msg.decode() if msg else "")


def _prec(p) -> int:
    return _PREC[p.lower()] if isinstance(p, str) else int(p)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _device_buffer(t, n: int, device, name: str, dtype=None):
    """Check a tensor whose pointer goes to the library: on `device`, contiguous,
    `n` elements of `dtype` (float64 by default).  Raises ValueError."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
    return t


def make_desc(spec: dict) -> _Desc:
    """Descriptor from a problem dict (keys as in ``workloads.base_problem``)."""
    D = _Desc()
    d = int(spec["d"])
    D.d = d
    m = spec.get("m")
    for j in range(6):
        D.m[j] = int(m[j]) if (m is not None and j < len(m)) else 0
    D.q_lo = float(spec.get("q_lo", 0.05))
    D.q_hi = float(spec.get("q_hi", 0.95))
    D.rho_b = float(spec.get("rho_b", 0.0))
    D.info = float(spec["info"])
    D.alpha0 = float(spec.get("alpha0", 0.025))
    rule = spec.get("alpha_rule", "fwer")
    D.alpha_rule = _ALPHA[rule] if isinstance(rule, str) else int(rule)
    af = spec.get("alpha_fixed", (0.0, 0.0))
    D.alpha_fixed[0], D.alpha_fixed[1] = float(af[0]), float(af[1])
    eff = spec.get("effect", "step")
    D.effect = _EFFECT[eff] if isinstance(eff, str) else int(eff)
    for k in ("mu_b0", "sd_b0", "mu_b1", "sd_b1", "tau_lo", "tau_hi", "paper_a", "paper_b", "paper_events"):
        setattr(D, k, float(spec.get(k, 0.0)))
    D.indicator_width = float(spec.get("width", 0.0))
    bw = spec.get("bandwidth") or [0.02] * d
    for j in range(6):
        D.bandwidth[j] = float(bw[j]) if j < len(bw) else 0.0
    D.gh_nodes = int(spec.get("gh_nodes", 0))
    D.seed = int(spec.get("seed", 0))
    D.scenario_id = int(spec.get("scenario", 0))
    D.design_space = _DESIGN[spec.get("design", "cutoffs")]
    D.r_lo = float(spec.get("r_lo", 0.0))
    D.r_hi = float(spec.get("r_hi", 0.0))
    D.r_4 = float(spec.get("r_4", 0.0))
    return D


class Problem:
    """One design problem on the current GPU (owns its device constants)."""

    def __init__(self, spec: dict, stream=None):
        import torch
        self.spec = dict(spec)
        self.d = int(spec["d"])
        self._h = ctypes.c_void_p()
        self._desc = make_desc(spec)
        _check(library().bmd_create_problem(ctypes.byref(self._desc), ctypes.byref(self._h), _stream(stream)))
        self.G = int(library().bmd_grid_size(self._h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            library().bmd_destroy_problem(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- entry points ---------------------------------------------------------
    def eval_grid(self, n_draws: int, precision="fp64", want_var=False, out=None, out_var=None, stream=None,
                  noalloc=False):
        """Monte Carlo power at every design (bmd_eval_grid).  noalloc: the
        variant that keeps its workspace in the library's fixed device scratch
        (bmd_eval_grid_noalloc); the outputs are still allocated here unless
        given."""
        import torch
        if out is not None:
            mean = _device_buffer(out, self.G, self.device, "out")
        else:
            mean = torch.empty(self.G, dtype=torch.float64, device=self.device)
        var = None
        if want_var:
            if out_var is not None:
                var = _device_buffer(out_var, self.G, self.device, "out_var")
                if var.data_ptr() == mean.data_ptr():
                    raise ValueError("out and out_var must be different buffers")
            else:
                var = torch.empty(self.G, dtype=torch.float64, device=self.device)
        fn = library().bmd_eval_grid_noalloc if noalloc else library().bmd_eval_grid
        _check(fn(self._h, int(n_draws), _prec(precision), ctypes.c_void_p(mean.data_ptr()),
                  ctypes.c_void_p(var.data_ptr()) if var is not None else None, _stream(stream)))
        return (mean, var) if want_var else mean

    def smooth(self, surface, precision="fp64", out=None, stream=None):
        import torch
        _device_buffer(surface, self.G, self.device, "surface")
        res = _device_buffer(out, self.G, self.device, "out") if out is not None else torch.empty_like(surface)
        if res.data_ptr() == surface.data_ptr():
            raise ValueError("out must not alias surface")
        _check(library().bmd_smooth(self._h, ctypes.c_void_p(surface.data_ptr()), ctypes.c_void_p(res.data_ptr()),
                                    _prec(precision), _stream(stream)))
        return res

    def argmax(self, surface, stream=None):
        _device_buffer(surface, self.G, self.device, "surface")
        idx = ctypes.c_int64()
        val = ctypes.c_double()
        cell = (ctypes.c_int32 * 6)()
        _check(library().bmd_argmax(self._h, ctypes.c_void_p(surface.data_ptr()), ctypes.byref(idx),
                                    ctypes.byref(val), cell, _stream(stream)))
        return int(idx.value), float(val.value), tuple(int(cell[j]) for j in range(self.d))

    def smooth_at(self, surface, q, stream=None):
        """Smoothed surface at the continuous design q: (value, gradient [d],
        Hessian [d, d]) (bmd_smooth_at)."""
        _device_buffer(surface, self.G, self.device, "surface")
        qq = np.ascontiguousarray(np.asarray(q, dtype=np.float64).ravel())
        if qq.size != self.d:
            raise ValueError(f"q has {qq.size} coordinates, the problem {self.d}")
        val = ctypes.c_double()
        grad = np.zeros(self.d)
        hess = np.zeros((self.d, self.d))
        _check(library().bmd_smooth_at(self._h, ctypes.c_void_p(surface.data_ptr()), qq.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(val), grad.ctypes.data_as(ctypes.c_void_p),
                                       hess.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return float(val.value), grad, hess

    def refine_smoothed(self, surface, q0, max_iter: int = 50, tol: float = 1e-9, stream=None):
        """Newton refinement of the smoothed surface from q0 (bmd_refine_smoothed):
        returns (design, smoothed value, steps)."""
        _device_buffer(surface, self.G, self.device, "surface")
        q0 = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).ravel())
        if q0.size != self.d:
            raise ValueError(f"q0 has {q0.size} coordinates, the problem {self.d}")
        q = np.zeros(self.d)
        val = ctypes.c_double()
        it = ctypes.c_int32()
        _check(library().bmd_refine_smoothed(self._h, ctypes.c_void_p(surface.data_ptr()),
                                             q0.ctypes.data_as(ctypes.c_void_p), int(max_iter), float(tol),
                                             q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(val), ctypes.byref(it),
                                             _stream(stream)))
        return q, float(val.value), int(it.value)

    def smooth_tps(self, surface, lam: float, out=None, stream=None):
        """Thin-plate spline fit of the surface's designs with a value and the
        fitted surface at every design (bmd_smooth_tps): returns (surface,
        designs fitted).  The fit stays with the problem for tps_at and
        refine_tps."""
        import torch
        _device_buffer(surface, self.G, self.device, "surface")
        res = _device_buffer(out, self.G, self.device, "out") if out is not None else torch.empty_like(surface)
        if res.data_ptr() == surface.data_ptr():
            raise ValueError("out must not alias surface")
        n = ctypes.c_int64()
        _check(library().bmd_smooth_tps(self._h, ctypes.c_void_p(surface.data_ptr()), float(lam),
                                        ctypes.c_void_p(res.data_ptr()), ctypes.byref(n), _stream(stream)))
        return res, int(n.value)

    def tps_at(self, q, stream=None):
        """The last thin-plate fit at the design q: (value, gradient [d],
        Hessian [d, d]) (bmd_tps_at)."""
        qq = np.ascontiguousarray(np.asarray(q, dtype=np.float64).ravel())
        if qq.size != self.d:
            raise ValueError(f"q has {qq.size} coordinates, the problem {self.d}")
        val = ctypes.c_double()
        grad = np.zeros(self.d)
        hess = np.zeros((self.d, self.d))
        _check(library().bmd_tps_at(self._h, qq.ctypes.data_as(ctypes.c_void_p), ctypes.byref(val),
                                    grad.ctypes.data_as(ctypes.c_void_p), hess.ctypes.data_as(ctypes.c_void_p),
                                    _stream(stream)))
        return float(val.value), grad, hess

    def refine_tps(self, q0, max_iter: int = 50, tol: float = 1e-9, stream=None):
        """Newton refinement on the last thin-plate fit from q0 (bmd_refine_tps):
        returns (design, fitted value, steps)."""
        q0 = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).ravel())
        if q0.size != self.d:
            raise ValueError(f"q0 has {q0.size} coordinates, the problem {self.d}")
        q = np.zeros(self.d)
        val = ctypes.c_double()
        it = ctypes.c_int32()
        _check(library().bmd_refine_tps(self._h, q0.ctypes.data_as(ctypes.c_void_p), int(max_iter), float(tol),
                                        q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(val), ctypes.byref(it),
                                        _stream(stream)))
        return q, float(val.value), int(it.value)

    def grad_design(self, q, n_draws: int, precision="fp32", want_grad=True, stream=None):
        import torch
        q = torch.as_tensor(q).to(device=self.device, dtype=torch.float64).contiguous()
        if q.dim() != 2 or q.shape[1] != self.d or q.shape[0] < 1:
            raise ValueError(f"q: shape {tuple(q.shape)}, expected (B, {self.d}) with B >= 1")
        B = q.shape[0]
        obj = torch.empty(B, dtype=torch.float64, device=self.device)
        gq = torch.empty(B, self.d, dtype=torch.float64, device=self.device) if want_grad else None
        gmu = torch.empty(B, 2, dtype=torch.float64, device=self.device) if want_grad else None
        _check(library().bmd_grad_design(self._h, ctypes.c_void_p(q.data_ptr()), B, int(n_draws), _prec(precision),
                                         ctypes.c_void_p(obj.data_ptr()),
                                         ctypes.c_void_p(gq.data_ptr()) if gq is not None else None,
                                         ctypes.c_void_p(gmu.data_ptr()) if gmu is not None else None,
                                         _stream(stream)))
        return obj, gq, gmu

    def eval_grid_levels(self, n_draws: int, alphas, precision="fp64", stream=None):
        """Best Monte Carlo power per design over first-test levels ``alphas``
        (second level on each design's FWER boundary); returns (best, level index)."""
        import torch
        a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).ravel())
        best = torch.empty(self.G, dtype=torch.float64, device=self.device)
        k = torch.empty(self.G, dtype=torch.int32, device=self.device)
        _check(library().bmd_eval_grid_levels(self._h, int(n_draws), _prec(precision),
                                              a.ctypes.data_as(ctypes.c_void_p), a.size,
                                              ctypes.c_void_p(best.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                              _stream(stream)))
        return best, k

    def optimize_levels(self, n_draws: int, a_lo: float, a_hi: float, n_iter: int = 20, precision="fp64",
                        stream=None):
        """Per-design golden-section search of the first-test level over
        [a_lo, a_hi] (second level on each design's FWER boundary); returns
        (best power, its first level) per design."""
        import torch
        best = torch.empty(self.G, dtype=torch.float64, device=self.device)
        a1 = torch.empty(self.G, dtype=torch.float64, device=self.device)
        _check(library().bmd_optimize_levels(self._h, int(n_draws), _prec(precision), float(a_lo), float(a_hi),
                                             int(n_iter), ctypes.c_void_p(best.data_ptr()),
                                             ctypes.c_void_p(a1.data_ptr()), _stream(stream)))
        return best, a1

    def eval_grid_two_layer(self, n_outer: int, n_inner: int, precision="fp64", blocks=(16, 16), want_var=True,
                            stream=None):
        """The two-layer sampling estimate of Formula 7 at every grid design
        (Formula 10 prior) and, with want_var, an unbiased estimate of its
        variance; returns (mean, var or None)."""
        import torch
        mean = torch.empty(self.G, dtype=torch.float64, device=self.device)
        var = torch.empty(self.G, dtype=torch.float64, device=self.device) if want_var else None
        _check(library().bmd_eval_grid_two_layer(self._h, int(n_outer), int(n_inner), _prec(precision),
                                                 int(blocks[0]), int(blocks[1]), ctypes.c_void_p(mean.data_ptr()),
                                                 ctypes.c_void_p(var.data_ptr()) if var is not None else None,
                                                 _stream(stream)))
        return mean, var

    def eval_grid_dalpha(self, n_draws: int, precision="fp64", stream=None):
        """Monte Carlo estimate and its derivative in the first level alpha_1 at
        every grid design (rules "split" and "fixed"); returns (mean, dmean)."""
        import torch
        mean = torch.empty(self.G, dtype=torch.float64, device=self.device)
        dmean = torch.empty(self.G, dtype=torch.float64, device=self.device)
        _check(library().bmd_eval_grid_dalpha(self._h, int(n_draws), _prec(precision),
                                              ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(dmean.data_ptr()),
                                              _stream(stream)))
        return mean, dmean

    def optimize_levels_newton(self, n_draws: int, a_lo: float, a_hi: float, n_iter: int = 20, tol: float = 1e-10,
                               precision="fp64", stream=None):
        """Per-design root of the power's alpha_1 derivative over [a_lo, a_hi]
        (false position, second level on each design's FWER boundary); returns
        (best power, its first level) per design."""
        import torch
        best = torch.empty(self.G, dtype=torch.float64, device=self.device)
        a1 = torch.empty(self.G, dtype=torch.float64, device=self.device)
        _check(library().bmd_optimize_levels_newton(self._h, int(n_draws), _prec(precision), float(a_lo),
                                                    float(a_hi), int(n_iter), float(tol),
                                                    ctypes.c_void_p(best.data_ptr()), ctypes.c_void_p(a1.data_ptr()),
                                                    _stream(stream)))
        return best, a1

    def refine_design(self, q0, n_draws: int, precision="fp64", max_iter=50, tol=1e-6, stream=None):
        """Local maximiser of the Monte Carlo objective from q0 (projected
        gradient ascent in the design box); returns (q, objective, iterations)."""
        q0 = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).reshape(self.d))
        q = np.zeros(self.d)
        obj = ctypes.c_double()
        its = ctypes.c_int32()
        _check(library().bmd_refine_design(self._h, q0.ctypes.data_as(ctypes.c_void_p), int(n_draws),
                                           _prec(precision), int(max_iter), float(tol),
                                           q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(obj),
                                           ctypes.byref(its), _stream(stream)))
        return q, obj.value, its.value

    def profile(self, enable: bool = True):
        _check(library().bmd_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Device ms of the latest profiled phases: draws, sweep, finalize, smooth, argmax."""
        out = np.zeros(5, dtype=np.float64)
        _check(library().bmd_profile_read(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return dict(zip(("draws", "sweep", "finalize", "smooth", "argmax"), out.tolist()))

    def draws(self, k0: int, n: int, stream=None):
        import torch
        u = torch.empty(n, 8, dtype=torch.float64, device=self.device)
        f = torch.empty(n, DRAW_FIELDS, dtype=torch.float64, device=self.device)
        _check(library().bmd_draws(self._h, int(k0), int(n), ctypes.c_void_p(u.data_ptr()),
                                   ctypes.c_void_p(f.data_ptr()), _stream(stream)))
        return u, f

    def designs(self, g0: int, n: int, stream=None):
        import torch
        f = torch.empty(n, DESIGN_FIELDS, dtype=torch.float64, device=self.device)
        _check(library().bmd_designs(self._h, int(g0), int(n), ctypes.c_void_p(f.data_ptr()), _stream(stream)))
        return f


def gh_nodes(problem: "Problem", precision="fp64") -> int:
    return int(library().bmd_gh_nodes(problem.handle, _prec(precision)))


def sweep_kind(problem: "Problem") -> str:
    """'direct' or 'matrix': the sweep kernel eval_grid uses for this problem."""
    k = int(library().bmd_sweep_kind(problem.handle))
    if k < 0:
        raise BmdError(-1, "sweep_kind needs a grid problem")
    return "matrix" if k == 1 else "direct"


def eval_batch(problems, n_draws, precision="fp32", stream=None):
    """Evaluate several grid problems in one launch; returns (means, wall_ms)."""
    import torch
    n = len(problems)
    handles = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    draws = (ctypes.c_uint64 * n)(*[int(x) for x in n_draws])
    outs = [torch.empty(p.G, dtype=torch.float64, device=p.device) for p in problems]
    ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    wall = np.zeros(n, dtype=np.float64)
    _check(library().bmd_eval_batch(handles, n, draws, _prec(precision), ptrs,
                                    wall.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return outs, wall


def batch_autotune(mode: int):
    """bmd_batch_autotune: 1 tune each batch launch kind on first use (the
    default), 0 fixed settings, 2 forget the tuned settings."""
    _check(library().bmd_batch_autotune(int(mode)))


def batch_settings(precision, d: int, kind: int):
    """bmd_batch_settings: the tuned settings of launch kind (d, kind) on the
    current device as a dict, or None when no batch has tuned it yet."""
    out = (ctypes.c_int32 * 5)()
    st = library().bmd_batch_settings(_prec(precision), int(d), int(kind), out)
    if st == -6:
        return None
    _check(st)
    return {"chunk": out[0], "rounds": out[1], "variant": out[2], "waves_per_simd": out[3],
            "calibration_us": out[4]}
