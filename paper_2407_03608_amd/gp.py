"""Thin Python binding of libgpnufft (the C ABI of include/gpnufft.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (tensors on ``cuda``) and the current
stream.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpnufft.so")

GP_OK = 0
GP_EINVAL = -1
GP_EDOMAIN = -2
GP_ERANGE = -3
GP_ENOMEM = -4
GP_ENOCONV = -5
GP_EDEVICE = -6
GP_EUNSUPPORTED = -7
GP_FP64 = 0
GP_FP32_BULK = 1
GP_SERVE_FIFO = 0
GP_SERVE_SMALLEST = 1

_c_d = ctypes.c_double
_c_i = ctypes.c_int
_c_i64 = ctypes.c_int64
_c_p = ctypes.c_void_p
_c_sz = ctypes.c_size_t


class GpOpts(ctypes.Structure):
    _fields_ = [
        ("precision", _c_i),
        ("nufft_tol", _c_d),
        ("upsample", _c_d),
        ("n_sigma", _c_i),
        ("n_t", _c_i),
        ("t_min", _c_d),
        ("t_max", _c_d),
        ("dw", _c_d),
        ("M", _c_i64),
        ("M_cap", _c_i64),
        ("s_min", _c_d),
        ("s_max", _c_d),
        ("use_box", _c_i),
        ("box_lo", _c_d * 3),
        ("box_hi", _c_d * 3),
        ("l_lo", _c_d),
        ("l_hi", _c_d),
        ("max_device_bytes", _c_sz),
        ("spread", _c_i),
        ("interp", _c_i),
        ("step3", _c_i),
        ("stream", _c_p),
        ("keep_t", _c_i),
    ]


class GpPlanParams(ctypes.Structure):
    _fields_ = [
        ("d", _c_i),
        ("n", _c_i64),
        ("precision", _c_i),
        ("nu", _c_d),
        ("eta", _c_d),
        ("t_min", _c_d),
        ("t_max", _c_d),
        ("n_t", _c_i),
        ("s_min", _c_d),
        ("s_max", _c_d),
        ("n_sigma", _c_i),
        ("dw", _c_d),
        ("M", _c_i64),
        ("center", _c_d * 3),
        ("scale", _c_d),
        ("nf", _c_i * 3),
        ("w", _c_i),
        ("beta", _c_d),
        ("upsample", _c_d),
        ("nufft_tol", _c_d),
        ("lo", _c_i * 3),
        ("na", _c_i * 3),
        ("tile", _c_i * 3),
        ("n_pairs", _c_i),
        ("device_bytes", _c_sz),
        ("pred_tail", _c_d),
        ("m_capped", _c_i),
        ("step3", _c_i),
        ("spread", _c_i),
        ("interp", _c_i),
        ("a_rows", _c_i64),
        ("n_t_merged", _c_i),
        ("lr_rank_max", _c_i),
        ("lr_rank_mean", _c_d),
    ]


class GpCgInfo(ctypes.Structure):
    _fields_ = [
        ("iters", _c_i),
        ("status", _c_i),
        ("rel_res", _c_d),
        ("rel_res_true", _c_d),
        ("seconds", _c_d),
        ("refinements", _c_i),
    ]


EXPORTS = [
    "gp_opts_init",
    "gp_plan",
    "gp_plan_query",
    "gp_plan_info",
    "gp_matvec",
    "gp_cg_solve",
    "gp_cg_solve_refined",
    "gp_cg_solve_noalloc",
    "gp_cg_solve_multi",
    "gp_posterior_mean",
    "gp_plan_set_stream",
    "gp_plan_destroy",
    "gp_last_error",
    "gp_residual",
    "gp_posterior_cov",
    "gp_plan_rules",
    "gp_plan_set_timing",
    "gp_plan_get_timing",
    "gp_server_opts_init",
    "gp_server_create",
    "gp_server_submit",
    "gp_server_wait",
    "gp_server_poll",
    "gp_server_stats",
    "gp_server_destroy",
]


class GpServerOpts(ctypes.Structure):
    _fields_ = [
        ("max_slots", _c_i),
        ("max_device_bytes", _c_sz),
        ("precision", _c_i),
        ("plan_tol", _c_d),
        ("plan_tol_bulk", _c_d),
        ("cg_tol", _c_d),
        ("inner_tol", _c_d),
        ("max_iter", _c_i),
        ("max_refine", _c_i),
        ("fp64_below_bytes", _c_sz),
        ("policy", _c_i),
        ("aging_bytes_per_s", _c_d),
    ]


class GpRequestInfo(ctypes.Structure):
    _fields_ = [
        ("status", _c_i),
        ("iters", _c_i),
        ("refinements", _c_i),
        ("rel_res", _c_d),
        ("t_submit", _c_d),
        ("t_start", _c_d),
        ("t_done", _c_d),
        ("device_bytes", _c_sz),
        ("slot", _c_i),
        ("precision", _c_i),
        ("t_ready", _c_d),
    ]


class GpServerCounters(ctypes.Structure):
    _fields_ = [
        ("submitted", _c_i64),
        ("completed", _c_i64),
        ("queued", _c_i64),
        ("running", _c_i),
        ("peak_running", _c_i),
        ("bytes_in_use", _c_sz),
        ("peak_bytes", _c_sz),
        ("seconds", _c_d),
    ]

TIMING_PHASES = 10


class GpTiming(ctypes.Structure):
    _fields_ = [
        ("n_phases", _c_i),
        ("name", ctypes.c_char_p * TIMING_PHASES),
        ("launches", _c_i64 * TIMING_PHASES),
        ("ms", _c_d * TIMING_PHASES),
    ]

_lib = None


def load(path: str = LIB_PATH):
    """Load libgpnufft.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} not found: build it first (python -m paper_2407_03608_amd.build); "
            "there is no fallback path")
    L = ctypes.CDLL(path)
    L.gp_opts_init.argtypes = [ctypes.POINTER(GpOpts)]
    L.gp_opts_init.restype = _c_i
    L.gp_plan.argtypes = [_c_i, _c_i64, _c_p, _c_p, _c_p, _c_d, _c_d, _c_d,
                          ctypes.POINTER(GpOpts), ctypes.POINTER(_c_p)]
    L.gp_plan.restype = _c_i
    L.gp_plan_query.argtypes = [_c_i, _c_i64, _c_p, _c_p, _c_p, _c_d, _c_d, _c_d,
                                ctypes.POINTER(GpOpts), ctypes.POINTER(_c_sz)]
    L.gp_plan_query.restype = _c_i
    L.gp_plan_info.argtypes = [_c_p, ctypes.POINTER(GpPlanParams)]
    L.gp_plan_info.restype = _c_i
    L.gp_matvec.argtypes = [_c_p, _c_p, _c_p, _c_i]
    L.gp_matvec.restype = _c_i
    L.gp_cg_solve.argtypes = [_c_p, _c_p, _c_p, _c_i, _c_d, _c_i, _c_i, ctypes.POINTER(GpCgInfo)]
    L.gp_cg_solve.restype = _c_i
    L.gp_cg_solve_multi.argtypes = [_c_p, _c_i, _c_p, _c_p, _c_d, _c_i, _c_i, _c_p, _c_p,
                                    ctypes.POINTER(GpCgInfo)]
    L.gp_cg_solve_multi.restype = _c_i
    L.gp_cg_solve_noalloc.argtypes = [_c_p, _c_p, _c_p, _c_i, _c_d, _c_i, _c_i, ctypes.POINTER(GpCgInfo)]
    L.gp_cg_solve_noalloc.restype = _c_i
    L.gp_cg_solve_refined.argtypes = [_c_p, _c_p, _c_p, _c_p, _c_d, _c_d, _c_i, _c_i, _c_i,
                                      ctypes.POINTER(GpCgInfo)]
    L.gp_cg_solve_refined.restype = _c_i
    L.gp_posterior_mean.argtypes = [_c_p, _c_p, _c_i64, _c_p, _c_p, _c_p, _c_p]
    L.gp_posterior_mean.restype = _c_i
    L.gp_plan_set_stream.argtypes = [_c_p, _c_p]
    L.gp_plan_set_stream.restype = _c_i
    L.gp_plan_destroy.argtypes = [_c_p]
    L.gp_plan_destroy.restype = _c_i
    L.gp_last_error.argtypes = []
    L.gp_last_error.restype = ctypes.c_char_p
    L.gp_residual.argtypes = [_c_p, _c_p, _c_p, ctypes.POINTER(_c_d)]
    L.gp_residual.restype = _c_i
    L.gp_plan_set_timing.argtypes = [_c_p, _c_i]
    L.gp_plan_set_timing.restype = _c_i
    L.gp_plan_rules.argtypes = [_c_i, _c_d, _c_d, _c_d, _c_d, _c_d, ctypes.POINTER(GpOpts),
                                ctypes.POINTER(GpPlanParams)]
    L.gp_plan_rules.restype = _c_i
    L.gp_posterior_cov.argtypes = [_c_p, _c_i64, _c_p, _c_p, _c_p, _c_d, _c_i, _c_p, _c_p,
                                   ctypes.POINTER(GpCgInfo)]
    L.gp_posterior_cov.restype = _c_i
    L.gp_plan_get_timing.argtypes = [_c_p, ctypes.POINTER(GpTiming)]
    L.gp_plan_get_timing.restype = _c_i
    L.gp_server_opts_init.argtypes = [ctypes.POINTER(GpServerOpts)]
    L.gp_server_opts_init.restype = _c_i
    L.gp_server_create.argtypes = [ctypes.POINTER(GpServerOpts), ctypes.POINTER(_c_p)]
    L.gp_server_create.restype = _c_i
    L.gp_server_submit.argtypes = [_c_p, _c_i, _c_i64, _c_p, _c_p, _c_p, _c_d, _c_d, _c_p, _c_p,
                                   _c_p, ctypes.POINTER(_c_i64)]
    L.gp_server_submit.restype = _c_i
    L.gp_server_wait.argtypes = [_c_p, _c_i64, ctypes.POINTER(GpRequestInfo)]
    L.gp_server_wait.restype = _c_i
    L.gp_server_poll.argtypes = [_c_p, _c_i64, ctypes.POINTER(_c_i)]
    L.gp_server_poll.restype = _c_i
    L.gp_server_stats.argtypes = [_c_p, ctypes.POINTER(GpServerCounters)]
    L.gp_server_stats.restype = _c_i
    L.gp_server_destroy.argtypes = [_c_p]
    L.gp_server_destroy.restype = _c_i
    _lib = L
    return L


class GpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpnufft error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != GP_OK:
        raise GpError(rc, load().gp_last_error().decode())


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    return t.contiguous()


def make_opts(precision: int = GP_FP64, stream=None, host_only: bool = False, **kw) -> GpOpts:
    o = GpOpts()
    _check(load().gp_opts_init(ctypes.byref(o)))
    o.precision = precision
    for k, v in kw.items():
        if v is None:
            continue
        if k in ("box_lo", "box_hi"):
            arr = getattr(o, k)
            for a, x in enumerate(v):
                arr[a] = float(x)
            o.use_box = 1
        else:
            setattr(o, k, v)
    if not host_only:
        s = stream if stream is not None else torch.cuda.current_stream()
        o.stream = ctypes.c_void_p(s.cuda_stream)
    return o


class Plan:
    """A resident plan for one point set (gp_plan)."""

    def __init__(self, x: torch.Tensor, sigma: torch.Tensor, l: torch.Tensor, nu: float,
                 eta: float, tol: float, precision: int = GP_FP64, stream=None, **opts):
        L = load()
        x = _dev(x, "x")
        if x.dim() == 1:
            x = x[:, None].contiguous()
        self.d = x.shape[1]
        self.n = x.shape[0]
        self.sigma = _dev(sigma, "sigma")
        self.l = _dev(l, "l")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        o = make_opts(precision, self.stream, **opts)
        h = _c_p()
        _check(L.gp_plan(self.d, self.n, x.data_ptr(), self.sigma.data_ptr(), self.l.data_ptr(),
                         float(nu), float(eta), float(tol), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.nu, self.eta, self.precision = nu, eta, precision

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        p = GpPlanParams()
        _check(load().gp_plan_info(self._h, ctypes.byref(p)))
        out = {}
        for name, _ in GpPlanParams._fields_:
            v = getattr(p, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out

    def matvec(self, alpha: torch.Tensor, add_noise: bool = False, out=None) -> torch.Tensor:
        alpha = _dev(alpha, "alpha")
        if out is None:
            out = torch.empty_like(alpha)
        _check(load().gp_matvec(self._h, alpha.data_ptr(), out.data_ptr(), int(add_noise)))
        return out

    def cg_solve(self, y: torch.Tensor, tol: float = 1e-6, max_iter: int = 10000, x0=None,
                 replace_every: int = 0):
        y = _dev(y, "y")
        alpha = torch.zeros_like(y) if x0 is None else _dev(x0, "x0").clone()
        info = GpCgInfo()
        rc = load().gp_cg_solve(self._h, y.data_ptr(), alpha.data_ptr(), int(x0 is not None),
                                float(tol), int(max_iter), int(replace_every), ctypes.byref(info))
        if rc not in (GP_OK, GP_ENOCONV):
            _check(rc)
        return alpha, _info_dict(info)

    def cg_solve_multi(self, Y: torch.Tensor, tol: float = 1e-6, max_iter: int = 10000,
                       block: bool = False):
        """gp_cg_solve_multi: Y is (m, n) (row j = right-hand side j); block
        selects block CG; returns (alpha (m, n), per-column iterations,
        per-column relative residuals, info)."""
        Y = _dev(Y, "Y")
        if Y.dim() == 1:
            Y = Y[None, :].contiguous()
        m = Y.shape[0]
        alpha = torch.zeros_like(Y)
        its = (ctypes.c_int * m)()
        rel = (ctypes.c_double * m)()
        info = GpCgInfo()
        rc = load().gp_cg_solve_multi(self._h, m, Y.data_ptr(), alpha.data_ptr(), float(tol),
                                      int(max_iter), int(block), its, rel, ctypes.byref(info))
        if rc not in (GP_OK, GP_ENOCONV):
            _check(rc)
        return alpha, list(its), list(rel), _info_dict(info)

    def cg_solve_noalloc(self, y: torch.Tensor, alpha: torch.Tensor, tol: float = 1e-6,
                         max_iter: int = 10000, use_x0: bool = False, replace_every: int = 0):
        """gp_cg_solve_noalloc: the solve into the caller's `alpha` (initial guess
        if use_x0), with no allocation in the library."""
        y = _dev(y, "y")
        if not (isinstance(alpha, torch.Tensor) and alpha.is_contiguous()):
            raise TypeError("alpha must be a contiguous float64 CUDA tensor")
        alpha = _dev(alpha, "alpha")
        info = GpCgInfo()
        rc = load().gp_cg_solve_noalloc(self._h, y.data_ptr(), alpha.data_ptr(), int(use_x0),
                                        float(tol), int(max_iter), int(replace_every),
                                        ctypes.byref(info))
        if rc not in (GP_OK, GP_ENOCONV):
            _check(rc)
        return alpha, _info_dict(info)

    def posterior_mean(self, alpha: torch.Tensor, targets: torch.Tensor, sigma_t: torch.Tensor,
                       l_t: torch.Tensor) -> torch.Tensor:
        alpha = _dev(alpha, "alpha")
        targets = _dev(targets, "targets")
        if targets.dim() == 1:
            targets = targets[:, None].contiguous()
        sigma_t = _dev(sigma_t, "sigma_t")
        l_t = _dev(l_t, "l_t")
        mu = torch.empty(targets.shape[0], dtype=torch.float64, device=alpha.device)
        _check(load().gp_posterior_mean(self._h, alpha.data_ptr(), targets.shape[0],
                                        targets.data_ptr(), sigma_t.data_ptr(), l_t.data_ptr(),
                                        mu.data_ptr()))
        return mu

    def posterior_cov(self, targets: torch.Tensor, sigma_t: torch.Tensor, l_t: torch.Tensor,
                      tol: float = 1e-8, max_iter: int = 10000, full: bool = True):
        """(cov m x m or None, var m, info) of eq:postcov at the targets."""
        targets = _dev(targets, "targets")
        if targets.dim() == 1:
            targets = targets[:, None].contiguous()
        sigma_t = _dev(sigma_t, "sigma_t")
        l_t = _dev(l_t, "l_t")
        m = targets.shape[0]
        var = torch.empty(m, dtype=torch.float64, device=targets.device)
        cov = torch.empty((m, m), dtype=torch.float64, device=targets.device) if full else None
        info = GpCgInfo()
        rc = load().gp_posterior_cov(self._h, m, targets.data_ptr(), sigma_t.data_ptr(),
                                     l_t.data_ptr(), float(tol), int(max_iter),
                                     cov.data_ptr() if full else None, var.data_ptr(),
                                     ctypes.byref(info))
        if rc not in (GP_OK, GP_ENOCONV):
            _check(rc)
        return cov, var, _info_dict(info)

    def residual(self, y: torch.Tensor, alpha: torch.Tensor) -> float:
        """||y - (K~ + eta^2 I) alpha|| / ||y|| with this plan's operator."""
        r = _c_d()
        _check(load().gp_residual(self._h, _dev(y, "y").data_ptr(), _dev(alpha, "alpha").data_ptr(),
                                  ctypes.byref(r)))
        return r.value

    def set_timing(self, enable: bool = True):
        _check(load().gp_plan_set_timing(self._h, int(enable)))

    def timing(self) -> dict:
        """{phase: (launches, total ms)} from the plan's HIP events."""
        t = GpTiming()
        _check(load().gp_plan_get_timing(self._h, ctypes.byref(t)))
        return {t.name[k].decode(): (t.launches[k], t.ms[k]) for k in range(t.n_phases)}

    def set_stream(self, stream):
        self.stream = stream
        _check(load().gp_plan_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().gp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _info_dict(info: GpCgInfo) -> dict:
    return {name: getattr(info, name) for name, _ in GpCgInfo._fields_}


def _params_dict(p: "GpPlanParams") -> dict:
    out = {}
    for name, _ in GpPlanParams._fields_:
        v = getattr(p, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def plan_rules(d: int, nu: float, tol: float, l_min: float, l_max: float, extent: float = 1.0,
               precision: int = GP_FP64, **opts) -> dict:
    """gp_plan_rules: the plan's numbers from the problem's ranges (host only)."""
    o = make_opts(precision, host_only=True, **opts)
    p = GpPlanParams()
    _check(load().gp_plan_rules(int(d), float(nu), float(tol), float(l_min), float(l_max),
                                float(extent), ctypes.byref(o), ctypes.byref(p)))
    return _params_dict(p)


def plan_query(x, sigma, l, nu, eta, tol, precision=GP_FP64, **opts) -> int:
    x = _dev(x, "x")
    if x.dim() == 1:
        x = x[:, None].contiguous()
    o = make_opts(precision, None, **opts)
    b = _c_sz()
    _check(load().gp_plan_query(x.shape[1], x.shape[0], x.data_ptr(), _dev(sigma, "sigma").data_ptr(),
                                _dev(l, "l").data_ptr(), float(nu), float(eta), float(tol),
                                ctypes.byref(o), ctypes.byref(b)))
    return b.value


def cg_solve_refined(inner: Plan, outer: Plan, y: torch.Tensor, tol: float = 1e-6,
                     inner_tol: float = 1e-3, max_iter: int = 100000, max_refine: int = 20,
                     replace_every: int = 0):
    y = _dev(y, "y")
    alpha = torch.zeros_like(y)
    info = GpCgInfo()
    rc = load().gp_cg_solve_refined(inner.handle, outer.handle, y.data_ptr(), alpha.data_ptr(),
                                    float(tol), float(inner_tol), int(max_iter), int(max_refine),
                                    int(replace_every), ctypes.byref(info))
    if rc not in (GP_OK, GP_ENOCONV):
        _check(rc)
    return alpha, _info_dict(info)


class Server:
    """Continuous-batching solve server (gp_server_*).  Submitted tensors are
    kept alive here until their request has been waited for."""

    def __init__(self, max_slots: int = 4, max_device_bytes: int = 64 << 30,
                 precision: int = GP_FP32_BULK, **kw):
        L = load()
        o = GpServerOpts()
        _check(L.gp_server_opts_init(ctypes.byref(o)))
        o.max_slots = max_slots
        o.max_device_bytes = max_device_bytes
        o.precision = precision
        for k, v in kw.items():
            setattr(o, k, v)
        h = _c_p()
        _check(L.gp_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, x, sigma, l, nu, eta, y, stream=None) -> int:
        """Queue a solve.  `stream` is the torch stream the inputs were made on
        (default: the current stream); the server orders its reads after it."""
        x = _dev(x, "x")
        if x.dim() == 1:
            x = x[:, None].contiguous()
        sigma, l, y = _dev(sigma, "sigma"), _dev(l, "l"), _dev(y, "y")
        alpha = torch.empty_like(y)
        s = stream if stream is not None else torch.cuda.current_stream()
        rid = _c_i64()
        _check(load().gp_server_submit(self._h, x.shape[1], x.shape[0], x.data_ptr(),
                                       sigma.data_ptr(), l.data_ptr(), float(nu), float(eta),
                                       y.data_ptr(), alpha.data_ptr(),
                                       ctypes.c_void_p(s.cuda_stream), ctypes.byref(rid)))
        self._live[rid.value] = (x, sigma, l, y, alpha)
        return rid.value

    def wait(self, rid: int):
        info = GpRequestInfo()
        rc = load().gp_server_wait(self._h, rid, ctypes.byref(info))
        if rc not in (GP_OK, GP_ENOCONV):
            _check(rc)
        alpha = self._live.pop(rid)[4]
        return alpha, {name: getattr(info, name) for name, _ in GpRequestInfo._fields_}

    def poll(self, rid: int) -> bool:
        d = _c_i()
        _check(load().gp_server_poll(self._h, rid, ctypes.byref(d)))
        return bool(d.value)

    def stats(self) -> dict:
        c = GpServerCounters()
        _check(load().gp_server_stats(self._h, ctypes.byref(c)))
        return {name: getattr(c, name) for name, _ in GpServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().gp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
