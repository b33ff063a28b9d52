"""Plain CPU oracle (fp64) for the non-stationary Matern GPR path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
``cpu_baseline`` leg are the only permitted users.  The product library never
imports, links or calls anything here, and this package imports nothing from
the product.

Most of the arithmetic lives in ``oracle.cpp`` (compiled into ``liboracle.so``
by ``build()`` below, with g++ and OpenMP); see its header for the formulas
(Kielstra & Lindsey, arXiv 2407.03608).  This module marshals numpy arrays to
it and adds two plain numpy steps: the Schur complement of eq:postcov
(``_schur``: one oracle Cholesky, one triangular solve per target column and a
matrix product) and the assembly of the dense blocks it takes.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_int = ctypes.c_int
_p = ctypes.c_void_p


class OrcPlan(ctypes.Structure):
    _fields_ = [
        ("d", _int),
        ("nu", _d),
        ("t_min", _d),
        ("t_max", _d),
        ("n_t", _int),
        ("s_min", _d),
        ("s_max", _d),
        ("n_sigma", _int),
        ("dw", _d),
        ("M", _i64),
        ("center", _d * 3),
        ("scale", _d),
    ]


@dataclass
class Params:
    """The numbers that define the approximate operator K~ (section 3.5)."""

    d: int
    nu: float
    t_min: float
    t_max: float
    n_t: int
    s_min: float
    s_max: float
    n_sigma: int
    dw: float
    M: int
    center: tuple = (0.0, 0.0, 0.0)
    scale: float = 1.0

    def c(self) -> OrcPlan:
        p = OrcPlan()
        p.d, p.nu = self.d, self.nu
        p.t_min, p.t_max, p.n_t = self.t_min, self.t_max, self.n_t
        p.s_min, p.s_max, p.n_sigma = self.s_min, self.s_max, self.n_sigma
        p.dw, p.M = self.dw, int(self.M)
        c = list(self.center) + [0.0] * (3 - len(self.center))
        for a in range(3):
            p.center[a] = c[a]
        p.scale = self.scale
        return p


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", tmp, src]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_matern.restype = _d
        L.orc_matern.argtypes = [_d, _d]
        L.orc_matern_bessel.restype = _d
        L.orc_matern_bessel.argtypes = [_d, _d]
        L.orc_matern_schoenberg.restype = _d
        L.orc_matern_schoenberg.argtypes = [_d, _d, _d, _d, _int]
        L.orc_kernel_block.restype = None
        L.orc_kernel_block.argtypes = [_int, _i64, _p, _p, _p, _i64, _p, _p, _p, _d, _p]
        L.orc_exact_matvec_rows.restype = None
        L.orc_exact_matvec_rows.argtypes = [_int, _i64, _p, _p, _p, _d, _p, _i64, _i64, _p]
        L.orc_cholesky.restype = _int
        L.orc_cholesky.argtypes = [_i64, _p]
        L.orc_chol_solve.restype = None
        L.orc_chol_solve.argtypes = [_i64, _p, _p, _p]
        L.orc_tgrid.restype = None
        L.orc_tgrid.argtypes = [ctypes.POINTER(OrcPlan), _p, _p, _p]
        L.orc_sigma_nodes.restype = None
        L.orc_sigma_nodes.argtypes = [ctypes.POINTER(OrcPlan), _p]
        L.orc_lagrange.restype = None
        L.orc_lagrange.argtypes = [_int, _p, _d, _p]
        L.orc_weights.restype = None
        L.orc_weights.argtypes = [ctypes.POINTER(OrcPlan), _i64, _p, _p, _p]
        L.orc_ktilde_matvec.restype = _int
        L.orc_ktilde_matvec.argtypes = [ctypes.POINTER(OrcPlan), _i64, _p, _p, _p, _p, _p]
        L.orc_ktilde_entries.restype = _int
        L.orc_ktilde_entries.argtypes = [ctypes.POINTER(OrcPlan), _i64, _p, _p, _p, _i64, _p, _p, _p, _p]
        L.orc_posterior_mean.restype = None
        L.orc_posterior_mean.argtypes = [_int, _i64, _p, _p, _p, _d, _p, _i64, _p, _p, _p, _p]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_p)


# ------------------------------------------------------------------ phi_nu --

def matern(nu: float, r) -> np.ndarray:
    r = np.atleast_1d(_f64(r))
    return np.array([lib().orc_matern(nu, float(v)) for v in r])


def matern_bessel(nu: float, r) -> np.ndarray:
    r = np.atleast_1d(_f64(r))
    return np.array([lib().orc_matern_bessel(nu, float(v)) for v in r])


def matern_schoenberg(nu: float, r, tmin: float, tmax: float, nt: int) -> np.ndarray:
    r = np.atleast_1d(_f64(r))
    return np.array([lib().orc_matern_schoenberg(nu, float(v), tmin, tmax, nt) for v in r])


# ---------------------------------------------------------------- exact O1 --

def kernel_matrix(x, sig, l, nu, y=None, sig_y=None, l_y=None) -> np.ndarray:
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    d = x.shape[1]
    if y is None:
        y, sig_y, l_y = x, sig, l
    y = _f64(y)
    if y.ndim == 1:
        y = y[:, None]
    sig, l, sig_y, l_y = _f64(sig), _f64(l), _f64(sig_y), _f64(l_y)
    K = np.empty((x.shape[0], y.shape[0]))
    lib().orc_kernel_block(d, x.shape[0], _ptr(x), _ptr(sig), _ptr(l), y.shape[0], _ptr(y),
                           _ptr(sig_y), _ptr(l_y), nu, _ptr(K))
    return K


def exact_matvec(x, sig, l, nu, alpha, rows=None) -> np.ndarray:
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    n, d = x.shape
    sig, l, alpha = _f64(sig), _f64(l), _f64(alpha)
    r0, r1 = (0, n) if rows is None else rows
    out = np.empty(r1 - r0)
    lib().orc_exact_matvec_rows(d, n, _ptr(x), _ptr(sig), _ptr(l), nu, _ptr(alpha), r0, r1, _ptr(out))
    return out


def cholesky(A) -> np.ndarray:
    L = np.array(A, dtype=np.float64, copy=True, order="C")
    rc = lib().orc_cholesky(L.shape[0], _ptr(L))
    if rc != 0:
        raise np.linalg.LinAlgError(f"oracle Cholesky: non-positive pivot at column {-rc - 1}")
    return np.tril(L)


def chol_solve(L, b) -> np.ndarray:
    L = _f64(L)
    b = _f64(b)
    x = np.empty_like(b)
    lib().orc_chol_solve(L.shape[0], _ptr(L), _ptr(b), _ptr(x))
    return x


def gpr_solve_exact(x, sig, l, nu, eta, y, lapack: bool = False) -> np.ndarray:
    """alpha = (K + eta^2 I)^{-1} y (eq:gprsolve) with the exact kernel matrix.
    The factorisation is the oracle's own Cholesky, or LAPACK's (numpy, a
    library primitive pinned against the oracle's in the tests) for sizes where
    the plain loop would take minutes."""
    K = kernel_matrix(x, sig, l, nu)
    K[np.diag_indices_from(K)] += eta * eta
    if lapack:
        import scipy.linalg
        return scipy.linalg.cho_solve(scipy.linalg.cho_factor(K, lower=True), _f64(y))
    return chol_solve(cholesky(K), y)


def posterior_mean_exact(x, sig, l, nu, alpha, xt, sig_t, l_t) -> np.ndarray:
    x, xt = _f64(x), _f64(xt)
    if x.ndim == 1:
        x = x[:, None]
    if xt.ndim == 1:
        xt = xt[:, None]
    n, d = x.shape
    m = xt.shape[0]
    sig, l, alpha, sig_t, l_t = map(_f64, (sig, l, alpha, sig_t, l_t))
    mu = np.empty(m)
    lib().orc_posterior_mean(d, n, _ptr(x), _ptr(sig), _ptr(l), nu, _ptr(alpha), m, _ptr(xt),
                             _ptr(sig_t), _ptr(l_t), _ptr(mu))
    return mu


def _schur(Kxx, Kxs, Kss, eta) -> np.ndarray:
    """Kss - Kxs^T (Kxx + eta^2 I)^{-1} Kxs, one oracle Cholesky solve per column."""
    A = np.array(Kxx, dtype=np.float64, copy=True)
    A[np.diag_indices_from(A)] += eta * eta
    L = cholesky(A)
    V = np.stack([chol_solve(L, np.ascontiguousarray(Kxs[:, j])) for j in range(Kxs.shape[1])], axis=1)
    return np.asarray(Kss) - np.asarray(Kxs).T @ V


def posterior_cov_exact(x, sig, l, nu, eta, xt, sig_t, l_t) -> np.ndarray:
    """Posterior covariance eq:postcov at the targets with the exact kernel:
    K(X*,X*) - K(X*,X) (K + eta^2 I)^{-1} K(X,X*)."""
    Kxx = kernel_matrix(x, sig, l, nu)
    Kxs = kernel_matrix(x, sig, l, nu, xt, sig_t, l_t)
    Kss = kernel_matrix(xt, sig_t, l_t, nu)
    return _schur(Kxx, Kxs, Kss, eta)


# ------------------------------------------------------------ K-tilde O2 ----

def tgrid(p: Params):
    n = 1 if math.isinf(p.nu) else p.n_t + 1
    t, vt, chi = np.empty(n), np.empty(n), np.empty(n)
    c = p.c()
    lib().orc_tgrid(ctypes.byref(c), _ptr(t), _ptr(vt), _ptr(chi))
    return t, vt, chi


def sigma_nodes(p: Params) -> np.ndarray:
    s = np.empty(p.n_sigma + 1)
    c = p.c()
    lib().orc_sigma_nodes(ctypes.byref(c), _ptr(s))
    return s


def lagrange(nodes, s: float) -> np.ndarray:
    nodes = _f64(nodes)
    P = np.empty(nodes.shape[0])
    lib().orc_lagrange(nodes.shape[0] - 1, _ptr(nodes), float(s), _ptr(P))
    return P


def weights(p: Params, sig, l) -> np.ndarray:
    sig, l = _f64(sig), _f64(l)
    wk = np.empty((sig.shape[0], p.n_sigma + 1))
    c = p.c()
    lib().orc_weights(ctypes.byref(c), sig.shape[0], _ptr(sig), _ptr(l), _ptr(wk))
    return wk


def ktilde_matvec(p: Params, x, sig, l, alpha) -> np.ndarray:
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    sig, l, alpha = _f64(sig), _f64(l), _f64(alpha)
    out = np.empty(x.shape[0])
    c = p.c()
    rc = lib().orc_ktilde_matvec(ctypes.byref(c), x.shape[0], _ptr(x), _ptr(sig), _ptr(l),
                                 _ptr(alpha), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_ktilde_matvec failed: {rc}")
    return out


def ktilde_entries(p: Params, x, sig, l, y=None, sig_y=None, l_y=None) -> np.ndarray:
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    if y is None:
        y, sig_y, l_y = x, sig, l
    y = _f64(y)
    if y.ndim == 1:
        y = y[:, None]
    sig, l, sig_y, l_y = map(_f64, (sig, l, sig_y, l_y))
    K = np.empty((x.shape[0], y.shape[0]))
    c = p.c()
    rc = lib().orc_ktilde_entries(ctypes.byref(c), x.shape[0], _ptr(x), _ptr(sig), _ptr(l),
                                  y.shape[0], _ptr(y), _ptr(sig_y), _ptr(l_y), _ptr(K))
    if rc:
        raise RuntimeError(f"orc_ktilde_entries failed: {rc}")
    return K


def ktilde_posterior_cov(p: Params, x, sig, l, eta, xt, sig_t, l_t) -> np.ndarray:
    """eq:postcov with the approximate operator K~ in every term (entries by the
    theta-sum form)."""
    Kxx = ktilde_entries(p, x, sig, l)
    Kxs = ktilde_entries(p, x, sig, l, xt, sig_t, l_t)
    Kss = ktilde_entries(p, xt, sig_t, l_t)
    return _schur(Kxx, Kxs, Kss, eta)

