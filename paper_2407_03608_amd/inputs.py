"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method: it only draws points, the two
scale functions sigma(x) (vertical) and l(x) (length) and observations y.
Every generator uses numpy's PCG64 ``default_rng(seed)``; points are drawn
first, then noise.  Arrays are fp64, points are row-major ``(N, d)``.

Workloads
---------
* ``matern_1d``   d=1, N=2000, nu=3/2, sigma=1+0.5 sin 2 pi x, l=0.05+0.03 cos 2 pi x,
                  eta=0.1, y = sin(10 x) + N(0, eta^2)                   (seed 1)
* ``matern_2d``   d=2, N=1e6 on [0,1]^2, nu=1/2, sigma=exp(0.3 x1),
                  l=0.02+0.02 x2, eta=0.05, y = sin(8 x1) cos(6 x2) + N(0, eta^2)  (seed 2)
* ``matern_3d``   d=3, N=1e7 from an 8-component Gaussian mixture (std 0.1,
                  centres U[0.2,0.8]^3, equal weights) clipped to [0,1]^3,
                  nu=5/2, sigma=1, l=0.03+0.02 |x-0.5|, eta=0.1          (seed 4)
* ``paper_setup`` the paper's own experiment inputs (section 6): points
                  uniform on [-1,1]^d, w(x)=1 and the width
                  sigma_p(x) = (prod_i cos(pi x_i) + 2)/6, expressed in the
                  (sigma, l) parameterisation used by the library
* ``serving``     a stream of independent GPR solve requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    d: int
    x: np.ndarray          # (N, d) points
    sigma: np.ndarray      # (N,) vertical scale
    l: np.ndarray          # (N,) length scale
    nu: float              # Matern smoothness (math.inf = squared exponential)
    eta: float             # noise standard deviation
    y: np.ndarray          # (N,) observations
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]


def matern_1d(n: int = 2000, seed: int = 1) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 1))
    eta = 0.1
    noise = rng.normal(0.0, eta, size=n)
    t = x[:, 0]
    sigma = 1.0 + 0.5 * np.sin(2 * np.pi * t)
    l = 0.05 + 0.03 * np.cos(2 * np.pi * t)
    y = np.sin(10.0 * t) + noise
    return Problem("matern_1d", 1, x, sigma, l, 1.5, eta, y)


def matern_2d(n: int = 1_000_000, seed: int = 2) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 2))
    eta = 0.05
    noise = rng.normal(0.0, eta, size=n)
    sigma = np.exp(0.3 * x[:, 0])
    l = 0.02 + 0.02 * x[:, 1]
    y = np.sin(8.0 * x[:, 0]) * np.cos(6.0 * x[:, 1]) + noise
    return Problem("matern_2d", 2, x, sigma, l, 0.5, eta, y)


def matern_3d(n: int = 10_000_000, seed: int = 4) -> Problem:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(8, 3))
    comp = rng.integers(0, 8, size=n)
    x = centres[comp] + rng.normal(0.0, 0.1, size=(n, 3))
    np.clip(x, 0.0, 1.0, out=x)
    eta = 0.1
    noise = rng.normal(0.0, eta, size=n)
    sigma = np.ones(n)
    l = 0.03 + 0.02 * np.linalg.norm(x - 0.5, axis=1)
    y = np.sin(4.0 * x[:, 0]) * np.cos(3.0 * x[:, 1]) + 0.5 * np.sin(5.0 * x[:, 2]) + noise
    return Problem("matern_3d", 3, x, sigma, l, 2.5, eta, y)


def subsample(p: Problem, m: int, seed: int = 0) -> Problem:
    """The first m points of a problem (the generators draw points iid)."""
    return Problem(p.name + f"_sub{m}", p.d, p.x[:m].copy(), p.sigma[:m].copy(), p.l[:m].copy(),
                   p.nu, p.eta, p.y[:m].copy(), dict(p.meta))


def paper_setup(d: int, n: int, nu: float = 1.5, seed: int = 7, eta: float = 0.1) -> Problem:
    """Points uniform on [-1,1]^d with the paper's reference width function and
    unit weight, translated to (sigma, l): l = sqrt(2) sigma_p and
    sigma = (sqrt(2 pi) l)^(-d/2) so that w(x) = 1."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, d))
    y = rng.uniform(0.0, 1.0, size=n)
    sp = (np.prod(np.cos(np.pi * x), axis=1) + 2.0) / 6.0
    l = math.sqrt(2.0) * sp
    sigma = (math.sqrt(2.0 * math.pi) * l) ** (-0.5 * d)
    return Problem(f"paper_d{d}", d, x, sigma, l, nu, eta, y, {"sigma_p": sp})


def random_small(d: int, n: int, seed: int, nu: float = 1.5, lmin: float = 0.1,
                 lmax: float = 0.25, eta: float = 0.1, constant_scales: bool = False) -> Problem:
    """Small random non-stationary problem on [0,1]^d for parity tests."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, d))
    y = rng.standard_normal(n)
    if constant_scales:
        sigma = np.full(n, 1.3)
        l = np.full(n, 0.5 * (lmin + lmax))
    else:
        ph = rng.uniform(0, 2 * np.pi, size=d)
        s = np.mean(np.sin(2 * np.pi * x + ph), axis=1)
        c = np.mean(np.cos(2 * np.pi * x + ph), axis=1)
        sigma = 1.0 + 0.4 * s
        l = lmin + (lmax - lmin) * 0.5 * (1.0 + c)
    return Problem(f"small_d{d}_n{n}_s{seed}", d, x, sigma, l, nu, eta, y)


# ------------------------------------------------------------------ serving --

def _fourier_series(rng, t: np.ndarray) -> np.ndarray:
    """A random smooth periodic function of 4 terms, scaled so max|s| <= 1."""
    a = rng.normal(size=4)
    b = rng.normal(size=4)
    m = np.arange(1, 5)
    grid = np.linspace(0.0, 1.0, 513)
    def ev(u):
        u = np.asarray(u)[..., None]
        return np.sum((a * np.cos(2 * np.pi * m * u) + b * np.sin(2 * np.pi * m * u)) / m, axis=-1)
    scale = max(1e-12, np.abs(ev(grid)).max())
    return ev(t) / scale


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    problem: Problem


def serving_stream(n_requests: int = 512, rate: float = 50.0, seed: int = 5,
                   n_min: int = 1000, n_max: int = 500_000) -> list:
    """GPR solve requests with Poisson arrivals: d in {1,2}, N log-uniform in
    [n_min, n_max], nu in {1/2, 3/2, 5/2}, eta ~ U[0.01, 0.2], sigma and l from
    random 4-term Fourier series (sigma = exp(0.3 s), l = l0 exp(0.3 s') with
    l0 log-uniform in [0.02, 0.2]); y a random 4-term series plus noise."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        d = int(rng.integers(1, 3))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        eta = float(rng.uniform(0.01, 0.2))
        x = rng.uniform(0.0, 1.0, size=(n, d))
        def field_(xx):
            return np.mean([_fourier_series(rng, xx[:, a]) for a in range(d)], axis=0)
        s_sig = field_(x)
        s_l = field_(x)
        l0 = math.exp(rng.uniform(math.log(0.02), math.log(0.2)))
        sigma = np.exp(0.3 * s_sig)
        l = l0 * np.exp(0.3 * s_l)
        y = field_(x) + rng.normal(0.0, eta, size=n)
        out.append(Request(rid, t, Problem(f"req{rid}", d, x, sigma, l, nu, eta, y)))
    return out
