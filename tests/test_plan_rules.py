"""Host logic of the plan (gp_plan_rules, no GPU): every discretisation number
is checked against what it has to guarantee, computed independently of the
library (oracle quadrature and interpolation, scipy distributions).

Readings (section 3 of the paper sizes the discretisation only up to
constants): N_sigma is the smallest degree (rounded up to odd) whose Chebyshev
interpolation of sigma -> exp(-x^2 / 2 sigma^2) meets eps/10 (lemma
lem:interp); the t grid reproduces phi_nu (lemma lem:dt); Delta-omega puts the
periodic images (eq:PSF) where phi_nu <= eps/10; M is the smallest half-width
whose spectral tail of the narrowest kernel is <= eps.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as O
from paper_2407_03608_amd import gp

CASES = [
    # d, nu, tol, l_min, l_max, extent, precision
    (2, 0.5, 1e-8, 0.02, 0.04, 1.0, 0),     # the d=2 N=1e6 workload (M capped)
    (2, 0.5, 1e-4, 0.02, 0.04, 1.0, 1),     # its fp32-bulk operator
    (1, 1.5, 1e-8, 0.02, 0.08, 1.0, 0),     # the d=1 workload
    (3, 2.5, 1e-4, 0.03, 0.047, 1.0, 1),    # the d=3 workload
    (2, 1.5, 1e-6, 0.05, 0.2, 2.0, 0),
    (1, 2.5, 1e-10, 0.1, 0.15, 1.0, 0),
    (2, math.inf, 1e-8, 0.1, 0.3, 1.0, 0),  # squared exponential
    (1, 0.5, 1e-6, 0.1, 0.1, 1.0, 0),       # stationary scales
]
IDS = [f"d{c[0]}-nu{c[1]}-tol{c[2]:g}-p{c[6]}" for c in CASES]


@pytest.fixture(scope="module", autouse=True)
def lib():
    gp.load()
    O.build()


def _rules(case, **opts):
    d, nu, tol, lmin, lmax, ext, prec = case
    return gp.plan_rules(d, nu, tol, lmin, lmax, ext, precision=prec, **opts)


def _interp_error(p, n_sigma, smin, smax):
    """Sup error of interpolating sigma -> exp(-x^2/(2 sigma^2)) at the
    Chebyshev-Lobatto nodes of degree n_sigma (oracle nodes, product-form
    Lagrange basis), sampled off the nodes."""
    q = O.Params(d=1, nu=1.5, t_min=0.0, t_max=1.0, n_t=1, s_min=smin, s_max=smax,
                 n_sigma=n_sigma, dw=0.1, M=4)
    nodes = O.sigma_nodes(q)
    worst = 0.0
    xs = np.linspace(0.0, 6.0 * smax, 131)
    for s in smin + (smax - smin) * (np.arange(89) + 0.37) / 89:
        L = O.lagrange(nodes, s)
        approx = np.exp(-xs[:, None] ** 2 / (2 * nodes[None, :] ** 2)) @ L
        worst = max(worst, float(np.abs(approx - np.exp(-xs ** 2 / (2 * s * s))).max()))
    return worst


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_n_sigma_meets_the_interpolation_target_and_is_minimal(case):
    p = _rules(case)
    tol = case[2]
    if case[3] == case[4]:
        assert p["n_sigma"] == 0
        return
    ns = p["n_sigma"]
    assert ns % 2 == 1, "N_sigma + 1 grids pack into complex pairs"
    assert p["n_pairs"] == (ns + 2) // 2
    e = _interp_error(p, ns, p["s_min"], p["s_max"])
    assert e <= 2 * tol / 10, e
    if ns >= 3:
        assert _interp_error(p, ns - 2, p["s_min"], p["s_max"]) > 0.5 * tol / 10


@pytest.mark.parametrize("case", [c for c in CASES if not math.isinf(c[1])],
                         ids=[i for c, i in zip(CASES, IDS) if not math.isinf(c[1])])
def test_t_grid_reproduces_the_matern_correlation(case):
    p = _rules(case)
    nu, tol = case[1], case[2]
    r = np.linspace(0.0, 12.0, 241)
    approx = O.matern_schoenberg(nu, r, p["t_min"], p["t_max"], p["n_t"])
    err = float(np.abs(approx - O.matern(nu, r)).max())
    assert err <= tol, err


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_delta_omega_puts_the_periodic_images_in_the_kernel_tail(case):
    p = _rules(case)
    d, nu, tol, lmin, lmax, ext, prec = case
    lpmax = lmax * 2.0 / ext
    r = (1.0 / p["dw"] - 2.0) / lpmax
    assert 0 < p["dw"] < 0.5
    assert float(O.matern(nu, np.array([r]))[0]) <= tol / 10 * (1 + 1e-6)


def _tail(nu, d, ell, omega):
    """Spectral mass of the stationary kernel outside radius omega: the Matern
    density (1 + (2 pi ell w)^2/(2 nu))^-(nu+d/2) is a multivariate t with
    2 nu degrees of freedom in t = 2 pi ell w (|t|^2/d ~ F(d, 2 nu)); the
    squared exponential's is Gaussian (|t|^2 ~ chi^2_d)."""
    t2 = (2 * math.pi * ell * omega) ** 2
    if math.isinf(nu):
        return float(scipy.stats.chi2.sf(t2, d))
    return float(scipy.stats.f.sf(t2 / d, d, 2 * nu))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_m_is_the_smallest_half_width_meeting_the_spectral_tail(case):
    p = _rules(case)
    d, nu, tol, lmin, lmax, ext, prec = case
    lpmin = lmin * 2.0 / ext
    M, dw = p["M"], p["dw"]
    tail = _tail(nu, d, lpmin, M * dw)
    assert p["pred_tail"] == pytest.approx(tail, rel=1e-9, abs=1e-300)
    if p["m_capped"]:
        assert M == (2047 if d > 1 else 1 << 18) and tail > tol
    else:
        assert tail <= tol * 1.01
        if M > 4:
            assert _tail(nu, d, lpmin, (M - 1) * dw) > tol * 0.99


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_window_grid_and_active_box(case):
    p = _rules(case)
    d, prec = case[0], case[6]
    ntol = p["nufft_tol"]
    if prec == 1:
        assert ntol >= 1e-6
    # automatic oversampling: 1.25 asked in 2-D, 2 otherwise; the window is
    # sized for the oversampling reached
    nf, mc, s = p["nf"][0], 2 * p["M"] + 1, p["upsample"]
    assert nf >= (1.25 if d == 2 else 2.0) * mc
    assert s == pytest.approx(min(2.0, nf / mc))
    if s >= 2:
        assert p["w"] == min(16, max(2, math.ceil(math.log10(1 / ntol)) + 1))
        assert p["beta"] == pytest.approx(2.30 * p["w"])
    else:
        w = min(16, max(2, math.ceil(math.log(10 / ntol) / (math.pi * math.sqrt(1 - 1 / s)))))
        assert p["w"] == w
        assert p["beta"] == pytest.approx(0.97 * math.pi * (1 - 0.5 / s) * w)
    m = nf
    while m % 2 == 0:
        m //= 2
    while m % 3 == 0:
        m //= 3
    assert m == 1, "FFT lengths are 2^a 3^b"
    for r in range(d):
        assert p["nf"][r] == nf
        lo, na, tile = p["lo"][r], p["na"][r], p["tile"][r]
        assert na % tile == 0 and 0 <= lo and lo + na <= nf
        # every window of a point in [-1, 1] starts and ends inside the box
        assert lo <= 0.5 * nf - nf * p["dw"] - 0.5 * p["w"]
        assert lo + na >= 0.5 * nf + nf * p["dw"] + 0.5 * p["w"]


# Small grids of length 3*2^a (192, 96): a whole number of default tiles
# (256 cells in 1-D) does not fit in the grid, so the tile is halved until one
# does; the box must still hold every window.  These plans once got a box cut
# to a power of two (128 of 192 cells) and failed at build time.
@pytest.mark.parametrize("d,nu,tol,lmin,lmax,ups", [
    (1, math.inf, 1e-4, 0.02, 0.04, 0.0),
    (1, 2.5, 1e-4, 0.1, 0.1, 1.25),
    (1, math.inf, 1e-6, 0.1, 0.1, 1.25),
    (2, math.inf, 1e-4, 0.1, 0.1, 2.0),
])
def test_small_grid_active_box_holds_every_window(d, nu, tol, lmin, lmax, ups):
    p = gp.plan_rules(d, nu, tol, lmin, lmax, 1.0, upsample=ups)
    for r in range(d):
        nf, lo, na, tile = p["nf"][r], p["lo"][r], p["na"][r], p["tile"][r]
        assert tile & (tile - 1) == 0 and na % tile == 0 and 0 <= lo and lo + na <= nf
        first = math.ceil(0.5 * nf - nf * p["dw"] - 0.5 * p["w"])
        last = math.ceil(0.5 * nf + nf * p["dw"] - 0.5 * p["w"]) + p["w"]
        assert lo <= first and last <= lo + na, (nf, lo, na, tile, p["w"])


@pytest.mark.parametrize("case", CASES[:4], ids=IDS[:4])
@pytest.mark.parametrize("ups", [1.25, 1.5])
def test_upsampled_grid_and_window_rule(case, ups):
    """Oversampling below 2: n_f is the smallest supported length >= ups (2M+1),
    and the window is sized for the oversampling reached, s = min(2, n_f/(2M+1)),
    by the exponential-of-semicircle rule w = ceil(ln(10/eps) / (pi sqrt(1 - 1/s))),
    beta = 0.97 pi (1 - 1/(2s)) w."""
    d = case[0]
    p = _rules(case, upsample=ups)
    base = _rules(case)
    mc = 2 * p["M"] + 1
    nf = p["nf"][0]
    assert nf >= ups * mc and nf <= base["nf"][0]
    s = min(2.0, nf / mc)
    assert p["upsample"] == pytest.approx(s)
    if s < 2:
        w = min(16, max(2, math.ceil(math.log(10 / p["nufft_tol"]) / (math.pi * math.sqrt(1 - 1 / s)))))
        assert p["w"] == w
        assert p["beta"] == pytest.approx(0.97 * math.pi * (1 - 0.5 / s) * w)
    assert p["w"] >= base["w"]
    if d > 1:
        # the grid length is one of the FFT's single-pass lengths
        assert nf in [k << j for k in (1, 3) for j in range(3, 14) if (k << j) <= 8192]


def _es_type2_error(M, nf, w, beta, seed=0, npts=1500):
    """Relative 2-norm error of a 1-D type-2 NUFFT f(theta) = sum_{|k|<=M} c_k
    e^{i k theta} done the usual way with the exponential-of-semicircle window
    psi(z) = exp(beta (sqrt(1 - z^2) - 1)) of w cells on nf cells (deconvolve by
    the window's Fourier transform, inverse FFT, interpolate), against the
    direct sum.  Uses only (M, nf, w, beta)."""
    rng = np.random.default_rng(seed)
    k = np.arange(-M, M + 1)
    c = rng.standard_normal(k.size) + 1j * rng.standard_normal(k.size)
    h = 2 * np.pi / nf
    z, gw = np.polynomial.legendre.leggauss(400)
    psi = np.exp(beta * (np.sqrt(1 - z * z) - 1))
    # psi_hat(k) = (1/h) int psi(2u/(w h)) e^{-iku} du
    ph = 0.5 * w * (np.cos(np.outer(k, 0.5 * w * h * z)) @ (gw * psi))
    arr = np.zeros(nf, complex)
    arr[k % nf] = c / ph * (-1.0) ** k      # grid cell l sits at theta_l = l h - pi
    G = nf * np.fft.ifft(arr)
    theta = rng.uniform(-np.pi, np.pi, npts)
    s = np.ceil((theta + np.pi) / h - 0.5 * w).astype(int)
    f = np.zeros(npts, complex)
    for q in range(w):
        cell = s + q
        u = (cell * h - np.pi - theta) / (0.5 * w * h)
        wt = np.where(np.abs(u) <= 1, np.exp(beta * (np.sqrt(np.clip(1 - u * u, 0, None)) - 1)), 0.0)
        f += wt * G[cell % nf]
    ex = np.exp(1j * np.outer(theta, k)) @ c
    return float(np.linalg.norm(f - ex) / np.linalg.norm(ex))


@pytest.mark.parametrize("tol", [1e-4, 1e-8, 1e-11])
@pytest.mark.parametrize("ups,M", [(2.0, 700), (1.5, 1000), (1.25, 700)])
def test_window_rule_reaches_the_nufft_tolerance(tol, ups, M):
    """The (w, beta, n_f) the plan picks give a type-2 NUFFT as accurate as
    asked, checked by an independent numpy NUFFT against the direct sum; a
    window two cells narrower misses it."""
    p = gp.plan_rules(1, 1.5, 1e-6, 0.01, 0.02, M=M, nufft_tol=tol, upsample=ups)
    if ups < 2:
        assert p["upsample"] < 2
    e = _es_type2_error(p["M"], p["nf"][0], p["w"], p["beta"])
    assert e <= tol, (e, p["w"], p["nf"][0])
    w2 = p["w"] - 2
    assert _es_type2_error(p["M"], p["nf"][0], w2, p["beta"] * w2 / p["w"]) > tol


@pytest.mark.parametrize("ups", [1.0, 1.2, 2.5])
def test_upsample_outside_its_range_is_rejected(ups):
    with pytest.raises(gp.GpError) as e:
        gp.plan_rules(2, 1.5, 1e-6, 0.1, 0.2, upsample=ups)
    assert e.value.code == gp.GP_EINVAL


def test_rules_are_invariant_under_a_joint_scaling_of_box_and_lengths():
    """K depends on x and l only through (x - y)/l, so scaling the box and the
    length scales together must not change any discretisation number."""
    a = gp.plan_rules(2, 1.5, 1e-7, 0.03, 0.09, 1.0)
    b = gp.plan_rules(2, 1.5, 1e-7, 0.03 * 7.5, 0.09 * 7.5, 7.5)
    for k in ("n_sigma", "n_t", "M", "nf", "na", "w", "m_capped"):
        assert a[k] == b[k], k
    for k in ("dw", "t_min", "t_max", "s_min", "s_max", "pred_tail"):
        assert a[k] == pytest.approx(b[k], rel=1e-12), k


def test_fp32_plan_shares_dw_and_m_when_given():
    a = gp.plan_rules(2, 0.5, 1e-8, 0.02, 0.04)
    b = gp.plan_rules(2, 0.5, 1e-4, 0.02, 0.04, precision=gp.GP_FP32_BULK, dw=a["dw"], M=a["M"])
    assert b["dw"] == a["dw"] and b["M"] == a["M"] and b["nf"] == a["nf"]
    assert b["w"] < a["w"] and b["n_sigma"] < a["n_sigma"] and b["n_t"] < a["n_t"]


def test_overrides_are_taken_as_given():
    p = gp.plan_rules(1, 1.5, 1e-8, 0.05, 0.1, n_sigma=5, M=300, dw=0.2, n_t=17, t_min=-9.0,
                      t_max=3.0, nufft_tol=1e-10)
    assert (p["n_sigma"], p["M"], p["dw"], p["n_t"], p["t_min"], p["t_max"]) == (5, 300, 0.2, 17, -9.0, 3.0)
    assert p["w"] == 11 and not p["m_capped"]


@pytest.mark.parametrize("args,code", [
    ((0, 1.5, 1e-6, 0.1, 0.2), gp.GP_EINVAL),
    ((2, -1.0, 1e-6, 0.1, 0.2), gp.GP_EDOMAIN),
    ((2, 1.5, 0.0, 0.1, 0.2), gp.GP_EDOMAIN),
    ((2, 1.5, 1e-6, 0.2, 0.1), gp.GP_EDOMAIN),
    ((2, 1.5, 1e-6, 0.0, 0.1), gp.GP_EDOMAIN),
])
def test_rules_reject_bad_arguments(args, code):
    with pytest.raises(gp.GpError) as e:
        gp.plan_rules(*args)
    assert e.value.code == code


@pytest.mark.parametrize("d,nu,tol,lmin,lmax,M", [(2, 0.5, 1e-8, 0.02, 0.04, 0), (2, 0.5, 1e-8, 0.02, 0.04, 40),
                                                (1, 0.5, 1e-10, 0.05, 0.1, 200), (2, 1.5, 1e-8, 0.05, 0.1, 0)])
def test_flat_t_nodes_merged_where_constant_over_the_box(d, nu, tol, lmin, lmax, M):
    """rem:step3 with the reading that t terms whose Fourier multiplier is
    constant over the mode box merge into one term: the merged nodes are exactly
    the leading nodes whose largest exponent 2 pi^2 sigma_max^2 chi_j^2 dw^2 d M^2
    is <= 1e-3 tol (recomputed here from the plan's t grid), and keep_t = 1
    turns the merge off."""
    kw = {"M": M} if M else {}
    r = gp.plan_rules(d, nu, tol, lmin, lmax, 1.0, **kw)
    nt = r["n_t"]
    t = r["t_min"] + np.arange(nt + 1) / nt * (r["t_max"] - r["t_min"])
    chi2 = np.exp(t) / nu
    x = 2 * np.pi ** 2 * r["s_max"] ** 2 * chi2 * r["dw"] ** 2 * d * r["M"] ** 2
    flat = int(np.argmax(x > 1e-3 * tol)) if np.any(x > 1e-3 * tol) else nt + 1
    want = flat if flat >= 2 else 0
    assert r["n_t_merged"] == want
    assert gp.plan_rules(d, nu, tol, lmin, lmax, 1.0, keep_t=1, **kw)["n_t_merged"] == 0
    if want:
        # the merged terms are constant over the box to 1e-3 tol: exp(-x) >= 1 - 1e-3 tol
        assert np.all(1.0 - np.exp(-x[:want]) <= 1e-3 * tol)
