"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses a closed form,
a library routine (scipy / numpy), an invariant, brute-force quadrature or a
number printed in the paper (tests/golden/paper_setups.json).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle as O
from paper_2407_03608_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_setups.json")))


def setup_module(_):
    O.build()


# ------------------------------------------------------------------ phi_nu --

@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_closed_forms_match_bessel(nu):
    r = np.linspace(0.0, 8.0, 81)
    # scipy's kv is an independent Bessel implementation (library routine)
    z = np.sqrt(2 * nu) * r[1:]
    ref = np.concatenate([[1.0], 2 ** (1 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z)])
    assert np.abs(O.matern(nu, r) - ref).max() < 1e-14
    assert np.abs(O.matern_bessel(nu, r) - ref).max() < 1e-14


def test_matern_half_is_exponential_and_se_limit():
    r = np.linspace(0, 6, 31)
    assert np.abs(O.matern(0.5, r) - np.exp(-r)).max() < 1e-15
    assert np.abs(O.matern(math.inf, r) - np.exp(-r ** 2 / 2)).max() < 1e-15
    # nu -> infinity recovers the squared exponential (section 2)
    e50 = np.abs(O.matern_bessel(50.0, r) - np.exp(-r ** 2 / 2)).max()
    e120 = np.abs(O.matern_bessel(120.0, r) - np.exp(-r ** 2 / 2)).max()
    assert e120 < 2e-3 and e120 < e50 / 2


@pytest.mark.parametrize("nu", [0.5, 0.7, 1.5, 2.5, 3.3])
def test_schoenberg_representation(nu):
    """Appendix C: u(t) = e^{nu t - e^t}/Gamma(nu), chi^2 = e^t/nu reproduces phi_nu."""
    r = np.array([0.0, 0.05, 0.3, 1.0, 2.5])
    ref = np.array([1.0] + [2 ** (1 - nu) / scipy.special.gamma(nu) * (math.sqrt(2 * nu) * v) ** nu
                            * scipy.special.kv(nu, math.sqrt(2 * nu) * v) for v in r[1:]])
    got = O.matern_schoenberg(nu, r, -40.0 / nu - 40, 5.0, 20000)
    assert np.abs(got - ref).max() < 1e-10


# ------------------------------------------------------------ exact kernel --

def test_kernel_diagonal_symmetry_and_ps_form():
    p = inputs.random_small(2, 40, seed=3, nu=1.5)
    K = O.kernel_matrix(p.x, p.sigma, p.l, p.nu)
    assert np.abs(np.diag(K) - p.sigma ** 2).max() < 1e-13
    assert np.abs(K - K.T).max() == 0.0
    # Paciorek-Schervish closed form written in its own parameterisation
    lx, ly = p.l[:, None], p.l[None, :]
    q = lx ** 2 + ly ** 2
    r = np.linalg.norm(p.x[:, None, :] - p.x[None, :, :], axis=-1) * np.sqrt(2.0 / q)
    ps = p.sigma[:, None] * p.sigma[None, :] * (2 * lx * ly / q) ** (p.d / 2) * (1 + math.sqrt(3) * r) * np.exp(-math.sqrt(3) * r)
    assert np.abs(K - ps).max() < 1e-13


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, math.inf])
def test_kernel_stationary_reduction(nu):
    """Constant sigma and l give the textbook Matern sigma^2 phi_nu(|x-y|/l)."""
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, (30, 2))
    s, l = 1.7, 0.23
    K = O.kernel_matrix(x, np.full(30, s), np.full(30, l), nu)
    r = np.linalg.norm(x[:, None] - x[None], axis=-1) / l
    if math.isinf(nu):
        ref = np.exp(-r ** 2 / 2)
    else:
        z = np.sqrt(2 * nu) * np.maximum(r, 1e-300)
        ref = np.where(r == 0, 1.0, 2 ** (1 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z))
    assert np.abs(K - s * s * ref).max() < 1e-13


@pytest.mark.parametrize("d,nu", [(1, 0.5), (2, 1.5), (3, 2.5)])
def test_kernel_positive_definite(d, nu):
    p = inputs.random_small(d, 64, seed=d, nu=nu)
    K = O.kernel_matrix(p.x, p.sigma, p.l, nu)
    assert np.linalg.eigvalsh(K).min() > 0.0
    O.cholesky(K)  # must not raise


def test_cholesky_solve_matches_lapack():
    p = inputs.random_small(2, 300, seed=5, nu=1.5)
    K = O.kernel_matrix(p.x, p.sigma, p.l, p.nu) + p.eta ** 2 * np.eye(p.n)
    a = O.gpr_solve_exact(p.x, p.sigma, p.l, p.nu, p.eta, p.y)
    ref = np.linalg.solve(K, p.y)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-10
    assert np.linalg.norm(K @ a - p.y) / np.linalg.norm(p.y) < 1e-12
    # the LAPACK-factorised variant used for large reference solves agrees
    al = O.gpr_solve_exact(p.x, p.sigma, p.l, p.nu, p.eta, p.y, lapack=True)
    assert np.linalg.norm(al - a) / np.linalg.norm(a) < 1e-10


def test_exact_matvec_rows_match_dense():
    p = inputs.random_small(2, 200, seed=9)
    K = O.kernel_matrix(p.x, p.sigma, p.l, p.nu)
    a = np.random.default_rng(1).standard_normal(p.n)
    assert np.abs(O.exact_matvec(p.x, p.sigma, p.l, p.nu, a) - K @ a).max() < 1e-12
    part = O.exact_matvec(p.x, p.sigma, p.l, p.nu, a, rows=(50, 70))
    assert np.abs(part - (K @ a)[50:70]).max() < 1e-12


def test_posterior_mean_at_training_points():
    """eq:postmean at the training points equals y - eta^2 alpha (eq:gprsolve)."""
    p = inputs.random_small(1, 150, seed=2)
    a = O.gpr_solve_exact(p.x, p.sigma, p.l, p.nu, p.eta, p.y)
    mu = O.posterior_mean_exact(p.x, p.sigma, p.l, p.nu, a, p.x, p.sigma, p.l)
    assert np.abs(mu - (p.y - p.eta ** 2 * a)).max() < 1e-10


# ----------------------------------------------------- approximation pieces --

def _params(d, nu, sp, n_sigma, dw, M, eps=1e-10, n_t=None, center=None, scale=1.0, tmin=None, tmax=None):
    if math.isinf(nu):
        tmin_, tmax_, nt = 0.0, 0.0, 0
    else:
        tmin_ = math.log(eps / 10) / nu if tmin is None else tmin
        tmax_ = math.log(2 * math.log(10 / eps)) + 0.5 if tmax is None else tmax
        nt = n_t if n_t is not None else int(math.ceil((tmax_ - tmin_) / (math.pi ** 2 / math.log(10 / eps))))
    return O.Params(d=d, nu=nu, t_min=tmin_, t_max=tmax_, n_t=nt, s_min=float(np.min(sp)),
                    s_max=float(np.max(sp)), n_sigma=n_sigma, dw=dw, M=M,
                    center=tuple(center) if center is not None else (0.0, 0.0, 0.0), scale=scale)


def test_chebyshev_nodes_and_partition_of_unity():
    p = _params(1, 1.5, np.array([0.1, 0.4]), 12, 0.1, 10)
    sk = O.sigma_nodes(p)
    assert sk[0] == pytest.approx(0.4) and sk[-1] == pytest.approx(0.1)
    assert np.all(np.diff(sk) < 0)
    for s in np.linspace(0.1, 0.4, 37):
        P = O.lagrange(sk, s)
        assert abs(P.sum() - 1.0) < 1e-12
    for j in range(13):
        P = O.lagrange(sk, sk[j])
        assert np.abs(P - np.eye(13)[j]).max() < 1e-12


@pytest.mark.parametrize("nsig", [1, 2, 3, 5, 8, 13, 20, 31])
def test_chebyshev_lobatto_node_positions(nsig):
    """eq:chebscheme: the width nodes are the Chebyshev-Lobatto points, i.e. the
    N_sigma + 1 extrema of T_{N_sigma} on [-1, 1] mapped affinely onto
    [sigma_min, sigma_max].  The extrema are found independently of the oracle:
    the endpoints plus the roots of T'_{N_sigma} from numpy's Chebyshev class."""
    from numpy.polynomial import chebyshev as C
    smin, smax = 0.037, 0.21
    p = _params(1, 1.5, np.array([smin, smax]), nsig, 0.1, 10)
    sk = np.sort(O.sigma_nodes(p))
    inner = np.sort(C.Chebyshev.basis(nsig).deriv().roots().real) if nsig > 1 else np.array([])
    ext = np.concatenate([[-1.0], inner, [1.0]])
    want = smin + 0.5 * (ext + 1.0) * (smax - smin)
    assert sk.shape == want.shape
    assert np.abs(sk - want).max() < 1e-13 * smax
    # each is an extremum: |T_n| = 1 there
    tn = C.Chebyshev.basis(nsig)(2 * (sk - smin) / (smax - smin) - 1)
    assert np.allclose(np.abs(tn), 1.0, atol=1e-11)


@pytest.mark.parametrize("nsig", [4, 6, 8, 12, 16, 24, 32])
def test_chebyshev_lobatto_lebesgue_constant(nsig):
    """The interpolation of eq:chebscheme on the oracle's nodes has Lebesgue
    constant max_s sum_k |P_k(s)| <= (2/pi) ln(N_sigma + 1) + 1, the bound for
    Chebyshev extrema; equispaced nodes exceed it from N_sigma = 8 on, so the
    check sees a node set of the wrong family."""
    smin, smax = 0.1, 0.45
    p = _params(1, 1.5, np.array([smin, smax]), nsig, 0.1, 10)
    sk = O.sigma_nodes(p)
    grid = np.linspace(smin, smax, 4001)
    lam = max(np.abs(O.lagrange(sk, s)).sum() for s in grid)
    bound = 2 / np.pi * np.log(nsig + 1) + 1
    assert 1.0 <= lam <= bound, (lam, bound)
    if nsig >= 8:
        eq = np.linspace(smax, smin, nsig + 1)
        lam_eq = max(np.abs(O.lagrange(eq, s)).sum() for s in grid)
        assert lam_eq > bound


@pytest.mark.parametrize("kappa,nsig", [(1.5, 6), (2.0, 10), (3.0, 14), (4.0, 20)])
def test_lemma_interp_bound(kappa, nsig):
    """lemma lem:interp: sup_x |e^{-x^2/2s^2} - sum_k P_k(s) e^{-x^2/2 s_k^2}| <= eps_cheb."""
    smin, smax = 0.1, 0.1 * kappa
    p = _params(1, 1.5, np.array([smin, smax]), nsig, 0.1, 10)
    sk = O.sigma_nodes(p)
    bound = 2 * (kappa - 1) * ((kappa - 1) / (kappa + 1)) ** nsig
    xs = np.linspace(0, 8 * smax, 400)
    worst = 0.0
    for s in np.linspace(smin, smax, 121):
        P = O.lagrange(sk, s)
        approx = (P[None, :] * np.exp(-xs[:, None] ** 2 / (2 * sk[None, :] ** 2))).sum(1)
        worst = max(worst, np.abs(np.exp(-xs ** 2 / (2 * s * s)) - approx).max())
    assert worst <= bound


@pytest.mark.parametrize("nu,d", [(0.5, 1), (1.5, 2), (2.5, 3)])
def test_tgrid_reproduces_matern(nu, d):
    """eq:trapsum with eq:maternpres: sum_j v_j chi_j^d e^{-r^2/2chi_j^2} -> phi_nu(r)
    (the integrand of eq:BtBtstar0 at unit weights), and v~ = dw^d v."""
    eps = 1e-12
    p = _params(d, nu, np.array([0.2, 0.2]), 0, 0.3, 4, eps=eps)
    t, vt, chi = O.tgrid(p)
    v = vt / 0.3 ** d
    assert np.allclose(np.diff(t), (p.t_max - p.t_min) / p.n_t)
    r = np.array([0.0, 0.1, 0.5, 1.3, 3.0])
    approx = (v[None, :] * chi[None, :] ** d * np.exp(-r[:, None] ** 2 / (2 * chi[None, :] ** 2))).sum(1)
    z = np.sqrt(2 * nu) * np.maximum(r, 1e-300)
    ref = np.where(r == 0, 1.0, 2 ** (1 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z))
    assert np.abs(approx - ref).max() < 1e-9


def test_gaussian_product_integral():
    """Appendix B identity used to derive eq:BtBtstar (checked by quadrature)."""
    a, b, x, y = 0.13, 0.31, 0.2, -0.15
    num, _ = scipy.integrate.quad(lambda z: math.exp(-(x - z) ** 2 / (2 * a * a)) * math.exp(-(y - z) ** 2 / (2 * b * b)), -5, 5, epsabs=1e-14)
    closed = math.sqrt(2 * math.pi * a * a * b * b / (a * a + b * b)) * math.exp(-(x - y) ** 2 / (2 * (a * a + b * b)))
    assert abs(num - closed) < 1e-13


# ---------------------------------------------------------- K-tilde (O2) ----

def _paper_params(prob, n_sigma, M, eps_nufft=1e-6):
    sp = prob.meta["sigma_p"]
    smin, smax = 1 / 6 - 0.01, 1 / 2 + 0.01
    if math.isinf(prob.nu):
        rho_max = smax
        tmin = tmax = 0.0
        nt = 0
    else:
        tmin = (1 + math.log(eps_nufft)) / prob.nu
        tmax = math.log(-2 * math.log(eps_nufft))
        nt = 20
        rho_max = smax * math.exp(tmax / 2) / math.sqrt(prob.nu)
    dw = min(1 / 8, 1 / (4 * rho_max * math.sqrt(math.log(1 / eps_nufft))))
    return O.Params(d=prob.d, nu=prob.nu, t_min=tmin, t_max=tmax, n_t=nt, s_min=smin, s_max=smax,
                    n_sigma=n_sigma, dw=dw, M=M, center=(0, 0, 0), scale=1.0)


@pytest.mark.parametrize("d", [1, 2])
def test_ktilde_se_printed_accuracy(d):
    """section 6.1: with the squared-exponential parameters of fig:matvec1d-gauss /
    fig:matvec2d-gauss the relative matvec error is roughly 1e-7, independent of N."""
    g = GOLDEN["se_ablation"][f"d{d}"]
    prob = inputs.paper_setup(d, 1500 if d == 1 else 600, nu=math.inf)
    p = _paper_params(prob, g["n_sigma"], g["M"])
    a = np.random.default_rng(3).standard_normal(prob.n)
    ex = O.exact_matvec(prob.x, prob.sigma, prob.l, math.inf, a)
    kt = O.ktilde_matvec(p, prob.x, prob.sigma, prob.l, a)
    err = np.linalg.norm(kt - ex) / np.linalg.norm(ex)
    assert err < 10 * GOLDEN["se_ablation"]["relative_matvec_error"], err


def test_ktilde_se_solve_setting_accuracy():
    """section 6.2 noisy regime: N_sigma = 15, M = 75 keeps matvec errors below 1e-5."""
    g = GOLDEN["se_solves_noisy"]
    prob = inputs.paper_setup(2, 600, nu=math.inf)
    p = _paper_params(prob, g["n_sigma"], g["M"])
    a = np.random.default_rng(4).uniform(0, 1, prob.n)
    ex = O.exact_matvec(prob.x, prob.sigma, prob.l, math.inf, a)
    kt = O.ktilde_matvec(p, prob.x, prob.sigma, prob.l, a)
    assert np.linalg.norm(kt - ex) / np.linalg.norm(ex) < g["max_relative_matvec_error"]


def test_ktilde_matern_ablation_decays_in_m_then_saturates():
    """section 6.1, d=1 Matern with N_t = N_sigma = 20: the error falls as M grows
    from the reference value M = 400 and settles at the level the eps = 1e-6
    choices of t_min, t_max allow (each parameter adds its own error term)."""
    g = GOLDEN["matern_ablation"]["d1"]
    prob = inputs.paper_setup(1, 800, nu=1.5)
    a = np.random.default_rng(5).standard_normal(prob.n)
    ex = O.exact_matvec(prob.x, prob.sigma, prob.l, 1.5, a)
    errs = []
    for M in (g["M"], 4 * g["M"]):
        p = _paper_params(prob, g["n_sigma"], M)
        assert p.n_t == g["n_t"]
        kt = O.ktilde_matvec(p, prob.x, prob.sigma, prob.l, a)
        errs.append(np.linalg.norm(kt - ex) / np.linalg.norm(ex))
    assert errs[0] < 1e-3
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-5


def _small_case(d, nu, n, seed, lmin=0.15, lmax=0.3):
    prob = inputs.random_small(d, n, seed, nu=nu, lmin=lmin, lmax=lmax)
    scale = 2.0
    sp = prob.l * scale / math.sqrt(2)
    return prob, sp, scale


@pytest.mark.parametrize("d,nu", [(1, 1.5), (2, 2.5), (1, math.inf), (3, math.inf)])
def test_ktilde_two_independent_forms_agree_and_psd(d, nu):
    """NUDFT five-step matvec vs theta-sum entries (two independent evaluations of
    eq:Ktilde); K~ symmetric and positive semidefinite (section 4)."""
    prob, sp, scale = _small_case(d, nu, 24, seed=d + 10)
    M = {1: 40, 2: 12, 3: 6}[d]
    p = _params(d, nu, sp, 4, 0.15, M, eps=1e-6, center=(0.5, 0.5, 0.5), scale=scale)
    Kt = O.ktilde_entries(p, prob.x, prob.sigma, prob.l)
    assert np.abs(Kt - Kt.T).max() < 1e-12 * np.abs(Kt).max()
    ev = np.linalg.eigvalsh(Kt)
    assert ev.min() > -1e-12 * ev.max()
    a = np.random.default_rng(0).standard_normal(prob.n)
    mv = O.ktilde_matvec(p, prob.x, prob.sigma, prob.l, a)
    assert np.linalg.norm(mv - Kt @ a) / np.linalg.norm(Kt @ a) < 1e-12


def test_ktilde_converges_to_k_1d_matern():
    """K~ -> K as M grows with Delta-omega fixed; the error falls like (M dw)^(-2 nu)
    once the t- and sigma-discretisations are resolved (section 5 / theorem main)."""
    prob, sp, scale = _small_case(1, 1.5, 60, seed=21, lmin=0.2, lmax=0.3)
    a = np.random.default_rng(2).standard_normal(prob.n)
    ex = O.exact_matvec(prob.x, prob.sigma, prob.l, 1.5, a)
    errs = []
    for M in (200, 400, 800, 1600):
        p = _params(1, 1.5, sp, 16, 0.1, M, eps=1e-11, center=(0.5, 0, 0), scale=scale)
        kt = O.ktilde_matvec(p, prob.x, prob.sigma, prob.l, a)
        errs.append(np.linalg.norm(kt - ex) / np.linalg.norm(ex))
    assert errs[-1] < 1e-7
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 4  # at least (1/2)^2; theory gives ~(1/2)^3


def test_ktilde_diagonal_deficit_is_spectral_tail():
    """At the diagonal, K - K~ is the Matern spectral mass outside the Fourier box;
    for d=1 constant scales it is the regularised incomplete beta tail."""
    nu, l = 1.5, 0.3
    x = np.array([[0.5]])
    s = np.array([1.0])
    ll = np.array([l])
    scale = 2.0
    sp = np.array([l * scale / math.sqrt(2)])
    for M in (100, 200):
        p = _params(1, nu, sp, 0, 0.1, M, eps=1e-13, center=(0.5, 0, 0), scale=scale)
        Kt = O.ktilde_entries(p, x, s, ll)[0, 0]
        Om = M * 0.1
        U = 2 * math.pi * (l * scale) * Om / math.sqrt(2 * nu)
        tail = scipy.special.betainc(nu, 0.5, 1 / (1 + U * U))
        assert abs((1.0 - Kt) - tail) < 0.03 * tail


def test_ktilde_stationary_se_matches_textbook_kernel():
    prob, sp, scale = _small_case(2, math.inf, 30, seed=4)
    s = np.full(prob.n, 0.8)
    l = np.full(prob.n, 0.22)
    spc = l * scale / math.sqrt(2)
    p = _params(2, math.inf, spc, 0, 0.12, 60, center=(0.5, 0.5, 0), scale=scale)
    Kt = O.ktilde_entries(p, prob.x, s, l)
    r2 = ((prob.x[:, None] - prob.x[None]) ** 2).sum(-1)
    assert np.abs(Kt - 0.64 * np.exp(-r2 / (2 * 0.22 ** 2))).max() < 1e-10


# ------------------------------------------------- posterior covariance ----

def test_posterior_cov_single_training_point_closed_form():
    """eq:postcov with one observation: Sigma(a, b) = k(a, b) - k(a, x1) k(x1, b) / (k(x1, x1) + eta^2)."""
    rng = np.random.default_rng(31)
    x = rng.uniform(0, 1, (1, 2))
    sx, lx = np.array([1.3]), np.array([0.2])
    xt = rng.uniform(0, 1, (4, 2))
    st, lt = rng.uniform(0.8, 1.2, 4), rng.uniform(0.1, 0.3, 4)
    eta = 0.3
    got = O.posterior_cov_exact(x, sx, lx, 1.5, eta, xt, st, lt)
    kab = O.kernel_matrix(xt, st, lt, 1.5)
    ka1 = O.kernel_matrix(xt, st, lt, 1.5, x, sx, lx)[:, 0]
    ref = kab - np.outer(ka1, ka1) / (sx[0] ** 2 + eta ** 2)
    assert np.allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("nu", [0.5, 2.5])
def test_posterior_cov_at_training_points_noise_identity(nu):
    """At the training points eq:postcov equals eta^2 K (K + eta^2 I)^{-1}."""
    prob = inputs.random_small(2, 60, seed=32, nu=nu, eta=0.2)
    C = O.posterior_cov_exact(prob.x, prob.sigma, prob.l, nu, prob.eta, prob.x, prob.sigma, prob.l)
    K = O.kernel_matrix(prob.x, prob.sigma, prob.l, nu)
    ref = prob.eta ** 2 * np.linalg.solve(K + prob.eta ** 2 * np.eye(prob.n), K).T
    assert np.abs(C - ref).max() < 1e-10 * np.abs(ref).max()


def test_posterior_cov_is_psd_below_prior_and_prior_far_away():
    prob = inputs.random_small(1, 80, seed=33, nu=1.5, eta=0.1, constant_scales=True)
    xt = np.concatenate([np.linspace(0, 1, 7), [40.0]])[:, None]
    st = np.full(8, prob.sigma[0])
    lt = np.full(8, prob.l[0])
    C = O.posterior_cov_exact(prob.x, prob.sigma, prob.l, 1.5, prob.eta, xt, st, lt)
    assert np.abs(C - C.T).max() < 1e-12
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > -1e-12
    assert np.all(np.diag(C) <= st ** 2 + 1e-14)
    # inside the data the variance is reduced; far away it returns to the prior
    assert np.all(np.diag(C)[:7] < 0.5 * st[:7] ** 2)
    assert abs(C[7, 7] - st[7] ** 2) < 1e-12


def test_ktilde_posterior_cov_noise_identity_and_psd():
    """The K~ version (every term from K~ entries) obeys the same identity at the
    training points and is positive semidefinite over targets."""
    prob, sp, scale = _small_case(1, 1.5, 24, seed=34, lmin=0.2, lmax=0.3)
    p = _params(1, 1.5, sp, 6, 0.1, 60, eps=1e-6, center=(0.5, 0, 0), scale=scale)
    Kt = O.ktilde_entries(p, prob.x, prob.sigma, prob.l)
    C = O.ktilde_posterior_cov(p, prob.x, prob.sigma, prob.l, 0.2, prob.x, prob.sigma, prob.l)
    ref = 0.04 * np.linalg.solve(Kt + 0.04 * np.eye(prob.n), Kt).T
    assert np.abs(C - ref).max() < 1e-10 * np.abs(ref).max()
    xt = np.linspace(0.05, 0.95, 5)[:, None]
    st, lt = np.full(5, 1.0), np.full(5, 0.25)
    Ck = O.ktilde_posterior_cov(p, prob.x, prob.sigma, prob.l, 0.2, xt, st, lt)
    assert np.abs(Ck - Ck.T).max() < 1e-12
    assert np.linalg.eigvalsh(Ck).min() > -1e-12
