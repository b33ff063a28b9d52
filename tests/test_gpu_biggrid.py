"""Dense parity on the large-grid FFT paths of the d=2 N=1e6 workload.

The headline plan has M = 2047: its fine grid is 6144 points per side at the
automatic 2-D oversampling (radix-24 passes) and 8192 at oversampling 2.  Here
a few hundred points carry a dense alpha through exactly those passes: the
plan forces M = 2047 and the workload's Delta-omega, with a small N_sigma and
N_t so that the oracle can form every entry of K~ (eq:Ktilde, theta-sum form)
and the product K~ alpha is compared element by element.  The points include
the corners and edges of the box and points whose first window cell lies on a
spreading-tile or interpolation-block boundary.
"""
import numpy as np
import pytest

import oracle as O
from paper_2407_03608_amd import inputs
from tests.gpu_common import cuda, host, max_rel, oracle_params, rel, say

pytestmark = pytest.mark.gpu

N_SIGMA, N_T = 3, 6


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_03608_amd import gp as g
    g.load()
    O.build()
    return g


def _edge_points(rules, n_rand, seed):
    """Points in [0,1]^2 (the box is fixed to it): box corners and edge
    midpoints, points whose first window cell is the first or last cell of a
    tile or of a 2x2 interpolation block, and uniform points."""
    nf, dw, w = rules["nf"][0], rules["dw"], rules["w"]
    lo, tile = rules["lo"][0], rules["tile"][0]
    rng = np.random.default_rng(seed)
    pts = [[0, 0], [1, 0], [0, 1], [1, 1], [0.5, 0], [0.5, 1], [0, 0.5], [1, 0.5]]
    # first window cell s = ceil(g - w/2) with g = nf/2 + nf dw x', x' = 2x - 1
    def x_for_cell(c):
        g = (c + lo) + 0.5 * w - 0.5      # inside (s - 1, s] after the shift
        return ((g - 0.5 * nf) / (nf * dw) + 1.0) / 2.0
    cells = []
    for j in range(1, rules["na"][0] // tile - 1, 7):
        cells += [j * tile, j * tile + tile - 1, 2 * j * tile + 2 * tile - 1]
    cells = [c for c in cells if c + w <= rules["na"][0]]
    for k in range(24):
        cx, cy = rng.choice(cells, 2)
        p = [x_for_cell(cx), x_for_cell(cy)]
        if 0 <= p[0] <= 1 and 0 <= p[1] <= 1:
            pts.append(p)
    pts = np.array(pts, dtype=np.float64)
    return np.concatenate([pts, rng.uniform(0, 1, size=(n_rand, 2))])


@pytest.mark.parametrize("ups,nf", [(1.25, 6144), (2.0, 8192)])
def test_dense_alpha_on_headline_grid(gp, ups, nf):
    base = inputs.matern_2d(n=16)  # the workload's scales and nu
    rules = gp.plan_rules(2, base.nu, 1e-8, 0.02, 0.04, 1.0, upsample=ups)
    x = _edge_points(rules, 150, seed=3)
    n = x.shape[0]
    sigma = np.exp(0.3 * x[:, 0])
    l = 0.02 + 0.02 * x[:, 1]
    a = np.random.default_rng(4).standard_normal(n)
    ref = None
    outs = {}
    for prec, tol, bar in ((0, 1e-8, 1e-6), (1, 1e-4, 2e-4)):
        P = gp.Plan(cuda(x), cuda(sigma), cuda(l), base.nu, 0.05, tol, precision=prec,
                    M=2047, dw=rules["dw"], n_sigma=N_SIGMA, n_t=N_T, t_min=rules["t_min"],
                    t_max=rules["t_max"], upsample=ups, box_lo=(0, 0, 0), box_hi=(1, 1, 1))
        info = P.info()
        say(f"case big grid ups={ups} prec={prec}: nf={info['nf'][0]} w={info['w']} "
            f"na={info['na'][:2]} tile={info['tile'][:2]} n={n}")
        assert info["nf"][0] == nf and info["M"] == 2047
        if ref is None:
            ref = O.ktilde_entries(oracle_params(info), x, sigma, l) @ a
        got = host(P.matvec(cuda(a)))
        e, em = rel(got, ref), max_rel(got, ref)
        say(f"  vs oracle K~: {e:.3e} (2-norm), {em:.3e} (max element / max |ref|)")
        assert e <= bar and em <= bar
        outs[prec] = got
        P.close()
    # the two precisions realise the same K~ (same N_sigma, N_t, dw, M)
    assert rel(outs[1], outs[0]) <= 2e-4
