"""gp_cg_solve_noalloc, called through the C ABI, against gp_cg_solve.

The allocation-free solve runs the same kernels with its reduction scratch in
a static device array shared by every call on the GPU, so it must reproduce
gp_cg_solve bit for bit: iterates, iteration count and status.  Two calls in a
row, the second on a smaller problem (the scratch then holds the first call's
contents), plus a non-converged call and a warm start.
"""
import ctypes

import numpy as np
import pytest

from paper_2407_03608_amd import inputs
from tests.gpu_common import cuda, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_03608_amd import gp as g
    g.load()
    return g


def _noalloc(gp, P, y, alpha, tol, max_iter, use_x0=0, replace_every=0):
    info = gp.GpCgInfo()
    rc = gp.load().gp_cg_solve_noalloc(P.handle, y.data_ptr(), alpha.data_ptr(), int(use_x0),
                                       float(tol), int(max_iter), int(replace_every),
                                       ctypes.byref(info))
    return rc, info


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_solve_matches_cg_solve(gp, prec):
    import torch
    cases = [(2, 3000, 20, 31), (1, 700, 60, 32)]  # the second call is smaller
    for d, n, M, seed in cases:
        prob = inputs.random_small(d, n, seed=seed, nu=1.5, lmin=0.08, lmax=0.2, eta=0.2)
        tol_plan = 1e-9 if prec == 0 else 1e-4
        P = gp.Plan(cuda(prob.x), cuda(prob.sigma), cuda(prob.l), prob.nu, prob.eta, tol_plan,
                    precision=prec, M=M)
        y = cuda(prob.y)
        # the fp32-bulk operator's CG stalls near its own accuracy (~1e-3)
        tol = 1e-9 if prec == 0 else 3e-3
        ref, iref = P.cg_solve(y, tol=tol, max_iter=4000, replace_every=13)
        alpha = torch.full_like(y, 7.0)  # overwritten (use_x0 = 0)
        rc, info = _noalloc(gp, P, y, alpha, tol, 4000, replace_every=13)
        say(f"case noalloc d={d} n={n} prec={prec}: rc={rc} iters={info.iters} "
            f"(cg_solve {iref['iters']}) rel_res={info.rel_res:.2e}")
        assert rc == gp.GP_OK and info.status == gp.GP_OK
        assert info.iters == iref["iters"] and info.rel_res == iref["rel_res"]
        assert np.array_equal(host(alpha), host(ref))
        # not converged: status and the last iterate agree too
        r2, i2 = P.cg_solve(y, tol=1e-14, max_iter=9)
        a2 = torch.empty_like(y)
        rc, info = _noalloc(gp, P, y, a2, 1e-14, 9)
        assert rc == gp.GP_ENOCONV and info.iters == 9 == i2["iters"]
        assert np.array_equal(host(a2), host(r2))
        # warm start from that iterate
        r3, i3 = P.cg_solve(y, tol=tol, max_iter=4000, x0=r2)
        rc, info = _noalloc(gp, P, y, a2, tol, 4000, use_x0=1)
        assert rc == gp.GP_OK and info.iters == i3["iters"]
        assert np.array_equal(host(a2), host(r3))
        P.close()
