"""Determinism of the operator and the serving loop: a request's result is the
same alone and in a mix of concurrent requests."""
import numpy as np
import pytest

from paper_2407_03608_amd import inputs
from tests.gpu_common import cuda, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_03608_amd import gp as g
    g.load()
    return g


@pytest.mark.parametrize("d,prec", [(1, 0), (2, 0), (2, 1), (3, 1)])
def test_matvec_and_plan_are_bitwise_reproducible(gp, d, prec):
    prob = inputs.random_small(d, 2000 if d < 3 else 800, seed=70 + d, nu=1.5, lmin=0.05, lmax=0.15)
    tol = 1e-8 if prec == 0 else 1e-4
    P1 = gp.Plan(cuda(prob.x), cuda(prob.sigma), cuda(prob.l), prob.nu, prob.eta, tol, precision=prec)
    P2 = gp.Plan(cuda(prob.x), cuda(prob.sigma), cuda(prob.l), prob.nu, prob.eta, tol, precision=prec)
    a = cuda(np.random.default_rng(0).standard_normal(prob.n))
    r1 = host(P1.matvec(a))
    r1b = host(P1.matvec(a))
    r2 = host(P2.matvec(a))
    assert np.array_equal(r1, r1b) and np.array_equal(r1, r2)


def _requests(k):
    """A mix of small requests (d 1-2, N 500-8000, nu 1/2..5/2) that solve in
    well under a second each."""
    rng = np.random.default_rng(11)
    out = []
    for i in range(k):
        d = int(rng.integers(1, 3))
        n = int(rng.integers(500, 8000))
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        out.append(inputs.random_small(d, n, seed=100 + i, nu=nu, lmin=0.06, lmax=0.2, eta=0.1))
    return out


def test_server_alone_vs_mix(gp):
    probs = _requests(16)
    dev = [(cuda(p.x), cuda(p.sigma), cuda(p.l), cuda(p.y)) for p in probs]
    # alone: one slot, one request at a time
    S1 = gp.Server(max_slots=1, max_iter=6000)
    alone = []
    for p, (x, s, l, y) in zip(probs, dev):
        rid = S1.submit(x, s, l, p.nu, p.eta, y)
        a, info = S1.wait(rid)
        say(f"  alone req d={p.d} n={p.n} nu={p.nu} iters={info['iters']} rel={info['rel_res']:.2e} status={info['status']}")
        alone.append((host(a), info))
    S1.close()
    # mix: everything submitted at once to a 6-slot server (smallest-first admission)
    S6 = gp.Server(max_slots=6, max_iter=6000, policy=gp.GP_SERVE_SMALLEST)
    ids = [S6.submit(x, s, l, p.nu, p.eta, y) for p, (x, s, l, y) in zip(probs, dev)]
    mix = [S6.wait(i) for i in ids]
    st = S6.stats()
    say(f"  server stats {st}")
    S6.close()
    assert st["peak_running"] > 1
    for (aa, ia), (am, im) in zip(alone, mix):
        assert ia["status"] == im["status"]
        assert ia["iters"] == im["iters"]
        assert np.array_equal(aa, host(am))


def test_server_precision_routing(gp):
    """Small operators are solved in fp64 directly; with the threshold at zero
    every request takes the fp32-bulk refined path; both reach the tolerance."""
    probs = _requests(3)
    dev = [(cuda(p.x), cuda(p.sigma), cuda(p.l), cuda(p.y)) for p in probs]
    out = {}
    for thr in (1 << 40, 0):
        S = gp.Server(max_slots=2, max_iter=6000, fp64_below_bytes=thr)
        ids = [S.submit(x, s, l, p.nu, p.eta, y) for p, (x, s, l, y) in zip(probs, dev)]
        out[thr] = [S.wait(i) for i in ids]
        S.close()
    for (a64, i64), (a32, i32) in zip(out[1 << 40], out[0]):
        say(f"  fp64 iters={i64['iters']} rel={i64['rel_res']:.2e} | fp32-bulk iters={i32['iters']} "
            f"passes={i32['refinements']} rel={i32['rel_res']:.2e}")
        assert i64["precision"] == gp.GP_FP64 and i32["precision"] == gp.GP_FP32_BULK
        assert i64["status"] == 0 and i32["status"] == 0
        assert i64["rel_res"] <= 1e-6 and i32["rel_res"] <= 1e-6


def test_server_rejects_oversized_and_bad_requests(gp):
    p = _requests(1)[0]
    S = gp.Server(max_slots=2, max_device_bytes=1 << 20)
    with pytest.raises(gp.GpError) as e:
        S.submit(cuda(p.x), cuda(p.sigma), cuda(p.l), p.nu, p.eta, cuda(p.y))
    assert e.value.code == gp.GP_ENOMEM
    S.close()
    S = gp.Server(max_slots=2)
    bad = p.l.copy()
    bad[0] = -1.0
    with pytest.raises(gp.GpError) as e:
        S.submit(cuda(p.x), cuda(p.sigma), cuda(bad), p.nu, p.eta, cuda(p.y))
    assert e.value.code == gp.GP_EDOMAIN
    S.close()
