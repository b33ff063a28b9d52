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


@pytest.mark.parametrize("routing", ["split", "all_fp32"])
def test_server_alone_vs_mix(gp, routing):
    """Each request gives the same bits alone (one slot) and in a mix of
    concurrent requests (six slots, smallest-first admission).  "split" puts
    the fp64-routing threshold at the median fp64 plan size, so both paths
    (plain fp64 CG and fp32-bulk CG inside fp64 refinement) run in the mix;
    "all_fp32" routes every request to the refined fp32-bulk path."""
    probs = _requests(16)
    dev = [(cuda(p.x), cuda(p.sigma), cuda(p.l), cuda(p.y)) for p in probs]
    if routing == "split":
        b64 = sorted(gp.plan_query(x, s, l, p.nu, p.eta, 1e-8) for p, (x, s, l, _) in zip(probs, dev))
        thr = (b64[len(b64) // 2 - 1] + b64[len(b64) // 2]) // 2 + 1
    else:
        thr = 0
    # alone: one slot, one request at a time
    S1 = gp.Server(max_slots=1, max_iter=6000, fp64_below_bytes=thr)
    alone = []
    for p, (x, s, l, y) in zip(probs, dev):
        rid = S1.submit(x, s, l, p.nu, p.eta, y)
        a, info = S1.wait(rid)
        say(f"  alone req d={p.d} n={p.n} nu={p.nu} path={'fp64' if info['precision'] == 0 else 'fp32-bulk'} "
            f"iters={info['iters']} rel={info['rel_res']:.2e} status={info['status']}")
        alone.append((host(a), info))
    S1.close()
    # mix: everything submitted at once to a 6-slot server (smallest-first admission)
    S6 = gp.Server(max_slots=6, max_iter=6000, policy=gp.GP_SERVE_SMALLEST, fp64_below_bytes=thr)
    ids = [S6.submit(x, s, l, p.nu, p.eta, y) for p, (x, s, l, y) in zip(probs, dev)]
    mix = [S6.wait(i) for i in ids]
    st = S6.stats()
    say(f"  server stats {st}")
    S6.close()
    assert st["peak_running"] > 1
    paths = [im["precision"] for _, im in mix]
    say(f"  paths in the mix: {paths.count(gp.GP_FP64)} fp64, {paths.count(gp.GP_FP32_BULK)} fp32-bulk")
    if routing == "split":
        assert gp.GP_FP64 in paths and gp.GP_FP32_BULK in paths
    else:
        assert all(q == gp.GP_FP32_BULK for q in paths)
    for (aa, ia), (am, im) in zip(alone, mix):
        assert ia["precision"] == im["precision"]
        assert ia["status"] == im["status"] == 0
        assert ia["iters"] == im["iters"] and ia["refinements"] == im["refinements"]
        assert im["rel_res"] <= 1e-6
        assert np.array_equal(aa, host(am))


def test_server_orders_reads_after_the_producer_stream(gp):
    """Inputs still being written on a side stream at submit time: the server
    waits for that stream's work (an event recorded at submit) before reading
    them, so the result equals that of inputs produced synchronously."""
    import torch
    p = _requests(2)[1]
    S = gp.Server(max_slots=2, max_iter=6000)
    x, s, l, y = cuda(p.x), cuda(p.sigma), cuda(p.l), cuda(p.y)
    torch.cuda.synchronize()
    ref, iref = S.wait(S.submit(x, s, l, p.nu, p.eta, y))
    ref = host(ref)
    hx, hs, hl, hy = (torch.from_numpy(np.ascontiguousarray(v)).pin_memory()
                      for v in (p.x, p.sigma, p.l, p.y))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        big = torch.randn(4096, 4096, device="cuda", dtype=torch.float32)
        for _ in range(24):   # tens of milliseconds of work queued before the inputs
            big = big @ big
            big = big / big.norm()
        zero = 0.0 * big[0, 0].double()
        xs = hx.to("cuda", non_blocking=True) + zero
        ss = hs.to("cuda", non_blocking=True) + zero
        ls = hl.to("cuda", non_blocking=True) + zero
        ys = hy.to("cuda", non_blocking=True) + zero
        rid = S.submit(xs, ss, ls, p.nu, p.eta, ys)   # stream defaults to the current (side)
    got, info = S.wait(rid)
    S.close()
    say(f"  producer-stream request: iters {info['iters']} vs {iref['iters']}")
    assert info["status"] == 0 and info["iters"] == iref["iters"]
    assert np.array_equal(host(got), ref)


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
