"""Benchmark of the hot path on one MI355X.

Workload (default): d=2, N=1e6 points uniform on [0,1]^2, Matern nu=1/2,
sigma(x)=exp(0.3 x1), l(x)=0.02+0.02 x2, eta=0.05, fp64 end to end.  One
"step" is one conjugate-gradient iteration on (K~ + eta^2 I) alpha = y: the
full matvec (spread, forward FFT, Fourier mixing, inverse FFT, interpolation
and combine) plus the fp64 dot products and vector updates.  The value is
matvec points per second (N x steps / seconds).  The same problem is also
stepped through the fp32-bulk path (fp32 grids, fp64 vectors) and reported
beside it.  Inputs are synthetic (seeded) and resident in HBM before timing.

The default run also measures the rest of the headline metric:
  cg_solve  full CG solves to 1e-6 at d=2 N=1e6: the fp64 path and the
            fp32-bulk path (fp32-operator CG inside fp64 refinement), with
            iterations, true fp64 residuals and the difference of the two
            solutions; and, on the first 10^4 points as a sub-problem, both
            paths' solutions against the oracle's exact Cholesky solution
  serving   p50/p99 latency and solves/s of the first R requests (default 16)
            of the 512-request Poisson stream, continuous batching

  python bench.py [--steps K] [--warmup W] [--no-solve] [--serve-requests R] [--no-cpu]
  python bench.py --serving [--requests R] [--slots S]     (the whole stream)

--serving replays a Poisson stream of independent GPR solve requests
(d in {1,2}, N log-uniform in [1e3, 5e5], random smooth sigma/l, fp32-bulk
operator with fp64 refinement to 1e-6) against the continuous-batching server
and reports latency percentiles (arrival to alpha ready), solves/s and the
admitted concurrency.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--tol64", type=float, default=1e-8)
    ap.add_argument("--tol32", type=float, default=1e-4)
    ap.add_argument("--no-solve", action="store_true", help="skip the full CG solves to 1e-6")
    ap.add_argument("--oracle-sub", type=int, default=10000,
                    help="points of the sub-problem whose solutions are checked against the "
                         "oracle's exact Cholesky solution (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the serving leg in the default run (0 = skip)")
    ap.add_argument("--upsample", type=float, default=0.0,
                    help="fine-grid oversampling of every plan, 1.25..2 (window widened to "
                         "match); 0 = the library's automatic choice")
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--inner-tol", type=float, default=3e-3)
    ap.add_argument("--replace-every", type=int, default=0,
                    help="residual recomputation period inside the fp32-bulk inner CG")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="end with one device copy of this size (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary workloads (d=1 N=2000, d=3 N=1e7)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", choices=["matern_3d"], default=None,
                    help="run only this secondary workload (e.g. under a profiler) and print its line")
    ap.add_argument("--serving", action="store_true", help="serving benchmark instead of matvec steps")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--serve-bytes-gib", type=float, default=200.0)
    ap.add_argument("--serve-max-iter", type=int, default=20000)
    ap.add_argument("--policy", choices=["smallest", "fifo"], default="smallest",
                    help="admission order of queued requests")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(info: dict, kernel: str) -> float:
    """Algorithmic HBM bytes of one launch group of `kernel` for one matvec
    (each grid value of the active box or of the kept modes read or written
    once, plus the point rows and vectors)."""
    d = info["d"]
    s = 8 if info["precision"] == 0 else 4
    cs = 2 * s
    G = info["n_pairs"]
    na = info["na"][:d]
    mc = 2 * info["M"] + 1
    n = info["n"]
    act = math.prod(na)
    if kernel == "spread":
        return G * act * cs + n * (8 + 4 * d + s * d + 16)
    if kernel == "interp":
        return G * act * cs + n * (8 + 4 * d + s * d + 16 + 8)
    if kernel == "mode":
        return 2 * G * mc ** d * cs
    if kernel.startswith("fft"):
        r = int(kernel[-1])
        # pass over dim r: sizes before / after (dims < r already in modes)
        before = [mc] * r + list(na[r:])
        after = [mc] * (r + 1) + list(na[r + 1:])
        return G * (math.prod(before) + math.prod(after)) * cs
    if kernel == "cg_vec":
        return n * 8 * 8
    return 0.0


def run_steps(P, y, steps):
    """Exactly `steps` CG iterations from x0 = 0 (tolerance never reached)."""
    alpha, info = P.cg_solve(y, tol=1e-300, max_iter=steps)
    assert info["iters"] == steps, info
    return info


def time_path(gp, torch, P, y, steps, warmup):
    if warmup:
        run_steps(P, y, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(P, y, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel HIP-event times over a second identical run
    P.set_timing(True)
    run_steps(P, y, steps)
    tm = P.timing()
    P.set_timing(False)
    return (t1 - t0), tm


TRAFFIC_FILES = {"matern_2d": os.path.join(ROOT, "profiles", "matern_2d_hbm_counters.md"),
                 "matern_3d": os.path.join(ROOT, "profiles", "matern_3d_hbm_counters.md")}


def kernel_sources_sha256() -> str:
    """Hash of the HIP sources; the counter summary records the hash it was taken at."""
    import glob
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2407_03608_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(d, "*.hip")) + glob.glob(os.path.join(d, "*.h"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per matvec of `kernel` from the committed counter summary of
    the workload, or None when there is none or it was taken on other kernel
    sources."""
    try:
        txt = open(TRAFFIC_FILES[workload]).read()
        blk = txt.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(blk)
    except (OSError, IndexError, ValueError):
        return None
    if data.get("sources_sha256") != kernel_sources_sha256():
        return None
    k = data.get("per_matvec_bytes", {}).get(precision, {}).get(kernel)
    return None if k is None else k["read"] + k["write"]


def roofline(info, tm, steps):
    best = None
    for name, (launches, ms) in tm.items():
        if launches == 0 or name == "cg_vec":
            continue
        per_launch_ms = ms / steps  # one launch group per matvec
        if best is None or per_launch_ms > best[1]:
            best = (name, per_launch_ms)
    name, ms = best
    b = alg_bytes(info, name)
    achieved = b / (ms * 1e-3) / 1e9
    prec = "fp64" if info["precision"] == 0 else "fp32"
    wl = ("matern_2d" if info["d"] == 2 and info["n"] == 1_000_000 else
          "matern_3d" if info["d"] == 3 and info["n"] == 10_000_000 else None)
    tr = measured_traffic(wl, prec, name) if wl else None
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if tr is None else round(tr / 1e9, 4), "traffic_unit": "GB per launch group",
            "avg_ms": round(ms, 4), "alg_bytes": b}


def matern_3d_leg(gp, torch, args, steps=10, warmup=2):
    """d=3 N=1e7 Gaussian-mixture nu=5/2 in fp32-bulk (spreading-heavy)."""
    from paper_2407_03608_amd import inputs
    log("secondary: matern_3d fp32-bulk")
    p3 = inputs.matern_3d()
    X, S, L, Y = (torch.as_tensor(v).to("cuda") for v in (p3.x, p3.sigma, p3.l, p3.y))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = gp.Plan(X, S, L, p3.nu, p3.eta, 1e-4, precision=gp.GP_FP32_BULK, upsample=args.upsample)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    info = P.info()
    t, tm = time_path(gp, torch, P, Y, steps, warmup)
    rf = roofline(info, tm, steps)
    out = {
        "workload": "d=3 N=1e7 8-component Gaussian mixture clipped to [0,1]^3, nu=5/2, sigma=1, "
                    "l=0.03+0.02|x-0.5|, eta=0.1, fp32-bulk tol 1e-4",
        "ms_per_step": round(1e3 * t / steps, 4), "points_per_s": round(p3.n * steps / t, 1),
        "roofline": rf, "kernels_ms": {k: round(v[1] / steps, 4) for k, v in tm.items() if v[0]},
        "plan_seconds": round(tp, 3),
        "plan": {k: info[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "upsample", "na", "n_pairs", "device_bytes")}}
    P.close()
    return out


def secondary_workloads(gp, torch, args):
    """The other measured configurations, reported beside the headline:
    d=1 N=2000 nu=3/2 fp64 (launch-bound; full solve to 1e-8) and d=3 N=1e7
    Gaussian-mixture nu=5/2 in fp32-bulk (spreading-heavy)."""
    from paper_2407_03608_amd import inputs
    out = {}
    dev = "cuda"
    log("secondary: matern_1d")
    p1 = inputs.matern_1d()
    X, S, L, Y = (torch.as_tensor(v).to(dev) for v in (p1.x, p1.sigma, p1.l, p1.y))
    P = gp.Plan(X, S, L, p1.nu, p1.eta, 1e-8, upsample=args.upsample)
    info = P.info()
    t, tm = time_path(gp, torch, P, Y, 200, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ci = P.cg_solve(Y, tol=1e-8, max_iter=20000)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["matern_1d_fp64"] = {
        "workload": "d=1 N=2000 nu=3/2 sigma=1+0.5 sin 2 pi x, l=0.05+0.03 cos 2 pi x, eta=0.1, fp64 tol 1e-8",
        "ms_per_step": round(1e3 * t / 200, 4), "points_per_s": round(p1.n * 200 / t, 1),
        "solve_1e-8": {"seconds": round(ts, 4), "iters": ci["iters"], "status": ci["status"]},
        "kernels_ms": {k: round(v[1] / 200, 4) for k, v in tm.items() if v[0]},
        "plan": {k: info[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "upsample")}}
    P.close()
    del X, S, L, Y
    out["matern_3d_fp32_bulk"] = matern_3d_leg(gp, torch, args)
    out["multi_rhs_cg"] = multi_rhs_leg(gp, torch, inputs)
    return out


def multi_rhs_leg(gp, torch, inputs, m=16):
    """Solves for m right-hand sides on one plan, as in the posterior
    covariance (eq:postcov): d=2, N=1e5, nu=5/2, l in [0.03, 0.06], eta=0.3,
    fp64 tol 1e-8, CG to 1e-6.  Block CG (gp_cg_solve_multi, block = 1: one
    Krylov space, each operator application shared by the block) and lockstep
    multi-right-hand-side CG (block = 0) against m sequential gp_cg_solve
    calls; then gp_posterior_cov at m targets (block CG inside)."""
    import numpy as np
    log("secondary: multi-right-hand-side CG")
    p = inputs.random_small(2, 100_000, seed=12, nu=2.5, lmin=0.03, lmax=0.06, eta=0.3)
    X, S, L = (torch.as_tensor(v).to("cuda") for v in (p.x, p.sigma, p.l))
    P = gp.Plan(X, S, L, p.nu, p.eta, 1e-8)
    Y = torch.as_tensor(np.random.default_rng(3).standard_normal((m, p.n))).to("cuda")
    P.cg_solve_multi(Y[:2], tol=1e-6, max_iter=20000)  # warm-up (allocates the batched grids)
    out = {"workload": f"d=2 N=1e5 uniform, nu=5/2, l in [0.03,0.06], eta=0.3, fp64 tol 1e-8, "
                       f"{m} random right-hand sides, CG to 1e-6", "m": m}
    for name, blk in (("block", True), ("lockstep", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A, its, rels, info = P.cg_solve_multi(Y, tol=1e-6, max_iter=20000, block=blk)
        torch.cuda.synchronize()
        out[name] = {"seconds": round(time.perf_counter() - t0, 3), "iters": its[0] if blk else its,
                     "worst_rel_res": info["rel_res"], "status": info["status"]}
    t0 = time.perf_counter()
    its1 = []
    for j in range(m):
        _, ci = P.cg_solve(Y[j].contiguous(), tol=1e-6, max_iter=20000)
        its1.append(ci["iters"])
    torch.cuda.synchronize()
    out["serial"] = {"seconds": round(time.perf_counter() - t0, 3), "iters": its1}
    out["block_speedup_vs_serial"] = round(out["serial"]["seconds"] / out["block"]["seconds"], 2)
    rng = np.random.default_rng(5)
    xt = torch.as_tensor(rng.uniform(0.05, 0.95, size=(m, 2))).to("cuda")
    lt = torch.as_tensor(rng.uniform(p.l.min(), p.l.max(), size=m)).to("cuda")
    st = torch.as_tensor(rng.uniform(0.8, 1.2, size=m)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, var, ci = P.posterior_cov(xt, st, lt, tol=1e-6, max_iter=20000)
    torch.cuda.synchronize()
    out["posterior_cov"] = {"targets": m, "seconds": round(time.perf_counter() - t0, 3),
                            "block_iters": ci["iters"], "status": ci["status"]}
    inf = P.info()
    out["plan"] = {"M": inf["M"], "nf": inf["nf"][0], "n_pairs": inf["n_pairs"]}
    P.close()
    return out


def step_model(info, ms):
    """Whole-matvec bytes under the model that counts full oversampled grids:
    (N_sigma+1)(4 n_f^d + 4 (2M+1)^d) s + N (2d+7) s, with s the element size
    (pruning the grids to the active box is a gain against it, not credited)."""
    d = info["d"]
    s = 8 if info["precision"] == 0 else 4
    grids = info["n_sigma"] + 1
    b = grids * (4 * math.prod(info["nf"][:d]) + 4 * (2 * info["M"] + 1) ** d) * s + info["n"] * (2 * d + 7) * s
    gbs = b / (ms * 1e-3) / 1e9
    return {"model": "(N_sigma+1)(4 n_f^d + 4 (2M+1)^d) s + N (2d+7) s", "bytes": b,
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def cpu_baseline(prob, seconds):
    """The oracle's exact dense matvec (rows of K alpha formed on the fly)."""
    import numpy as np

    import oracle as O
    O.build()
    a = np.random.default_rng(0).standard_normal(prob.n)
    rows = 64
    t0 = time.perf_counter()
    O.exact_matvec(prob.x, prob.sigma, prob.l, prob.nu, a, rows=(0, rows))
    t = time.perf_counter() - t0
    rows = max(64, int(rows * seconds / max(t, 1e-3)))
    rows = min(rows, prob.n)
    t0 = time.perf_counter()
    O.exact_matvec(prob.x, prob.sigma, prob.l, prob.nu, a, rows=(0, rows))
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(rows / t, 3), "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} rows of the exact dense fp64 matvec K alpha at N={prob.n} "
                      f"({rows * prob.n:.2e} kernel evaluations, {t:.1f} s)"}


def run_serving(args, n_requests):
    """Replay the first n_requests of the seed-5 stream.  Requests are
    submitted at their arrival times; the server admits them as slots and
    device bytes allow.  Inputs are resident in HBM before the stream starts.
    Returns the latency / throughput summary."""
    import numpy as np
    import torch

    from paper_2407_03608_amd import gp, inputs

    assert torch.cuda.is_available()
    log(f"serving: generating {n_requests} requests")
    reqs = inputs.serving_stream(n_requests=n_requests, rate=args.rate, seed=5)
    dev = []
    for r in reqs:
        p = r.problem
        dev.append(tuple(torch.as_tensor(np.ascontiguousarray(v)).to("cuda")
                         for v in (p.x, p.sigma, p.l, p.y)))
    torch.cuda.synchronize()
    S = gp.Server(max_slots=args.slots, max_device_bytes=int(args.serve_bytes_gib * (1 << 30)),
                  precision=gp.GP_FP32_BULK, max_iter=args.serve_max_iter,
                  policy=gp.GP_SERVE_SMALLEST if args.policy == "smallest" else gp.GP_SERVE_FIFO)
    # warm-up: one small request end to end (kernel loading, first allocations)
    w = inputs.random_small(2, 2000, seed=9, nu=1.5, lmin=0.05, lmax=0.1)
    wid = S.submit(*(torch.as_tensor(v).to("cuda") for v in (w.x, w.sigma, w.l)), w.nu, w.eta,
                   torch.as_tensor(w.y).to("cuda"))
    S.wait(wid)
    log("serving: stream start")
    t0 = time.perf_counter()
    done = 0
    results = {}

    def drain(block):
        nonlocal done
        for rid, k in list(pending.items()):
            if block or S.poll(rid):
                _, info = S.wait(rid)
                results[k] = info
                del pending[rid]
                done += 1
                p = reqs[k].problem
                log(f"  done {done}/{len(reqs)} req {k} d={p.d} n={p.n} nu={p.nu} "
                    f"path={'fp64' if info['precision'] == gp.GP_FP64 else 'fp32-bulk'} "
                    f"iters={info['iters']} status={info['status']} "
                    f"latency={info['t_done'] - info['t_submit']:.3f}s")

    pending = {}
    for k, r in enumerate(reqs):
        while True:
            now = time.perf_counter() - t0
            if now >= r.arrival:
                break
            drain(False)
            time.sleep(min(0.002, r.arrival - now))
        x, sg, l, y = dev[k]
        pending[S.submit(x, sg, l, r.problem.nu, r.problem.eta, y)] = k
    while pending:
        drain(False)
        time.sleep(0.005)
    wall = time.perf_counter() - t0
    st = S.stats()
    S.close()
    del dev
    lat = np.array([results[k]["t_done"] - results[k]["t_submit"] for k in range(len(reqs))])
    queue = np.array([results[k]["t_start"] - results[k]["t_submit"] for k in range(len(reqs))])
    ready = np.array([results[k]["t_ready"] - results[k]["t_start"] for k in range(len(reqs))])
    iters = np.array([results[k]["iters"] for k in range(len(reqs))])
    nonconv = int(sum(results[k]["status"] != 0 for k in range(len(reqs))))
    return {"requests": len(reqs),
            "subset": f"the first {len(reqs)} requests of the seed-5 stream of 512",
            "rate_per_s": args.rate, "slots": args.slots, "policy": args.policy,
            "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p90_s": round(float(np.percentile(lat, 90)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4),
            "max_s": round(float(lat.max()), 4),
            "mean_queue_s": round(float(queue.mean()), 4),
            "admission_to_first_matvec_s": {"p50": round(float(np.percentile(ready, 50)), 4),
                                            "p99": round(float(np.percentile(ready, 99)), 4),
                                            "max": round(float(ready.max()), 4),
                                            "what": "plan build of the request's operators, "
                                                    "from slot admission to the first matvec "
                                                    "queued"},
            "solves_per_s": round(len(reqs) / wall, 4),
            "wall_s": round(wall, 3),
            "peak_running": st["peak_running"],
            "peak_bytes": st["peak_bytes"],
            "nonconverged": nonconv,
            "fp64_routed": int(sum(results[k]["precision"] == gp.GP_FP64 for k in range(len(reqs)))),
            "iters_p50": int(np.percentile(iters, 50)),
            "iters_max": int(iters.max()),
            "points_total": int(sum(r.problem.n for r in reqs))}


def serving(args):
    """--serving: the whole stream as its own benchmark line (metric: p99)."""
    sv = run_serving(args, args.requests)
    out = {
        "metric": "p99 latency of GPR solve requests (arrival to alpha ready), Poisson stream",
        "value": sv["p99_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": sv["requests"],
        "warmup": 1,
        "ms_per_step": round(1e3 * sv["wall_s"] / sv["requests"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-bulk/f64",
        "data": "synthetic (seeded request stream)",
        "config": {"workload": f"serving: {sv['requests']} requests, Poisson {args.rate}/s, d in {{1,2}}, "
                               "N log-uniform [1e3,5e5], nu in {1/2,3/2,5/2}, fp32-bulk + fp64 refinement, "
                               "CG 1e-6", "slots": args.slots, "max_iter": args.serve_max_iter,
                   "policy": args.policy},
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


def solve_legs(gp, torch, O, inputs, prob, P64, P32, Y, args):
    """CG to 1e-6 on (K~ + eta^2 I) alpha = y at d=2 N=1e6 through the fp64 path
    and the fp32-bulk path (fp32-operator CG inside fp64 refinement), then the
    same two solves on the first `oracle_sub` points as a sub-problem, against
    the oracle's exact Cholesky solution (stated: the Fourier box capped at
    M = 2047 leaves K~ a spectral tail away from K for nu = 1/2, see pred_tail)."""
    out = {}
    log("solve: fp64 CG to 1e-6")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    al64, ci64 = P64.cg_solve(Y, tol=1e-6, max_iter=args.max_iter)
    torch.cuda.synchronize()
    s64 = time.perf_counter() - t0
    r64 = P64.residual(Y, al64)
    log(f"solve: fp64 {s64:.1f} s, {ci64['iters']} iterations, true residual {r64:.2e}")
    log("solve: fp32-bulk CG inside fp64 refinement to 1e-6")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    al32, ci32 = gp.cg_solve_refined(P32, P64, Y, tol=1e-6, inner_tol=args.inner_tol,
                                     max_iter=args.max_iter, max_refine=10,
                                     replace_every=args.replace_every)
    torch.cuda.synchronize()
    s32 = time.perf_counter() - t0
    diff = float(torch.linalg.norm(al32 - al64) / torch.linalg.norm(al64))
    log(f"solve: fp32-bulk {s32:.1f} s, {ci32['iters']} iterations, residual {ci32['rel_res_true']:.2e}")
    out["fp64"] = {"seconds": round(s64, 3), "iters": ci64["iters"], "status": ci64["status"],
                   "ms_per_iter": round(1e3 * s64 / max(ci64["iters"], 1), 4),
                   "rel_res_true": r64}
    out["fp32_bulk_refined"] = {
        "seconds": round(s32, 3), "iters": ci32["iters"], "refinements": ci32["refinements"],
        "status": ci32["status"], "inner_tol": args.inner_tol,
        "replace_every": args.replace_every,
        "replace_every_note": "the configuration's residual recomputation every 20 inner "
                              "iterations is available (--replace-every 20) and measured slower; "
                              "0 = off",
        "rel_res_true_fp64_operator": ci32["rel_res_true"],
        "rel_diff_vs_fp64_solution": diff}
    out["fp32_faster_than_fp64"] = bool(s32 < s64)
    del al64, al32
    if args.oracle_sub > 0:
        sub = inputs.subsample(prob, args.oracle_sub)
        log(f"solve: {sub.n}-point sub-problem, oracle exact Cholesky (LAPACK factorisation)")
        t0 = time.perf_counter()
        import numpy as np
        ref = O.gpr_solve_exact(sub.x, sub.sigma, sub.l, sub.nu, sub.eta, sub.y, lapack=True)
        t_or = time.perf_counter() - t0
        dev = [torch.as_tensor(v).to("cuda") for v in (sub.x, sub.sigma, sub.l, sub.y)]
        Q64 = gp.Plan(*dev[:3], sub.nu, sub.eta, args.tol64, upsample=args.upsample)
        qi = Q64.info()
        Q32 = gp.Plan(*dev[:3], sub.nu, sub.eta, args.tol32, precision=gp.GP_FP32_BULK,
                      dw=qi["dw"], M=qi["M"], upsample=args.upsample)
        # the operator's own error on this sub-problem, for context: K~ a vs K a
        ar = np.random.default_rng(1).standard_normal(sub.n)
        kex = O.exact_matvec(sub.x, sub.sigma, sub.l, sub.nu, ar)
        kt = Q64.matvec(torch.as_tensor(ar).to("cuda")).cpu().numpy()
        mv_err = float(np.linalg.norm(kt - kex) / np.linalg.norm(kex))
        a64, c64 = Q64.cg_solve(dev[3], tol=1e-6, max_iter=args.max_iter)
        a32, c32 = gp.cg_solve_refined(Q32, Q64, dev[3], tol=1e-6, inner_tol=args.inner_tol,
                                       max_iter=args.max_iter, max_refine=10)
        e = lambda a: float(np.linalg.norm(a.cpu().numpy() - ref) / np.linalg.norm(ref))
        out["oracle_subproblem"] = {
            "n": sub.n, "oracle": "exact K (eq:nonstat2), Cholesky of K + eta^2 I",
            "oracle_seconds": round(t_or, 2),
            "fp64_rel_err_vs_exact": e(a64), "fp32_bulk_refined_rel_err_vs_exact": e(a32),
            "fp64_iters": c64["iters"], "fp32_bulk_iters": c32["iters"],
            "plan_pred_tail": qi["pred_tail"], "M": qi["M"],
            "fp64_matvec_rel_err_vs_exact": mv_err,
            "note": "stated, not a parity bar: nu = 1/2 in d = 2 at l >= 0.02 with M capped at "
                    "2047 leaves K~ about pred_tail from K (matvec error above); eta^2 = 0.0025 "
                    "amplifies that operator error in the solution"}
        log(f"solve: sub-problem errors vs exact: fp64 {out['oracle_subproblem']['fp64_rel_err_vs_exact']:.2e}, "
            f"fp32-bulk {out['oracle_subproblem']['fp32_bulk_refined_rel_err_vs_exact']:.2e}")
        Q64.close()
        Q32.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
        return
    import torch

    from paper_2407_03608_amd import gp, inputs

    assert torch.cuda.is_available()
    dev = "cuda"
    if args.only == "matern_3d":
        out = matern_3d_leg(gp, torch, args, steps=args.steps, warmup=args.warmup)
        if args.calib_copy_mib:
            nb = args.calib_copy_mib * (1 << 20) // 8
            src = torch.ones(nb, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            out["calib_copy_bytes"] = nb * 8
        print(json.dumps(out), flush=True)
        return
    log("generating inputs")
    prob = inputs.matern_2d(n=args.n)
    X = torch.as_tensor(prob.x).to(dev)
    S = torch.as_tensor(prob.sigma).to(dev)
    Lx = torch.as_tensor(prob.l).to(dev)
    Y = torch.as_tensor(prob.y).to(dev)
    torch.cuda.synchronize()

    log("planning fp64")
    t0 = time.perf_counter()
    P64 = gp.Plan(X, S, Lx, prob.nu, prob.eta, args.tol64, upsample=args.upsample)
    torch.cuda.synchronize()
    plan64_s = time.perf_counter() - t0
    info64 = P64.info()
    log("plan64", {k: info64[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "na", "n_pairs",
                                           "pred_tail", "device_bytes")})
    log("planning fp32-bulk")
    t0 = time.perf_counter()
    P32 = gp.Plan(X, S, Lx, prob.nu, prob.eta, args.tol32, precision=gp.GP_FP32_BULK,
                  dw=info64["dw"], M=info64["M"], upsample=args.upsample)
    torch.cuda.synchronize()
    plan32_s = time.perf_counter() - t0
    info32 = P32.info()
    log("plan32", {k: info32[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "na", "n_pairs")})

    log("timing fp64 steps")
    t64, tm64 = time_path(gp, torch, P64, Y, args.steps, args.warmup)
    log("timing fp32 steps")
    t32, tm32 = time_path(gp, torch, P32, Y, args.steps, args.warmup)
    ms64 = 1e3 * t64 / args.steps
    ms32 = 1e3 * t32 / args.steps
    rf64 = roofline(info64, tm64, args.steps)
    rf32 = roofline(info32, tm32, args.steps)
    kernels64 = {k: round(v[1] / args.steps, 4) for k, v in tm64.items() if v[0]}
    kernels32 = {k: round(v[1] / args.steps, 4) for k, v in tm32.items() if v[0]}

    # agreement of the two paths on one matvec (stated, not asserted)
    a = torch.randn(prob.n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
    m64 = P64.matvec(a)
    m32 = P32.matvec(a)
    diff = float(torch.linalg.norm(m32 - m64) / torch.linalg.norm(m64))

    out = {
        "metric": "matvec points/s (CG iteration on (K~+eta^2 I)) at d=2 N=1e6, fp64 path",
        "value": round(prob.n * args.steps / t64, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform points, closed-form scales)",
        "config": {"workload": "matern_2d: d=2, N=1e6 uniform [0,1]^2, nu=1/2, "
                               "sigma=exp(0.3 x1), l=0.02+0.02 x2, eta=0.05, fp64, tol 1e-8",
                   "n": prob.n, "plan": {k: info64[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "upsample")}},
        "roofline": rf64,
        "matvec_model_roofline": step_model(info64, ms64),
        "kernels_ms": kernels64,
        "plan_seconds": round(plan64_s, 3),
        "fp32_bulk": {"value": round(prob.n * args.steps / t32, 1), "unit": "points/s",
                      "ms_per_step": round(ms32, 4), "roofline": rf32,
                      "matvec_model_roofline": step_model(info32, ms32), "kernels_ms": kernels32,
                      "plan": {k: info32[k] for k in ("n_sigma", "n_t", "dw", "M", "nf", "w", "upsample")},
                      "plan_seconds": round(plan32_s, 3),
                      "rel_diff_vs_fp64_matvec": diff},
    }

    if not args.no_solve:
        import oracle as O
        O.build()
        out["cg_solve"] = solve_legs(gp, torch, O, inputs, prob, P64, P32, Y, args)
    P64.close()
    P32.close()
    torch.cuda.empty_cache()

    if args.serve_requests > 0:
        out["serving"] = run_serving(args, args.serve_requests)

    if not args.no_extra:
        out["workloads"] = secondary_workloads(gp, torch, args)

    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)

    if args.calib_copy_mib:
        nb = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nb, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nb * 8

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
