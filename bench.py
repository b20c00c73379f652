"""Benchmark of the E-A-HALS outer iteration on one MI355X.

One step = one outer iteration of Algorithm 2 (both X-streaming products,
both HALS sweep blocks with their epilogues, the FP64 decision). The default
workload is the planted dense 16384 x 16384, r = 64 problem (X = W H +
1e-3 |N(0,1)|, seeded); X, W and H are resident in HBM before timing starts.

Prints one JSON line. `value` is outer iterations per second over the timed
graph launches. `roofline` covers the dominant kernel (the X-streaming
product; both products of an iteration are launches of that kernel): its
algorithmic bytes per launch over its mean duration, timed with HIP events
recorded around each launch on the stream the library launches it on, over
`--profile-iters` iterations run right after the timed ones. `eanls` times
E-ANLS (exact NNLS blocks) on the same workload, with the FP64 roofline of
its exact solves. `cpu_baseline`
times the FP64 oracle on a bounded sample of the same workload and scales it
by the iteration's flop count to the full size.

--copy-calib runs torch's plain device copy of 1 GiB a few times first: the
reference kernel for scaling the HBM byte counters (FETCH_SIZE, WRITE_SIZE)
of a profiler run.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E-A-HALS iters/s + HBM GB/s at 16384² r=64; batched solves/s, p99 latency"
HBM_PEAK_GBS = 8000.0
# Sources of the exact-integer product kernel (the dominant kernel of the
# default workload): the committed traffic figures apply while they are
# unchanged.
# Sources of the product kernel a workload's traffic summary was taken on:
# the exact-integer product (FP32 X) and the 16-bit X product.
PRODUCT_SOURCES = {"i8": ["paper_1805_06604_amd/csrc/prod_i8.h",
                          "paper_1805_06604_amd/csrc/prod_i8.hip"],
                   "x16": ["paper_1805_06604_amd/csrc/prod_x16.h",
                           "paper_1805_06604_amd/csrc/prod_x16.hip"]}
XBYTES = {"f32": 4, "bf16": 2, "f16": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--inner-k", type=int, default=10)
    ap.add_argument("--x-dtype", choices=list(XBYTES), default="f32")
    ap.add_argument("--prod", choices=["auto", "valu", "exact", "fast"], default="auto")
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="m = n of the oracle sample (0 disables the CPU baseline)")
    ap.add_argument("--cpu-serve-sample", type=int, default=16,
                    help="serving requests the oracle solves to the end (0: none)")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--cpu-full", type=int, default=1,
                    help="1: also time one oracle iteration on the full benchmark problem")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run the 1 GiB reference copy (counter calibration) first")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the batched-serving measurement (0 disables)")
    ap.add_argument("--serve-qps", type=float, default=2000.0,
                    help="Poisson arrival rate of the serving stream")
    ap.add_argument("--serve-seq", type=int, default=16,
                    help="requests of the same stream solved one at a time (baseline)")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-chunk", type=int, default=10,
                    help="batch iterations between completion checks")
    ap.add_argument("--serve-qps-low", type=float, default=100.0,
                    help="second arrival rate, below saturation (0: skip)")
    ap.add_argument("--x16", type=int, default=1,
                    help="1: time the same run with X stored in BF16 and in FP16")
    ap.add_argument("--workload-steps", type=int, default=50,
                    help="timed iterations on each of the other configurations (0: skip)")
    ap.add_argument("--workload-oracle", type=int, default=1,
                    help="1: also time the oracle on a few iterations of each")
    ap.add_argument("--k1-steps", type=int, default=50,
                    help="timed steps of the run with one inner sweep (0: skip)")
    ap.add_argument("--eanls-steps", type=int, default=20,
                    help="timed E-ANLS iterations on the same workload (0 disables)")
    ap.add_argument("--adaptive-steps", type=int, default=20,
                    help="timed E-A-HALS iterations with the adaptive inner loop (0 disables)")
    ap.add_argument("--adaptive-cap", type=int, default=20,
                    help="inner_k: upper bound on the adaptive loop's sweeps per side")
    return ap.parse_args()


def source_digest(kind="i8"):
    h = hashlib.sha256()
    for rel in PRODUCT_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key, kind="i8"):
    """HBM bytes per product launch from the committed counter summary, if it
    was taken on the current product kernel source for this workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload_key)
    if not rec or rec.get("source_sha") != source_digest(kind):
        return None
    return rec.get("bytes_per_launch")


def residual_fp64(X, W, H, block=1024):
    """||X - W H||_F / ||X||_F of the returned factors against the FP32 X,
    in FP64 on the host, a block of rows at a time."""
    W = np.asarray(W, np.float64)
    H = np.asarray(H, np.float64)
    num = den = 0.0
    for i in range(0, X.shape[0], block):
        Xb = X[i:i + block].astype(np.float64)
        R = Xb - W[i:i + block] @ H
        num += float(np.vdot(R, R))
        den += float(np.vdot(Xb, Xb))
    return float(np.sqrt(num / den))


def cpu_baseline(args, p_full):
    """The FP64 oracle as it stands (single thread), error by Remark 1 as on
    the GPU: one outer iteration of the full benchmark problem, timed as the
    difference of a solve with one iteration and a solve with none (which
    costs the set-up and e(0)); and a few iterations at the smaller sample
    size. The full-size figure is the value."""
    import nmf_synth as S
    import oracle
    kw = dict(hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5,
              inner_k=args.inner_k, flags=oracle.ERR_REMARK1)
    s = args.cpu_sample
    p = S.planted(0, m=s, n=s, r=args.r)
    t0 = time.perf_counter()
    oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=args.cpu_iters, **kw)
    t_small = time.perf_counter() - t0
    t_full = None
    if args.cpu_full and p_full is not None:
        q = p_full
        t0 = time.perf_counter()
        oracle.solve(q.X, q.r, q.W0, q.H0, max_iter=0, **kw)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.solve(q.X, q.r, q.W0, q.H0, max_iter=1, **kw)
        t_full = time.perf_counter() - t0 - t_setup
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    host = f"host {cpu}, os.cpu_count()={os.cpu_count()}, one thread"
    if t_full is not None:
        out = {"value": 1.0 / t_full, "unit": "iters/s", "cores": 1, "kind": "oracle",
               "sample": (f"FP64 oracle, error by Remark 1: one outer iteration of the planted "
                          f"{args.m}x{args.n}, r={args.r}, K={args.inner_k} workload took "
                          f"{t_full:.1f} s (a one-iteration solve minus the set-up and e(0) of a "
                          f"zero-iteration solve); {host}"),
               "seconds_per_iter_full": t_full}
    else:
        out = {"value": None, "unit": "iters/s", "cores": 1, "kind": "oracle",
               "sample": "full-size oracle iteration not run (--cpu-full 0)"}
    out["small_sample"] = {"workload": f"planted {s}x{s}, r={args.r}, K={args.inner_k}",
                           "iters": args.cpu_iters, "seconds": t_small,
                           "iters_per_s": args.cpu_iters / t_small}
    if args.workload_oracle and args.workload_steps > 0:
        # The oracle on the same problems as the workloads leg, a few iterations each.
        cfg = {}
        for name, make, iters in workload_specs(S):
            p = make()
            t0 = time.perf_counter()
            oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=iters, flags=oracle.ERR_REMARK1,
                         **WORKLOAD_PARAMS)
            t = time.perf_counter() - t0
            cfg[name] = {"iters_per_s": iters / t, "iters": iters, "seconds": t}
        out["workloads"] = cfg
    return out


def cpu_serving(args, probs):
    """The oracle (single thread, error by Remark 1) on a seeded random sample
    of the serving stream's requests, each solved to the end exactly as the
    batch solves it (<= 200 iterations or the tol rule)."""
    import oracle
    rng = np.random.default_rng(12345)
    idx = sorted(rng.choice(len(probs), size=min(args.cpu_serve_sample, len(probs)),
                            replace=False).tolist())
    t0 = time.perf_counter()
    iters = []
    for i in idx:
        p = probs[i]
        o = oracle.solve(p.X, p.r, p.W0, p.H0, max_iter=200, tol=1e-6, hp=3, beta0=0.5,
                         gamma=1.01, gamma_bar=1.005, eta=1.5, inner_k=args.inner_k,
                         flags=oracle.ERR_REMARK1)
        iters.append(o["n_iter"])
    t = time.perf_counter() - t0
    return {"solves_per_s": len(idx) / t, "requests": len(idx), "seconds": t,
            "mean_iters": float(np.mean(iters)),
            "mean_mn": float(np.mean([probs[i].X.shape[0] * probs[i].X.shape[1] for i in idx])),
            "sample": (f"{len(idx)} requests drawn at random (seed 12345) from the "
                       f"{len(probs)}-request stream, each solved to the end by the oracle")}


FP64_VECTOR_PEAK_TFS = 78.6


def nnls_flops(F, r):
    """Flops of the exact NNLS as the solve's usual route does it, per row
    with final support p (q = r - p coordinates held at zero): z = G^-1 c
    with the shared inverse (2 r^2), the q x q system of the held
    coordinates ((2/3) q^3) and the rank-q correction of z (2 r q). The
    inverse itself (2 r^3 once per side) and pivoting steps that end on
    another support are not counted."""
    p = np.count_nonzero(np.asarray(F) > 0, axis=1).astype(np.float64)
    q = r - p
    return float(np.sum(2.0 * r * r + (2.0 / 3.0) * q ** 3 + 2.0 * r * q))


def eanls(args, P, p, stream, torch):
    """E-ANLS (every block NNLS solved exactly, hp = 1 and the E-ANLS
    parameters of section 5.3.1) on the same resident workload."""
    m, n, r = args.m, args.n, args.r
    total = 5 + args.eanls_steps + args.profile_iters
    solver = P.Solver(p.X, r, hp=1, beta0=0.5, gamma=1.1, gamma_bar=1.05, eta=1.5,
                      inner_rule=P.Inner.EXACT, max_iter=total)
    solver.start(p.W0, p.H0, stream=stream)
    solver.iterate(5, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.iterate(args.eanls_steps, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.eanls_steps
    ph = solver.profile(args.profile_iters, stream=stream)
    res = solver.read(stream=stream)
    solver.close()
    # The exact-solve phases include the no-sweep epilogue launch after the
    # solve kernel; the flops are those of the usual route on the final
    # supports. The solve waits on chains of dependent LDS broadcasts and
    # FP64 divisions (pivoting steps), so it is latency-bound: the flop rate
    # is reported against the FP64 peak only for scale.
    solve_ms = ph["sweep_h"] + ph["sweep_w"]
    flops = nnls_flops(res.H.T, r) + nnls_flops(res.W, r)
    achieved = flops / (solve_ms * 1e-3) / 1e12
    return {"workload": f"planted dense {m}x{n} r={r}, E-ANLS hp=1 beta0=0.5 eta=1.5 gamma=1.1 "
                        f"gamma_bar=1.05", "value": 1e3 / ms, "unit": "iters/s", "ms_per_step": ms,
            "steps": args.eanls_steps, "phase_ms": ph, "rho_final": float(res.trace[-1]),
            "rho_fp64": residual_fp64(p.X, res.W, res.H),
            "roofline": {"bound": "latency", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFS,
                         "traffic": None, "kernel": "exact NNLS solve (both sides per iteration)",
                         "flops_per_iteration": flops, "ms_per_iteration": solve_ms}}


def device_cost_ratios(phases, K):
    """Cost ratios of the adaptive loop's caps measured on the device: 1 +
    the time of one side's X pass (slicing the fixed factor and the product)
    over that of one of its sweeps (the sweep kernel's time over its K
    sweeps, prologue and epilogue included), from the per-kernel times of
    the fixed-K headline run."""
    rho_h = 1.0 + (phases["slice_w"] + phases["prod_ct"]) / (phases["sweep_h"] / K)
    rho_w = 1.0 + (phases["slice_h"] + phases["prod_a"]) / (phases["sweep_w"] / K)
    return rho_h, rho_w


def adaptive(args, P, p, stream, torch, rho=None, steps=None):
    """E-A-HALS with the adaptive inner loop (cost-ratio cap bounded by
    --adaptive-cap, alpha 0.5, delta 0.1) on the same resident workload; the
    caps from the flop ratio, or from the cost ratios `rho` = (rho_H, rho_W)
    when given; `steps` timed iterations after 5 untimed ones."""
    steps = args.adaptive_steps if steps is None else steps
    total = 5 + steps
    extra = {} if rho is None else dict(inner_rho_h=rho[0], inner_rho_w=rho[1])
    solver = P.Solver(p.X, args.r, hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5,
                      inner_rule=P.Inner.ADAPTIVE, inner_k=args.adaptive_cap, max_iter=total,
                      **extra)
    solver.start(p.W0, p.H0, stream=stream)
    solver.iterate(5, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.iterate(steps, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    sw = solver.read_sweeps()
    res = solver.read(stream=stream)
    solver.close()
    timed = sw[5:]
    caps = "flop ratio" if rho is None else f"device cost ratios rho_H {rho[0]:.1f}, rho_W {rho[1]:.1f}"
    return {"workload": f"planted dense {args.m}x{args.n} r={args.r}, E-A-HALS hp=3 with the adaptive "
                        f"inner loop (alpha 0.5, delta 0.1, caps from the {caps}, at most "
                        f"{args.adaptive_cap} sweeps)",
            "value": 1e3 / ms, "unit": "iters/s", "ms_per_step": ms, "steps": steps,
            "mean_sweeps_h": float(timed[:, 0].mean()), "mean_sweeps_w": float(timed[:, 1].mean()),
            "iterations": int(res.n_iter), "rho_final": float(res.trace[-1]),
            "trace_timed": [float(x) for x in res.trace[5:]]}


def variant(args, P, S, p, stream, torch, x_dtype, prod, K, steps, label):
    """The headline run (same workload, parameters, warm-up and timing) with
    another X storage, product kernel or inner sweep count."""
    m, n, r = args.m, args.n, args.r
    total = args.warmup + steps + args.profile_iters
    xd = {"f32": P.XDtype.F32, "bf16": P.XDtype.BF16, "f16": P.XDtype.F16}[x_dtype]
    pm = {"auto": P.Prod.AUTO, "exact": P.Prod.MFMA_EXACT, "fast": P.Prod.MFMA_FAST}[prod]
    solver = P.Solver(p.X, r, hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5,
                      inner_k=K, max_iter=total, x_dtype=xd, prod=pm)
    W0, H0 = S.init_factors(m, n, r, 0)
    solver.start(W0, H0, stream=stream)
    solver.iterate(args.warmup, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.iterate(steps, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    ph = solver.profile(args.profile_iters, stream=stream)
    res = solver.read(stream=stream)
    solver.close()
    sx = XBYTES[x_dtype]
    nbytes = (m * n * sx + m * r * 4 + n * r * 8) + (m * n * sx + n * r * 4 + m * r * 8)
    achieved = nbytes / ((ph["prod_ct"] + ph["prod_a"]) * 1e-3) / 1e9
    return res, {
        "workload": label, "x_dtype": x_dtype, "prod": prod, "inner_k": K,
        "value": 1e3 / ms, "unit": "iters/s", "ms_per_step": ms, "steps": steps, "phase_ms": ph,
        "iterations": int(res.n_iter), "rho_final": float(res.trace[-1]),
        "rho_fp64": residual_fp64(p.X, res.W, res.H),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"planted_{m}x{n}_r{r}_{x_dtype}_{prod}",
                                                 "i8" if x_dtype == "f32" else "x16"),
                     "kernel": "X-streaming product", "bytes_per_launch": 0.5 * nbytes,
                     "ms_per_launch": 0.5 * (ph["prod_ct"] + ph["prod_a"])}}


def workloads(args, P, S, stream, torch):
    """The other configurations of the measurement plan, each as its own
    seeded synthetic stand-in (low-rank and full-rank synthetic sets, image-
    like dense, document-like CSR): GPU iterations/s with the effective bytes
    per second of the iteration (the oracle's rates on the same problems are
    in the cpu_baseline leg)."""
    kw = WORKLOAD_PARAMS
    out = {}
    for name, make, _ in workload_specs(S):
        p = make()
        steps, warm = args.workload_steps, 10
        with P.Solver(p.X, p.r, max_iter=warm + steps, **kw) as sv:
            sv.start(p.W0, p.H0, stream=stream)
            sv.iterate(warm, stream=stream)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sv.iterate(steps, stream=stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / steps
            res = sv.read(stream=stream)
        m, n, r = p.m, p.n, p.r
        if isinstance(p.X, S.Csr):
            # values and column indices of the CSR and CSC copies, and their row pointers
            xbytes = 2 * p.X.val.size * 8 + (m + n + 2) * 8
        else:
            xbytes = 2 * m * n * 4
        it_bytes = xbytes + 7 * (m + n) * r * 4
        out[name] = {"iters_per_s": 1e3 / ms, "ms_per_iter": ms, "steps": steps,
                     "effective_gbs": it_bytes / (ms * 1e-3) / 1e9,
                     "rho_final": float(res.trace[-1])}
    return out


# The other configurations: (name, generator, oracle iterations timed).
WORKLOAD_PARAMS = dict(hp=3, beta0=0.5, gamma=1.05, gamma_bar=1.01, eta=1.5, inner_k=10)


def workload_specs(S):
    return [("C1 low-rank synthetic 200x200 r=10", lambda: S.lowrank(0), 100),
            ("E2 full-rank synthetic 200x200 r=20", lambda: S.fullrank(0), 100),
            ("C2 image-like dense 10000x2000 r=49", lambda: S.imagelike(0), 5),
            ("C3 document-like CSR 30000x20000 r=20, nnz 1.8M", lambda: S.doclike(0), 10)]


def serving_problems(args, S):
    """The problems of the request stream (the same for every arrival rate:
    the stream draws sizes and seeds independently of the rate), generated
    on host threads."""
    from concurrent.futures import ThreadPoolExecutor
    reqs = S.requests(count=args.serve_requests, qps=1.0, seed=0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        probs = list(ex.map(S.request_problem, reqs))
    return probs, time.perf_counter() - t0


def serving(args, P, S, qps, n_seq, probs, t_gen):
    """Batched solves of a Poisson stream of small problems (m, n ~
    U{64..2048}, r in {5, 10, 20, 40}, X = max(0, W H + 1% noise)), each run
    to 200 iterations or |rho(k) - rho(k-1)| < 1e-6, replayed in real time:
    the main thread submits each request once its arrival time has passed,
    while a serving thread steps the batch and collects results; latency runs
    from arrival to the result on the host. The baseline solves the first
    requests of the same stream one at a time (one context each)."""
    import queue
    import threading
    reqs = S.requests(count=args.serve_requests, qps=qps, seed=0)
    assert all(q.seed == pr.seed and q.m == pr.X.shape[0] for q, pr in zip(reqs, probs))
    kw = dict(max_iter=200, tol=1e-6, hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5,
              inner_k=args.inner_k)
    lat = [None] * len(reqs)
    iters = []
    host = {"submit": 0.0, "step": 0.0, "result": 0.0}
    inbox = queue.Queue()
    with P.Batch(int(args.serve_budget_gb * (1 << 30)), max_active=512,
                 check_every=args.serve_chunk) as B:
        t0 = time.perf_counter()

        def serve():
            open_t = {}                       # request index -> ticket, oldest first
            finished = 0
            while finished < len(reqs):
                while True:
                    try:
                        i, t = inbox.get_nowait()
                    except queue.Empty:
                        break
                    open_t[i] = t
                h0 = time.perf_counter()
                a, q, d = B.step(args.serve_chunk)
                h1 = time.perf_counter()
                host["step"] += h1 - h0
                for i in list(open_t):
                    if d == 0:
                        break
                    g = B.result(open_t[i])
                    if g is not None:
                        lat[i] = time.perf_counter() - t0 - reqs[i].t_arrive
                        iters.append(g.n_iter)
                        del open_t[i]
                        finished += 1
                        d -= 1
                        if finished % 512 == 0:
                            print(f"serving at {qps:g} QPS: {finished} of {len(reqs)} results",
                                  file=sys.stderr, flush=True)
                host["result"] += time.perf_counter() - h1
                if finished < len(reqs) and a == 0 and q == 0 and not open_t:
                    i, t = inbox.get()        # idle until the next submission
                    open_t[i] = t

        th = threading.Thread(target=serve)
        th.start()
        for i, p in enumerate(probs[:len(reqs)]):
            wait = reqs[i].t_arrive - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            h0 = time.perf_counter()
            inbox.put((i, B.submit(p.X, p.r, p.W0, p.H0, **kw)))
            host["submit"] += time.perf_counter() - h0
        th.join()
        wall = time.perf_counter() - t0
    lat_ms = np.sort(np.asarray(lat) * 1e3)
    span = wall - reqs[0].t_arrive
    out = {
        "workload": (f"{len(reqs)} Poisson requests at {qps:g} QPS, m, n ~ U{{64..2048}}, "
                     f"r in {{5,10,20,40}}, <= 200 iterations or tol 1e-6"),
        "solves_per_s": len(reqs) / span, "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)), "max_ms": float(lat_ms[-1]),
        "mean_iters": float(np.mean(iters)), "generation_s": t_gen,
        "host_s": host,
    }
    n_seq = min(n_seq, len(reqs))
    if n_seq > 0:
        t1 = time.perf_counter()
        for p in probs[:n_seq]:
            with P.Solver(p.X, p.r, prod=P.Prod.MFMA_EXACT, **kw) as sv:
                sv.solve(p.W0, p.H0)
        seq = n_seq / (time.perf_counter() - t1)
        out.update({"sequential_solves_per_s": seq, "sequential_requests": n_seq,
                    "speedup_vs_sequential": len(reqs) / span / seq})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import nmf_synth as S
    import paper_1805_06604_amd as P

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    m, n, r, K = args.m, args.n, args.r, args.inner_k
    p = S.planted(0, m=m, n=n, r=r)
    total = args.warmup + args.steps + args.profile_iters
    xd = {"f32": P.XDtype.F32, "bf16": P.XDtype.BF16, "f16": P.XDtype.F16}[args.x_dtype]
    pm = {"auto": P.Prod.AUTO, "valu": P.Prod.VALU, "exact": P.Prod.MFMA_EXACT,
          "fast": P.Prod.MFMA_FAST}[args.prod]
    ea = eanls(args, P, p, stream, torch) if args.eanls_steps > 0 else None
    ad = adaptive(args, P, p, stream, torch) if args.adaptive_steps > 0 else None
    solver = P.Solver(p.X, r, hp=3, beta0=0.5, gamma=1.01, gamma_bar=1.005, eta=1.5,
                      inner_k=K, max_iter=total, x_dtype=xd, prod=pm)
    W0, H0 = S.init_factors(m, n, r, 0)
    solver.start(W0, H0, stream=stream)
    solver.iterate(args.warmup, stream=stream)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    solver.iterate(args.steps, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps

    phases = solver.profile(args.profile_iters, stream=stream)
    res = solver.read(stream=stream)
    solver.close()

    sx = XBYTES[args.x_dtype]
    # Algorithmic bytes of one product launch: X once, the factor once, the
    # FP64 result once (C^T = X^T W_y: n rows; A = X H_w^T: m rows).
    bytes_ct = m * n * sx + m * r * 4 + n * r * 8
    bytes_a = m * n * sx + n * r * 4 + m * r * 8
    prod_ms = 0.5 * (phases["prod_ct"] + phases["prod_a"])
    achieved = (bytes_ct + bytes_a) / ((phases["prod_ct"] + phases["prod_a"]) * 1e-3) / 1e9
    iter_bytes = 2 * m * n * sx + 7 * (m + n) * r * 4
    key = f"planted_{m}x{n}_r{r}_{args.x_dtype}_{args.prod}"
    traffic = measured_traffic(key, "i8" if args.x_dtype == "f32" else "x16")
    out = {
        "metric": METRIC,
        "value": args.steps / (ms * 1e-3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16", "f16": "f16"}[args.x_dtype],
        "data": "synthetic",
        "config": {"workload": f"planted dense {m}x{n} r={r}, X = WH + 1e-3|N(0,1)| (seed 0)",
                   "m": m, "n": n, "r": r, "x_dtype": args.x_dtype, "prod": args.prod,
                   "inner_k": K, "hp": 3, "beta0": 0.5, "gamma": 1.01, "gamma_bar": 1.005,
                   "eta": 1.5},
        "hbm_gbs": iter_bytes * args.steps / (ms * 1e-3) / 1e9,
        "phase_ms": phases,
        "iterations": int(res.n_iter),
        "rho_final": float(res.trace[-1]),
        "rho_fp64": residual_fp64(p.X, res.W, res.H),
        "accepted": int(res.accepted.sum()),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "X-streaming product",
                     "bytes_per_launch": 0.5 * (bytes_ct + bytes_a), "ms_per_launch": prod_ms},
    }
    # The same run (same iterations) with X stored in 16 bits (BF16
    # matrix-core products): its final error against the FP32 X, in FP64,
    # set against the FP32 run's; and with one inner sweep per block.
    if args.x16 and args.x_dtype == "f32":
        for xd16 in ("bf16", "f16"):
            r16, v = variant(args, P, S, p, stream, torch, xd16, "fast", K, args.steps,
                             f"planted dense {m}x{n} r={r}, X stored as {xd16}, K={K}")
            v["rho_fp64_f32_run"] = out["rho_fp64"]
            v["abs_rho_fp64_gap_vs_f32"] = abs(v["rho_fp64"] - out["rho_fp64"])
            out[f"x_{xd16}"] = v
    if args.k1_steps > 0:
        _, v = variant(args, P, S, p, stream, torch, args.x_dtype, args.prod, 1, args.k1_steps,
                       f"planted dense {m}x{n} r={r}, one inner sweep per block (K=1)")
        out["inner_k1"] = v
    # The adaptive loop again with its caps from the cost ratios of this
    # device, measured in the fixed-K run above.
    ad_dev = None
    if ad is not None:
        ad_dev = adaptive(args, P, p, stream, torch, device_cost_ratios(phases, K),
                          steps=2 * args.adaptive_steps)
        # Its error after the time the flop-ratio caps took for their timed
        # iterations (iteration times are uniform within a run).
        j = min(int(args.adaptive_steps * ad["ms_per_step"] / ad_dev["ms_per_step"]),
                len(ad_dev["trace_timed"]) - 1)
        ad_dev["rho_at_equal_time"] = ad_dev.pop("trace_timed")[j]
        ad["rho_at_equal_time"] = ad.pop("trace_timed")[-1]
    cpu = cpu_baseline(args, p) if args.cpu_sample > 0 else None
    del p
    if ea is not None:
        out["eanls"] = ea
    if ad is not None:
        out["adaptive_inner"] = ad
        out["adaptive_inner_device_cost"] = ad_dev
    if args.workload_steps > 0:
        out["workloads"] = workloads(args, P, S, stream, torch)
    if args.serve_requests > 0:
        probs, t_gen = serving_problems(args, S)
        out["serving"] = serving(args, P, S, args.serve_qps, args.serve_seq, probs, t_gen)
        if args.serve_qps_low > 0:
            out["serving_below_saturation"] = serving(args, P, S, args.serve_qps_low, 0, probs,
                                                      t_gen)
        if cpu is not None and args.cpu_serve_sample > 0:
            cpu["serving"] = cpu_serving(args, probs)
        del probs
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
