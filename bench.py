"""Benchmark: HIF-preconditioned Crank-Nicolson steps per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload heat2d-1024] [--store f32]

One timed "step" is one Crank-Nicolson step of the whole hot path: the right-hand side
(I + dt/2 M) u + dt r(u), then PCG to rtol 1e-8 with the HIF preconditioner (every CG
iteration: fused direction update + SpMV, vector update, HIF apply, r.z).  The factor is
built once before timing (its time is reported as t_factor_s).  Inputs are synthetic and
resident in HBM before the timed region.  The headline is the 1024^2 heat workload (N = 1M,
per-cell coefficient 10^U(-2,2), dt = 0.1, eps = 1e-3) with FP32 factor storage; the FP64 and
BF16 stores, the 256^2 Fisher-KPP and 64^3 heat workloads and the serving workload are reported
beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix, published
STAGES = ["cell_fwd", "group_fwd", "root", "group_bwd", "cell_bwd"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "cell_stage_level0_pmc.json")
APPLY_SRC = os.path.join(ROOT, "paper_2004_05566_amd", "csrc", "apply.hip")


def _log(msg: str):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


def _time_cn(h, u0, steps, warmup, rtol, reaction, maxit=500, warm=False):
    import torch
    u = u0.clone()
    if warmup:
        h.cn_solve(u, warmup, rtol=rtol, maxit=maxit, reaction=reaction, warm_start=warm)
    _sync()
    t0 = time.perf_counter()
    its, rel = h.cn_solve(u, steps, rtol=rtol, maxit=maxit, reaction=reaction, warm_start=warm)
    _sync()
    dt = time.perf_counter() - t0
    return dt, its, rel, u


def _time_op(fn, reps):
    import torch
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        fn()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def _time_replays(fn, reps=100, per=10):
    """Per-call duration of `fn`: the median over `reps` replays of a HIP graph holding `per`
    calls of it, each replay bracketed by HIP events on the replay stream, divided by `per` (the
    graph's own launch cost, ~15 us here, is spread over the calls it holds); per-call events on
    the current stream if the call cannot be captured.  Returns (seconds, how)."""
    import statistics

    import torch
    cur = torch.cuda.current_stream()
    how = "median of %d hipGraph replays of %d calls, per call" % (reps, per)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            for _ in range(3):
                fn()
        cur.wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(per):
                fn()
        run = g.replay
    except Exception:  # noqa: BLE001 - fall back to plain launches
        torch.cuda.synchronize()
        per = 1
        run, how = fn, "median of %d calls" % reps
        for _ in range(3):
            fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        run()
        e1.record()
    torch.cuda.synchronize()
    return statistics.median(e0.elapsed_time(e1) for e0, e1 in ev) / 1e3 / per, how


def method_apply_bytes(factor_bytes: int, N: int, dim: int) -> int:
    """Bytes one F^-1 application must move by the method's count: every stored factor block
    read once per sweep (2 F_b) plus the FP64 input and output and the level-0 working vector
    (32 N in 2D; 40 N in 3D, whose level-0 cells exchange more boundary values)."""
    return 2 * factor_bytes + (32 if dim == 2 else 40) * N


def spmv_bytes(N: int, dim: int) -> int:
    """x and y (FP64) and one link array per axis: 8 (2 + dim) bytes per DOF."""
    return (8 + 8 + 8 * dim) * N


def _build_mfma(info: dict) -> dict:
    """The factor build's matrix-core work (large cells and root): algorithmic FP64 flops over the
    summed duration of those kernels, against the FP64 matrix peak."""
    fl, ms = info["build_mfma_flops"], info["build_mfma_ms"]
    tf = fl / (ms * 1e9) if ms > 0 else None
    return {"flops": fl, "ms": ms, "TFLOP/s": tf, "peak": FP64_MFMA_PEAK_TFLOPS,
            "frac": tf / FP64_MFMA_PEAK_TFLOPS if tf else None}


def _src_sha() -> str:
    import hashlib
    return hashlib.sha256(open(APPLY_SRC, "rb").read()).hexdigest()[:16]


def pmc_traffic(kernel: str, store: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, scaled by
    the counters of a plain copy of known size; None if absent or if the kernel source changed
    since the counters were taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    d = json.load(open(PMC_SUMMARY))
    if d.get("apply_src_sha") != _src_sha():
        return None
    k = d.get("kernels", {}).get(f"{workload}/{store}/{kernel}")
    if not k:
        return None
    return (k["fetch_kib"] * 1024 * d["copy_scale_fetch"]
            + k["write_kib"] * 1024 * d["copy_scale_write"])


def stage_breakdown(h, x, y, levels, reps=20):
    """HIP-event time and algorithmic bytes of every apply stage (apply loop, no early exits)."""
    out = []
    for lev in range(levels + 1):
        for st in STAGES:
            if (st == "root") != (lev == levels):
                continue
            h.profile_stage(lev, st, True)
            for _ in range(reps):
                h.apply(x, out=y)
            p = h.profile_read()
            h.profile_stage(lev, st, False)
            if p["launches"]:
                us = 1e3 * p["ms"] / p["launches"]
                out.append({"level": lev, "stage": st, "us": us, "bytes": p["bytes"],
                            "GB/s": p["bytes"] / us / 1e3})
    return out


def copy_probe(nbytes: int):
    """A plain device copy of known size (calibrates the HBM byte counters)."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes}))


def serving_bench(count: int, rate: float, max_slots: int, budget_bytes: int,
                  builders: int = 8, seed_base: int = 5000, lanes: int = 1) -> dict:
    """The serving workload: `count` independent 2D Fisher-KPP solves of mixed size, dt and
    coefficient (50 CN steps each), arriving as a Poisson process of `rate` requests/s (rate 0:
    all at once), served by continuous batching.  Inputs are drawn before the clock starts."""
    import numpy as np

    from paper_2004_05566_amd.serve import Request, Server, percentiles
    from workloads import gen

    def req(w):
        return Request(w.n, w.a_cells, w.u0, w.dt, w.steps, eps=w.eps, reaction=w.reaction,
                       rtol=w.rtol, store="f32", tag=w.name)

    reqs = [req(gen.serving_request(i, seed_base)) for i in range(count)]
    # first-use costs (kernel loading, LDS attributes) outside the clock: one of each size
    warm = Server(budget_bytes, max_slots, builders, lanes=lanes)
    for f in [warm.submit(req(gen.serving_request(10_000 + i, seed_base, sizes=(n,))))
              for i, n in enumerate((64, 128, 256, 512))]:
        f.result()
    warm.close()
    arrivals = (gen.poisson_arrivals(count, rate, seed_base + 7) if rate > 0
                else np.zeros(count))
    srv = Server(budget_bytes, max_slots, builders, lanes=lanes)
    finished = [0]

    def progress(_f):
        finished[0] += 1
        if finished[0] % 32 == 0:
            print(f"serving: {finished[0]}/{count} done", file=sys.stderr, flush=True)

    t0 = time.perf_counter() + 0.01
    futs = []
    for r, ta in zip(reqs, arrivals):
        delay = t0 + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(srv.submit(r, t_arrival=t0 + ta))
        futs[-1].add_done_callback(progress)
    res = [f.result() for f in futs]
    srv.close()
    t_end = max(r.t_done for r in res)
    lat = [r.latency for r in res]
    steps = sum(len(r.iters) for r in res)
    st = srv.stats()
    out = {"requests": count, "arrival_rate_per_s": rate or None,
           "arrivals": "poisson" if rate > 0 else "all at t=0",
           **{k + "_latency_s": v for k, v in percentiles(lat).items()},
           "mean_latency_s": float(np.mean(lat)),
           "makespan_s": t_end - t0, "requests_per_s": count / (t_end - t0),
           "cn_steps_per_s": steps / (t_end - t0),
           "mean_build_s": float(np.mean([r.t_ready - r.t_admit for r in res])),
           "mean_queue_s": float(np.mean([r.t_admit - r.t_arrival for r in res])),
           "n_i_mean": float(np.mean(np.concatenate([r.iters for r in res]))),
           "sizes": sorted({int(r.u.shape[0]) for r in res}), "builders": builders,
           "lanes": lanes,
           **st}
    return out


def cpu_baseline(w, budget_steps: int, rtol: float = 1e-8):
    """The FP64 oracle on the same workload: its factor build (reported, not in the value), then
    `budget_steps` CN steps with BLAS threads = the host's cores, and the same steps again on
    one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cn, fd, phif
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    A, B = fd.cn_matrices(w.a_cells, w.dt)
    _log(f"cpu baseline: oracle build of {w.name}")
    with threadpool_limits(limits=nproc):
        t0 = time.perf_counter()
        F = phif.phif_build(A, w.n, w.dim, w.leaf, w.eps)
        tf = time.perf_counter() - t0
    times, its = {}, []
    for threads in (nproc, 1):
        _log(f"cpu baseline: {budget_steps} step(s) on {threads} thread(s)")
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            _, its, _ = cn.cn_solve(A, B, w.u0, w.dt, budget_steps,
                                    lambda r: phif.phif_apply(F, r), rtol, w.reaction,
                                    maxit=w.maxit, warm_start=w.x0 == "previous")
            times[threads] = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": budget_steps / times[nproc], "unit": "CN steps/s", "cores": nproc,
            "kind": "oracle",
            "sample": f"{w.name}: oracle PHIF build ({tf:.1f} s, not in the value) then the first "
                      f"{budget_steps} CN step(s) at rtol {rtol:g}, n_i {list(its)}, BLAS "
                      f"threads = {nproc}",
            "one_thread": {"value": budget_steps / times[1], "cores": 1},
            "t_factor_s": tf, "host_cpu": model, "host_nproc": os.cpu_count()}


def replica(sizes2d, sizes3d, steps, store, logistic=False):
    """The paper's Sec. 3 experiments at the given sizes (eps 1e-3 and 1e-6): mean n_i at rtol
    1e-12, build and per-step time, factor bytes, and at eps 1e-6 the estimate of
    ||I - A F^-1|| and the same steps solved by the factor alone (time per step, relative
    distance to the CG result), next to the values the paper prints."""
    import json as _json

    import numpy as np
    import torch

    from paper_2004_05566_amd import hifcn
    from workloads import gen
    gold = _json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                                        "golden", "paper_phif_iterations.json")))
    kind = "logistic" if logistic else "heat"
    out = []
    for dim, sizes in ((2, sizes2d), (3, sizes3d)):
        for n in sizes:
            for eps in (1e-3, 1e-6):
                w = gen.paper_heat(n, dim, eps, steps=steps, logistic=logistic)
                a_dev = torch.tensor(w.a_cells, dtype=torch.float64, device="cuda")
                u = torch.tensor(w.u0.ravel(), dtype=torch.float64, device="cuda")
                _sync()
                t0 = time.perf_counter()
                h = hifcn.factor(a_dev, w.dt, n, dim, eps, store=store, leaf=w.leaf)
                _sync()
                tf = time.perf_counter() - t0
                t0 = time.perf_counter()
                its, _ = h.cn_solve(u, steps, rtol=w.rtol, reaction=w.reaction)
                _sync()
                ts = (time.perf_counter() - t0) / steps
                paper = gold.get(f"{kind}_{dim}d", {}).get(f"eps_{eps:.0e}".replace("e-0", "e-"),
                                                          {}).get(str(n))
                row = {"case": w.name, "N": w.N, "steps": steps, "store": store,
                       "n_i_mean": float(np.mean(its)), "n_i_paper": paper,
                       "t_factor_s": tf, "t_step_s": ts, "factor_GB": h.factor_bytes() / 1e9}
                if eps == 1e-6:
                    row["inv_error"] = h.inverse_error(
                        torch.tensor(gen.normal_vector(w.N, 0), device="cuda"), 30)
                    # the same steps with the factor as the solver (no CG)
                    ud = torch.tensor(w.u0.ravel(), dtype=torch.float64, device="cuda")
                    h.cn_solve_direct(ud, 1, reaction=w.reaction)
                    ud.copy_(torch.tensor(w.u0.ravel(), dtype=torch.float64, device="cuda"))
                    _sync()
                    t0 = time.perf_counter()
                    h.cn_solve_direct(ud, steps, reaction=w.reaction)
                    _sync()
                    row["t_step_direct_s"] = (time.perf_counter() - t0) / steps
                    row["direct_vs_cg"] = float(torch.linalg.norm(ud - u) / torch.linalg.norm(u))
                    del ud
                h.close()
                del a_dev, u
                print(_json.dumps(row), flush=True)
                out.append(row)
    return out


def drift(w, steps, everies, store, amp=0.5):
    """A coefficient that drifts over the run (a(x, t) = a0(x) exp(amp sin(2 pi t / T) b(x)),
    T = steps dt; step k takes a(., (k + 1/2) dt)), with the factor rebuilt every K steps and the
    operator updated in between (K = 0: never rebuilt).  The coefficients are on the device
    before the clock starts; the rebuilds are inside the timed region."""
    import numpy as np
    import torch

    from paper_2004_05566_amd import hifcn
    from workloads import gen
    a_at = gen.drifting_coefficient(w.n, w.dim, 0.1, 2001, amp=amp, period=steps * w.dt)
    coeffs = [torch.tensor(a_at((k + 0.5) * w.dt), dtype=torch.float64, device="cuda")
              for k in range(steps)]
    out = []
    for every in everies:
        h = hifcn.factor(coeffs[0], w.dt, w.n, w.dim, w.eps, store=store, leaf=w.leaf)
        u = torch.tensor(w.u0.ravel(), dtype=torch.float64, device="cuda")
        its, t_re = [], 0.0
        _sync()
        t0 = time.perf_counter()
        for k in range(steps):
            if k and every and k % every == 0:
                t1 = time.perf_counter()
                h.refactor(coeffs[k])
                t_re += time.perf_counter() - t1
            elif k:
                h.set_coefficient(coeffs[k])
            it, _ = h.cn_solve(u, 1, rtol=w.rtol, reaction=w.reaction)
            its.append(int(it[0]))
        _sync()
        tt = time.perf_counter() - t0
        nre = (steps - 1) // every if every else 0
        row = {"case": w.name, "drift_amp": amp, "refactor_every": every, "steps": steps,
               "store": store, "steps_per_s": steps / tt, "t_total_s": tt,
               "refactors": nre, "t_refactor_s": t_re / nre if nre else None,
               "n_i_mean": float(np.mean(its)), "n_i_max": int(max(its))}
        print(json.dumps(row), flush=True)
        out.append(row)
        h.close()
    return out


def apply_loop(name: str, store: str, reps: int):
    """The factor of a workload, then `reps` applies to one vector (counter runs)."""
    import torch
    from paper_2004_05566_amd import hifcn
    from workloads import gen
    w = gen.workload(name)
    h = hifcn.factor(torch.tensor(w.a_cells, device="cuda"), w.dt, w.n, w.dim, w.eps,
                     store=store, leaf=w.leaf)
    x = torch.tensor(gen.normal_vector(w.N, 1), device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        h.apply(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"apply_loop": name, "store": store, "applies": reps}), flush=True)
    h.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="heat2d-1024",
                    help="a committed workload (workloads/configs/<name>.json) or a config path")
    ap.add_argument("--store", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--leaf", type=int, default=0, help="leaf box size (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the error check")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage breakdown")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the 256^2 and 64^3 workloads reported beside the headline")
    ap.add_argument("--cpu-steps", type=int, default=1,
                    help="CN steps of the oracle in the CPU baseline sample")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving workload (0: skip)")
    ap.add_argument("--serving-rate", type=float, default=-1.0,
                    help="Poisson arrival rate of serving requests per second; -1: 0.7 x the "
                         "saturated throughput measured first; 0: only the saturated run")
    ap.add_argument("--serving-slots", type=int, default=32)
    ap.add_argument("--serving-builders", type=int, default=8,
                    help="threads (each with its own stream) building factors concurrently")
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--serving-lanes", type=int, default=1,
                    help="scheduler lanes (each runs its own batch of solves of similar size)")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration)")
    ap.add_argument("--apply-loop", type=int, default=0,
                    help="only build the workload's factor and run this many applies (plain "
                         "launches on one stream, for hardware-counter runs)")
    ap.add_argument("--replica", default="",
                    help="only run the paper's Sec. 3 experiments, e.g. '2d:511,1023;3d:63' "
                         "(one JSON line per case; --steps steps each, --store storage)")
    ap.add_argument("--logistic", action="store_true",
                    help="with --replica: the logistic reaction (Example 2)")
    ap.add_argument("--drift", default="",
                    help="only run the workload with a drifting coefficient, the factor rebuilt "
                         "every K steps for each K listed, e.g. '1,5,20,0' (0: never)")
    args = ap.parse_args(argv)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return 0
    if args.apply_loop:
        apply_loop(args.workload, args.store, args.apply_loop)
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "hifcn runs on one GPU; --gpus must be 1"}))
        return 2
    if args.drift:
        from workloads import gen
        w = gen.workload(args.workload)
        drift(w, args.steps, [int(s) for s in args.drift.split(",")], args.store)
        return 0
    if args.replica:
        sz = {"2d": [], "3d": []}
        for part in args.replica.split(";"):
            k, v = part.split(":")
            sz[k.strip()] = [int(s) for s in v.split(",") if s.strip()]
        replica(sz["2d"], sz["3d"], args.steps, args.store, args.logistic)
        return 0

    from paper_2004_05566_amd import hifcn  # noqa: F401  (fails loudly without the library)
    from workloads import gen

    def serving():
        """Saturated run (all requests at t = 0) to measure the throughput mu, then Poisson
        arrivals at the stated rate (default 0.7 mu)."""
        budget = int(args.serving_budget_gb * (1 << 30))
        sat = serving_bench(args.serving, 0.0, args.serving_slots, budget, args.serving_builders,
                            lanes=args.serving_lanes)
        out = {"saturated": sat}
        rate = args.serving_rate
        if rate < 0:
            rate = round(0.7 * sat["requests_per_s"], 1)
            out["rate_rule"] = "0.7 x saturated requests/s"
        if rate > 0:
            out["poisson"] = serving_bench(args.serving, rate, args.serving_slots, budget,
                                           args.serving_builders, lanes=args.serving_lanes)
        return out

    if args.serving_only:
        print(json.dumps({"serving": serving()}))
        return 0

    w = gen.workload(args.workload)
    if args.leaf:
        w.leaf = args.leaf
    head = measure(w, args.store, args.steps, args.warmup, args.rtol, roofline=True,
                   stages=not args.no_stages, check=not args.no_check)
    side = {}
    for st in ("f64", "bf16"):
        if st != args.store:
            side[st] = measure(w, st, args.steps, args.warmup, args.rtol,
                               check=not args.no_check)
    others = {}
    if not args.no_others:
        for name in ("fisher2d-256", "heat3d-64"):
            if name == w.name:
                continue
            wo = gen.workload(name)
            others[name] = {st: measure(wo, st, args.steps, args.warmup, args.rtol,
                                        check=not args.no_check)
                            for st in ("f32", "f64")}
    roof = head.pop("roofline")
    out = {
        "metric": "CN steps/s at 1e-8 rel. resid (FP32-HIF vs FP64), HIF-apply GB/s; p99 latency",
        "value": head["value"],
        "unit": "CN steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f64 CG / f32 HIF storage", "bf16": "f64 CG / bf16 HIF storage",
                  "f64": "f64"}[args.store],
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "dim": w.dim, "n": w.n, "eps": w.eps,
                   "dt": w.dt, "leaf": w.leaf, "store": args.store, "rtol": args.rtol,
                   "maxit": w.maxit, "x0": w.x0, "reaction": list(w.reaction)},
        **head,
        "roofline": roof,
        "f64_store": side.get("f64"),
        "bf16_store": side.get("bf16"),
        "other_workloads": others,
    }
    if args.serving:
        out["serving"] = serving()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))
    return 0


def oracle_error(w, h, store, rtol):
    """Error of two GPU CN steps at `rtol` from u0 against the oracle's (FP64 block PHIF, PCG at
    rtol 1e-12) at the sampled nodes of the committed expected values (tests/golden/
    fullsize_*.npz, written by tests/golden/make_fullsize.py from the oracle alone); None for a
    workload without them."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{w.name}.npz")
    u = torch.tensor(w.u0.ravel(), dtype=torch.float64, device="cuda")
    if os.path.exists(path):
        g = np.load(path)
        out = {"against": "oracle PHIF-PCG at rtol 1e-12, sampled nodes", "steps": []}
        for k in range(1, int(g["steps"]) + 1):
            h.cn_solve(u, 1, rtol=rtol, reaction=w.reaction)
            ug = u.cpu().numpy()
            out["steps"].append({
                "max_rel": float(np.abs(ug[g["idx"]] - g[f"u{k}"]).max() / g[f"amax{k}"]),
                "norm_rel": float(abs(np.linalg.norm(ug) - g[f"norm{k}"]) / g[f"norm{k}"])})
        out["max_rel"] = max(x["max_rel"] for x in out["steps"])
        return out
    return None


def measure(w, store, steps, warmup, rtol, roofline=False, stages=False, check=True):
    """Build the factor of workload w in `store` precision, time `steps` CN steps (after
    `warmup`), the apply and the SpMV; optionally the dominant kernel's roofline, the per-stage
    breakdown and the error against the oracle."""
    import numpy as np
    import torch

    from paper_2004_05566_amd import hifcn
    _log(f"measure {w.name} store {store}")
    dev = torch.device("cuda:0")
    a_dev = torch.tensor(w.a_cells, dtype=torch.float64, device=dev)
    u0 = torch.tensor(w.u0.ravel(), dtype=torch.float64, device=dev)
    _sync()
    t0 = time.perf_counter()
    h = hifcn.factor(a_dev, w.dt, w.n, w.dim, w.eps, store=store, leaf=w.leaf)
    _sync()
    t_factor = time.perf_counter() - t0
    elapsed, its, rel, u = _time_cn(h, u0, steps, warmup, rtol, w.reaction, w.maxit,
                                    w.x0 == "previous")
    info = h.info()
    fb = h.factor_bytes()
    x = torch.randn(w.N, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    t_apply, how = _time_replays(lambda: h.apply(x, out=y))
    t_spmv, _ = _time_replays(lambda: h.spmv(x, out=y))
    mb = method_apply_bytes(fb, w.N, w.dim)
    sb = spmv_bytes(w.N, w.dim)
    res = {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "n_i_mean": float(np.mean(its)),
        "n_i": [int(i) for i in its],
        "t_factor_s": t_factor,
        "factor_bytes": fb,
        "device_bytes": info["device_bytes"],
        "build_mfma": _build_mfma(info),
        "apply": {"us": t_apply * 1e6, "GB/s": mb / t_apply / 1e9,
                  "frac_of_peak": mb / t_apply / 1e9 / HBM_PEAK_GBS, "method_bytes": mb,
                  "read_bytes": info["apply_bytes"],
                  "read_amplification": info["apply_bytes"] / mb, "timing": how},
        "spmv": {"us": t_spmv * 1e6, "GB/s": sb / t_spmv / 1e9,
                 "frac_of_peak": sb / t_spmv / 1e9 / HBM_PEAK_GBS, "bytes": sb, "timing": how},
    }
    if stages:
        res["apply_stages"] = stage_breakdown(h, x, y, info["levels"])
    if roofline:
        res["roofline"] = dominant_roofline(h, w, store, u0, steps, rtol, res.get("apply_stages"))
    if check:
        res["err_vs_oracle"] = oracle_error(w, h, store, rtol)
    h.close()
    del a_dev, u0, u, x, y
    torch.cuda.empty_cache()
    return res


def dominant_roofline(h, w, store, u0, steps, rtol, stages):
    """The apply stage that takes the most time per apply, timed live with HIP events on the
    stream it runs on over a second pass of the timed CN steps: algorithmic bytes per launch
    over the average launch duration, against the HBM peak."""
    cands = [("cell_fwd", 0), ("cell_bwd", 0)]
    if stages:
        top = max(stages, key=lambda r: r["us"])
        cands = [(top["stage"], top["level"])] + [c for c in cands
                                                  if c != (top["stage"], top["level"])]
    roof = {}
    for st, lev in cands:
        h.profile_stage(lev, st, True)
        _time_cn(h, u0, steps, 0, rtol, w.reaction, w.maxit, w.x0 == "previous")
        p = h.profile_read()
        h.profile_stage(lev, st, False)
        roof[(st, lev)] = p
    key = max(roof, key=lambda k: roof[k]["ms"])
    pd = roof[key]
    avg_s = pd["ms"] / 1e3 / max(1, pd["launches"])
    achieved = pd["bytes"] / avg_s / 1e9
    kname = pd.get("kernel") or {"cell_fwd": "k_cell_fwd", "cell_bwd": "k_cell_bwd",
                                 "group_fwd": "k_fuse_fwd", "group_bwd": "k_group_bwd",
                                 "root": "k_top_rows"}[key[0]]
    return {"bound": "hbm", "kernel": f"{kname} (level {key[1]}, {key[0]})",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": pmc_traffic(kname, store, w.name), "bytes_per_launch": pd["bytes"],
            "avg_us": avg_s * 1e6, "launches": pd["launches"],
            "stage_us": {f"{k[0]}@{k[1]}": 1e3 * v["ms"] / max(1, v["launches"])
                         for k, v in roof.items()}}


if __name__ == "__main__":
    sys.exit(main())
