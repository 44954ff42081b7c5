"""Benchmark: HIF-preconditioned Crank-Nicolson steps per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload fisher2d-256] [--store f32]

One timed "step" is one Crank-Nicolson step of the whole hot path: the right-hand side
(I + dt/2 M) u + dt r(u), then PCG to rtol 1e-8 with the HIF preconditioner (every CG
iteration: fused direction update + SpMV, vector update, HIF apply, r.z).  The factor is
built once before timing (its time is reported as t_factor_s).  Inputs are synthetic and
resident in HBM before the timed region.  Prints one JSON line.
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


def _sync():
    import torch
    torch.cuda.synchronize()


def _time_cn(h, u0, steps, warmup, rtol, reaction):
    import torch
    u = u0.clone()
    if warmup:
        h.cn_solve(u, warmup, rtol=rtol, reaction=reaction)
    _sync()
    t0 = time.perf_counter()
    its, rel = h.cn_solve(u, steps, rtol=rtol, reaction=reaction)
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
                  builders: int = 8, seed_base: int = 5000) -> dict:
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
    warm = Server(budget_bytes, max_slots, builders)
    for f in [warm.submit(req(gen.serving_request(10_000 + i, seed_base, sizes=(n,))))
              for i, n in enumerate((64, 128, 256, 512))]:
        f.result()
    warm.close()
    arrivals = (gen.poisson_arrivals(count, rate, seed_base + 7) if rate > 0
                else np.zeros(count))
    srv = Server(budget_bytes, max_slots, builders)
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
           **st}
    return out


def cpu_baseline(w, budget_steps: int):
    """The FP64 oracle on the same workload: factor build, then `budget_steps` CN steps."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cn, fd, phif
    with threadpool_limits(limits=1):
        A, B = fd.cn_matrices(w.a_cells, w.dt)
        t0 = time.perf_counter()
        F = phif.phif_build(A, w.n, w.dim, w.leaf, w.eps)
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, its, _ = cn.cn_solve(A, B, w.u0, w.dt, budget_steps,
                                lambda r: phif.phif_apply(F, r), 1e-8, w.reaction)
        ts = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": budget_steps / ts, "unit": "CN steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.name}: oracle PHIF build ({tf:.1f} s, untimed in value) then "
                      f"{budget_steps} CN steps at rtol 1e-8, mean n_i {np.mean(its):.2f}, "
                      f"one thread",
            "t_factor_s": tf, "host_cpu": model, "host_nproc": os.cpu_count()}


def inverse_error(h, N, iters=30, seed=0):
    """||I - A F^-1||_2 by power iteration on E^T E, E = I - A F^-1 (A and F^-1 symmetric, so
    E^T = I - F^-1 A), from a seeded random start; applies and products on the GPU."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    x /= torch.linalg.norm(x)
    t = torch.empty_like(x)
    s = torch.empty_like(x)
    lam = 0.0
    for _ in range(iters):
        h.apply(x, out=t)       # F^-1 x
        h.spmv(t, out=s)        # A F^-1 x
        y = x - s               # E x
        h.spmv(y, out=t)        # A y
        h.apply(t, out=s)       # F^-1 A y
        z = y - s               # E^T E x
        lam = float(torch.linalg.norm(z))
        x = z / lam
    return lam ** 0.5


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
                    row["inv_error"] = inverse_error(h, w.N)
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


def reference_error(w, u_gpu, nsteps):
    """Relative error of the GPU u against the FP64 sparse direct solution of the same steps."""
    import numpy as np
    import scipy.sparse.linalg as spla

    from oracle import cn, fd
    A, B = fd.cn_matrices(w.a_cells, w.dt)
    lu = spla.splu(A.tocsc())
    u = w.u0.ravel().copy()
    for _ in range(nsteps):
        u = lu.solve(cn.cn_rhs(B, u, w.dt, w.reaction))
    return float(np.linalg.norm(u_gpu - u) / np.linalg.norm(u))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fisher2d-256")
    ap.add_argument("--store", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--leaf", type=int, default=0, help="leaf box size (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the error check")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage breakdown")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving workload (0: skip)")
    ap.add_argument("--serving-rate", type=float, default=-1.0,
                    help="Poisson arrival rate of serving requests per second; -1: 0.7 x the "
                         "saturated throughput measured first; 0: only the saturated run")
    ap.add_argument("--serving-slots", type=int, default=32)
    ap.add_argument("--serving-builders", type=int, default=8,
                    help="threads (each with its own stream) building factors concurrently")
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration)")
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

    import numpy as np
    import torch

    from paper_2004_05566_amd import hifcn
    from workloads import gen

    def serving():
        """Saturated run (all requests at t = 0) to measure the throughput mu, then Poisson
        arrivals at the stated rate (default 0.7 mu)."""
        budget = int(args.serving_budget_gb * (1 << 30))
        sat = serving_bench(args.serving, 0.0, args.serving_slots, budget, args.serving_builders)
        out = {"saturated": sat}
        rate = args.serving_rate
        if rate < 0:
            rate = round(0.7 * sat["requests_per_s"], 1)
            out["rate_rule"] = "0.7 x saturated requests/s"
        if rate > 0:
            out["poisson"] = serving_bench(args.serving, rate, args.serving_slots, budget,
                                           args.serving_builders)
        return out

    if args.serving_only:
        print(json.dumps({"serving": serving()}))
        return 0

    w = gen.workload(args.workload)
    if args.leaf:
        w.leaf = args.leaf
    dev = torch.device("cuda:0")
    a_dev = torch.tensor(w.a_cells, dtype=torch.float64, device=dev)
    u0 = torch.tensor(w.u0.ravel(), dtype=torch.float64, device=dev)
    react = w.reaction

    _sync()
    t0 = time.perf_counter()
    h = hifcn.factor(a_dev, w.dt, w.n, w.dim, w.eps, store=args.store, leaf=w.leaf)
    _sync()
    t_factor = time.perf_counter() - t0

    elapsed, its, rel, u = _time_cn(h, u0, args.steps, args.warmup, args.rtol, react)
    value = args.steps / elapsed

    # dominant kernel: the level-0 cell stages, timed live with HIP events on the stream they
    # run on, over a second pass of the same timed steps
    roof = {}
    for st in ("cell_fwd", "cell_bwd"):
        h.profile_stage(0, st, True)
        _time_cn(h, u0, args.steps, 0, args.rtol, react)
        p = h.profile_read()
        h.profile_stage(0, st, False)
        roof[st] = p
    dom = max(roof, key=lambda k: roof[k]["ms"])
    pd = roof[dom]
    avg_s = pd["ms"] / 1e3 / max(1, pd["launches"])
    achieved = pd["bytes"] / avg_s / 1e9
    kname = {"cell_fwd": "k_cell_fwd", "cell_bwd": "k_cell_bwd"}[dom]
    traffic = pmc_traffic(kname, args.store, w.name)

    # FP64-stored factor, same workload (the metric compares both forms)
    h64 = hifcn.factor(a_dev, w.dt, w.n, w.dim, w.eps, store="f64", leaf=w.leaf)
    el64, its64, _, _ = _time_cn(h64, u0, args.steps, args.warmup, args.rtol, react)

    # apply and SpMV bandwidth (algorithmic bytes: the sum over the apply's stages of the factor
    # blocks in the form they are read, their index lists and the FP64 vectors they move)
    x = torch.randn(w.N, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    t_apply = _time_op(lambda: h.apply(x, out=y), 50)
    apply_bytes = h.info()["apply_bytes"]
    t_spmv = _time_op(lambda: h.spmv(x, out=y), 200)
    spmv_bytes = (8 + 8 + 8 * w.dim) * w.N
    stages = None if args.no_stages else stage_breakdown(h, x, y, h.info()["levels"])

    err = None
    if not args.no_check:
        err = reference_error(w, u.cpu().numpy(), args.warmup + args.steps)

    out = {
        "metric": "CN steps/s at 1e-8 rel. resid (FP32-HIF vs FP64), HIF-apply GB/s; p99 latency",
        "value": value,
        "unit": "CN steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f64 CG / f32 HIF storage", "bf16": "f64 CG / bf16 HIF storage",
                  "f64": "f64"}[args.store],
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "dim": w.dim, "n": w.n, "eps": w.eps,
                   "dt": w.dt, "leaf": w.leaf, "store": args.store, "rtol": args.rtol,
                   "reaction": list(react)},
        "n_i_mean": float(np.mean(its)),
        "f64_store": {"value": args.steps / el64, "n_i_mean": float(np.mean(its64))},
        "t_factor_s": t_factor,
        "build_mfma": _build_mfma(h.info()),
        "factor_bytes": h.factor_bytes(),
        "device_bytes": h.info()["device_bytes"],
        "apply": {"us": t_apply * 1e6, "GB/s": apply_bytes / t_apply / 1e9,
                  "bytes": apply_bytes},
        "spmv": {"us": t_spmv * 1e6, "GB/s": spmv_bytes / t_spmv / 1e9, "bytes": spmv_bytes},
        "rel_err_vs_direct": err,
        "roofline": {"bound": "hbm", "kernel": f"{kname} (level 0, {dom})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": pd["bytes"],
                     "avg_us": avg_s * 1e6, "launches": pd["launches"],
                     "other_level0_stage_us": {k: 1e3 * v["ms"] / max(1, v["launches"])
                                               for k, v in roof.items()}},
        "apply_stages": stages,
    }
    h.close()
    h64.close()
    if args.serving:
        out["serving"] = serving()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, 10)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
