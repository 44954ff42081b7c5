"""Continuous batching: cn_batch_step and the Server (GPU).

cn_batch_step runs the solves whose factors allow it with one launch per stage for all of them
(batched kernels over a table of solves; levels aligned from the leaves); the rest (BF16
storage) with per-solve launches.  Either way every solve keeps its own block counts and stage
plans, so its result is bitwise the same alone (a batch of one) and in any mix, iteration
counts included.  The batched kernels split some dot products differently from the single-solve
entry points (cn_step, cn_solve), so against those the bar is the FP64 parity bar: 1e-10 at
rtol 1e-12.  One solve of the mix is also checked against the oracle.
"""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _req(n, dt, seed, nsteps, reaction=(1, 1.0, 1.0), store="f32", eps=1e-4):
    from paper_2004_05566_amd.serve import Request
    a = gen.spectral_grf_coefficient(n, 2, 0.1, seed)
    u0 = gen.bumps(n, 2, 5, seed + 1)
    return Request(n, a, u0, dt, nsteps, eps=eps, reaction=reaction, store=store)


def _alone(r):
    """The request run by itself through cn_batch_step, a batch of one per step (with the
    factor options the Server uses: no dense top)."""
    import torch
    from paper_2004_05566_amd import hifcn
    a = torch.tensor(r.a_cells, dtype=torch.float64, device="cuda:0")
    u = torch.tensor(r.u0.ravel(), dtype=torch.float64, device="cuda:0")
    h = hifcn.factor(a, r.dt, r.n, r.dim, r.eps, store=r.store, leaf=r.leaf, dense_top=0)
    s = torch.cuda.current_stream()
    its, rels = [], []
    for _ in range(r.nsteps):
        it, rel, st = hifcn.cn_batch_step([h], [u], [r.reaction], [r.rtol], [r.maxit], [s])
        assert st[0] == hifcn.HIF_OK
        its.append(int(it[0]))
        rels.append(float(rel[0]))
    h.close()
    return u.cpu().numpy().reshape((r.n,) * r.dim), np.array(its, np.int32), np.array(rels)


def _single(r, rtol):
    """The request through cn_solve (the single-solve entry point)."""
    import torch
    from paper_2004_05566_amd import hifcn
    a = torch.tensor(r.a_cells, dtype=torch.float64, device="cuda:0")
    u = torch.tensor(r.u0.ravel(), dtype=torch.float64, device="cuda:0")
    h = hifcn.factor(a, r.dt, r.n, r.dim, r.eps, store=r.store, leaf=r.leaf, dense_top=0)
    its, rel = h.cn_solve(u, r.nsteps, rtol=rtol, maxit=r.maxit, reaction=r.reaction)
    h.close()
    return u.cpu().numpy().reshape((r.n,) * r.dim), its, rel


def test_batch_step_equals_single_steps(gpu_lib):
    """A mixed batch (sizes, dt, reaction, FP32/FP64 storage, which the batched kernels run as
    one launch per stage each, and BF16, which takes per-solve launches): each solve bitwise as
    alone, and within 1e-10 of cn_solve at rtol 1e-12."""
    import torch
    from paper_2004_05566_amd import hifcn
    reqs = [_req(40, 1e-2, 101, 3), _req(64, 1e-1, 111, 3, reaction=(0, 0.0, 1.0)),
            _req(33, 1e-3, 121, 3, store="f64"), _req(48, 1e-2, 131, 3, store="bf16"),
            _req(128, 1e-2, 141, 3), _req(24, 1e-1, 151, 3, store="f64")]
    for r in reqs:
        r.rtol = 1e-12
    handles, states, streams = [], [], []
    for r in reqs:
        a = torch.tensor(r.a_cells, dtype=torch.float64, device="cuda:0")
        handles.append(hifcn.factor(a, r.dt, r.n, 2, r.eps, store=r.store, dense_top=0))
        states.append(torch.tensor(r.u0.ravel(), dtype=torch.float64, device="cuda:0"))
        streams.append(torch.cuda.Stream())
    torch.cuda.synchronize()
    hist = []
    for _ in range(3):
        its, rel, sts = hifcn.cn_batch_step(handles, states, [r.reaction for r in reqs],
                                            [r.rtol for r in reqs], [r.maxit for r in reqs],
                                            streams)
        assert (sts == hifcn.HIF_OK).all()
        hist.append(its)
    for k, r in enumerate(reqs):
        print(f"[case] batch entry {k}: n={r.n} store={r.store}", flush=True)
        u, its, _ = _alone(r)
        got = states[k].cpu().numpy().reshape(u.shape)
        assert np.array_equal(got, u), k
        assert [int(h[k]) for h in hist] == list(its)
        us, its_s, _ = _single(r, 1e-12)
        assert np.linalg.norm(got - us) <= 1e-10 * np.linalg.norm(us), k
        assert np.abs(got - us).max() <= 1e-10 * np.abs(us).max(), k
        assert all(abs(int(x) - int(y)) <= 1 for x, y in zip(its, its_s))
    for h in handles:
        h.close()


def test_batch_step_rejects_duplicate_handle(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    r = _req(24, 1e-2, 131, 1)
    a = torch.tensor(r.a_cells, dtype=torch.float64, device="cuda:0")
    h = hifcn.factor(a, r.dt, r.n, 2, r.eps)
    u = torch.tensor(r.u0.ravel(), dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    with pytest.raises(hifcn.HifError) as e:
        hifcn.cn_batch_step([h, h], [u, u], [r.reaction] * 2, [1e-8] * 2, [100] * 2, [s, s])
    assert e.value.status == hifcn.HIF_ERR_ARG
    its, _, sts = hifcn.cn_batch_step([], [], [], [], [], [])
    assert its.size == 0 and sts.size == 0
    h.close()


def test_batch_step_reports_per_solve_no_convergence(gpu_lib):
    """A solve stopped by maxit reports HIF_ERR_NO_CONV; its partner still completes."""
    import torch
    from paper_2004_05566_amd import hifcn
    reqs = [_req(48, 1e-1, 141, 1, eps=1e-1), _req(32, 1e-2, 151, 1)]
    hs, us, ss = [], [], []
    for r in reqs:
        a = torch.tensor(r.a_cells, dtype=torch.float64, device="cuda:0")
        hs.append(hifcn.factor(a, r.dt, r.n, 2, r.eps, dense_top=0))
        us.append(torch.tensor(r.u0.ravel(), dtype=torch.float64, device="cuda:0"))
        ss.append(torch.cuda.Stream())
    its, rel, sts = hifcn.cn_batch_step(hs, us, [r.reaction for r in reqs], [1e-14, 1e-8],
                                        [2, 200], ss)
    assert sts[0] == hifcn.HIF_ERR_NO_CONV and its[0] == 2
    assert sts[1] == hifcn.HIF_OK and rel[1] <= 1e-8
    u_alone, its_alone, _ = _alone(reqs[1])
    assert np.array_equal(us[1].cpu().numpy().reshape(u_alone.shape), u_alone)
    for h in hs:
        h.close()


def test_server_mix_equals_alone(gpu_lib):
    """Requests of mixed size, dt, reaction and length arriving while others run: each result
    equals the same request run alone, and the server overlaps them in batches."""
    import time
    from paper_2004_05566_amd.serve import Server, percentiles
    specs = [(64, 1e-1, 8), (32, 1e-2, 5), (128, 1e-3, 4), (48, 1e-1, 7), (64, 1e-2, 3),
             (96, 1e-3, 6), (32, 1e-1, 9), (80, 1e-2, 4)]
    reqs = [_req(n, dt, 200 + 10 * i, k, reaction=((1, 1.0, 1.0) if i % 2 else (0, 0.0, 1.0)),
                 store=("f32", "f64", "bf16")[i % 3])
            for i, (n, dt, k) in enumerate(specs)]
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=3, builders=2, paused=True, lanes=1)
    futs = [srv.submit(r) for r in reqs[:5]]
    t_end = time.time() + 60
    while srv.ready_count() < 3 and time.time() < t_end:  # the first three slots are built
        time.sleep(0.005)
    srv.resume()
    for i, r in enumerate(reqs[5:]):  # the rest arrive while the batch runs
        time.sleep(0.002)
        futs.append(srv.submit(r))
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    st = srv.stats()
    assert st["max_batch"] == 3, st           # solves overlapped, up to the slot limit
    for r, res in zip(reqs, results):
        u, its, rel = _alone(r)
        assert np.array_equal(res.u, u)
        assert np.array_equal(res.iters, its)
        assert res.latency > 0 and res.t_done >= res.t_ready >= res.t_admit >= res.t_arrival
    p = percentiles([r.latency for r in results])
    assert 0 < p["p50"] <= p["p99"]


def test_server_result_matches_oracle(gpu_lib):
    """One FP64-stored request through the server against the oracle (FP64 parity bar)."""
    from oracle import cn, fd, phif
    from paper_2004_05566_amd.serve import Server
    r = _req(32, 1e-2, 301, 4, store="f64", eps=1e-6)
    r.rtol = 1e-12  # both solves tight enough that their rounding differences stay below 1e-10
    srv = Server(hbm_budget_bytes=1 << 28, max_slots=2)
    res = srv.submit(r).result(timeout=60)
    srv.close()
    A, B = fd.cn_matrices(r.a_cells, r.dt)
    F = phif.phif_build(A, r.n, 2, 8, r.eps)
    us, its, _ = cn.cn_solve(A, B, r.u0, r.dt, r.nsteps, lambda v: phif.phif_apply(F, v),
                             r.rtol, r.reaction)
    u = us[-1].reshape(res.u.shape)
    assert np.linalg.norm(res.u - u) <= 1e-10 * np.linalg.norm(u)
    assert np.all(np.abs(np.asarray(its) - res.iters) <= 1)


def test_server_admission_by_memory(gpu_lib):
    """A request that can never fit is rejected; ones that fit only one at a time are served
    one at a time (the budget, not the slot count, limits them)."""
    from paper_2004_05566_amd.serve import Server, estimate_bytes
    small = _req(32, 1e-2, 401, 2)
    big = _req(128, 1e-2, 411, 2)
    one = estimate_bytes(32, 2, "f32")
    budget = (3 * one) // 2
    assert estimate_bytes(128, 2, "f32") > budget
    srv = Server(hbm_budget_bytes=budget, max_slots=4)
    f_big = srv.submit(big)
    with pytest.raises(MemoryError):
        f_big.result(timeout=10)
    futs = [srv.submit(small)] + [srv.submit(_req(32, 1e-2, 421 + 10 * i, 2)) for i in range(3)]
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    assert srv.stats()["peak_held_bytes"] <= budget
    # two estimates never fit together, so no two factor builds overlapped in time
    spans = sorted((r.t_admit, r.t_ready) for r in res)
    assert all(b[0] >= a[1] for a, b in zip(spans, spans[1:])), spans
    u, its, _ = _alone(small)
    assert np.array_equal(res[0].u, u) and np.array_equal(res[0].iters, its)


def test_server_lanes_mix_equals_alone(gpu_lib):
    """Several scheduler lanes (solves grouped by size) running concurrently: same results."""
    from paper_2004_05566_amd.serve import Server
    specs = [(32, 1e-2, 3), (64, 1e-1, 4), (128, 1e-3, 2), (32, 1e-1, 5), (64, 1e-2, 3),
             (128, 1e-2, 2)]
    reqs = [_req(n, dt, 500 + 10 * i, k) for i, (n, dt, k) in enumerate(specs)]
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=6, builders=3, lanes=3)
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    for r, x in zip(reqs, res):
        u, its, _ = _alone(r)
        assert np.array_equal(x.u, u) and np.array_equal(x.iters, its)


def test_server_lane_failure_resolves_every_future(gpu_lib, monkeypatch):
    """When one scheduler lane's batched step raises, every submitted request still resolves
    (with that error or its result): the failing lane's solves, the other lanes' active solves,
    solves whose factor finishes building after the failure, and those still waiting."""
    import threading
    from concurrent.futures import wait

    from paper_2004_05566_amd import hifcn
    from paper_2004_05566_amd.serve import Server
    real = hifcn.cn_batch_step
    fired = {"done": False}
    lock = threading.Lock()

    def flaky(handles, *a, **k):
        with lock:  # the first batch holding a 64^2 solve fails
            boom = not fired["done"] and any(h.n == 64 for h in handles)
            fired["done"] = fired["done"] or boom
        if boom:
            raise RuntimeError("planted failure in one lane")
        return real(handles, *a, **k)

    monkeypatch.setattr(hifcn, "cn_batch_step", flaky)
    specs = [(32, 1e-2, 6), (64, 1e-1, 6), (128, 1e-3, 6), (64, 1e-2, 6), (32, 1e-1, 6),
             (128, 1e-2, 6), (96, 1e-2, 6), (48, 1e-3, 6)]
    reqs = [_req(n, dt, 700 + 10 * i, k) for i, (n, dt, k) in enumerate(specs)]
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=4, builders=2, lanes=3)
    futs = [srv.submit(r) for r in reqs]
    done, pending = wait(futs, timeout=120)
    assert not pending, f"{len(pending)} futures never resolved"
    errs = [f.exception() for f in futs]
    assert any(isinstance(e, RuntimeError) for e in errs)
    with pytest.raises(RuntimeError):
        srv.close()
    assert srv._slots == 0 and srv._held == 0


def test_server_cancel_waiting_building_and_running(gpu_lib):
    """Future.cancel() withdraws a request at any stage: one still waiting for a slot, one whose
    factor is being built or ready (the server is paused), and one in the middle of its steps.
    Each leaves its slot and memory; the requests left run to results bitwise equal to running
    alone."""
    import time
    from paper_2004_05566_amd.serve import Server
    keep = _req(48, 0.02, 71, 3)
    long_run = _req(64, 0.02, 73, 100000)    # would run for minutes if not withdrawn
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=2, builders=2, paused=True, lanes=1)
    f_keep = srv.submit(keep)
    f_ready = srv.submit(_req(40, 0.02, 75, 3))
    f_wait = srv.submit(_req(32, 0.02, 77, 3))   # no slot while the other two hold both
    assert f_wait.cancel()
    t0 = time.perf_counter()
    while srv.ready_count() < 2 and time.perf_counter() - t0 < 120:
        time.sleep(0.01)
    assert srv.ready_count() == 2
    assert f_ready.cancel()
    srv.resume()
    res = f_keep.result(timeout=120)
    f_long = srv.submit(long_run)
    t0 = time.perf_counter()
    while srv.rounds < 20 and time.perf_counter() - t0 < 120:  # the long solve is running
        time.sleep(0.01)
    assert f_long.cancel()
    srv.close(wait=True)
    assert f_wait.cancelled() and f_ready.cancelled() and f_long.cancelled()
    u, its, rel = _alone(keep)
    assert np.array_equal(res.u, u) and np.array_equal(res.iters, its)
    st = srv.stats()
    assert st["cancelled"] == 3
    assert srv._slots == 0 and srv._held == 0
    assert st["rounds"] < 100000
