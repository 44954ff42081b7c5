"""Continuous-batching server for independent Crank-Nicolson solves on one GPU.

Each request is a whole parabolic solve (its own grid, coefficient a, dt, reaction, step count;
eq1 and eq_CN, Sec. 2.1) preconditioned by its own HIF factor (Sec. 2.2).  The server

  * admits a request when a slot is free and its estimated HBM footprint fits the budget
    (a request that could never fit is rejected at once, one that does not fit now waits),
  * builds its factor on a builder thread, on a stream of its own, while the batch runs,
  * advances every resident solve by one Crank-Nicolson step per round with one call of the
    library's batched entry point (one launch per stage for all solves of a storage precision:
    the PCG vector kernels over a table of the solves and the apply with its levels aligned
    from the leaves; PCG iterations in lockstep, one convergence read-back per round for the
    whole batch), and newly built solves join at the next round; optionally several scheduler
    lanes (solves of similar size share one) run their batches concurrently,
  * copies a finished solve's state to the host, resolves its future and frees its memory,
  * honours Future.cancel() at any time before the future is resolved: a waiting request is
    dropped, one being built is freed once its build ends, a running one leaves the batch before
    the next round (its slot and memory are released like a finished solve's).

A solve's arithmetic does not depend on the other solves in the batch (every kernel touches only
its own handle's buffers and every reduction has a fixed order), so its result is bitwise the
same alone and in any mix.  This module only schedules: every step of every solve runs in the
library's kernels.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future, InvalidStateError, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import hifcn


@dataclass
class Request:
    """One independent solve: n^dim interior nodes, a on the (n+1)^dim cells, u0 on the nodes."""

    n: int
    a_cells: np.ndarray
    u0: np.ndarray
    dt: float
    nsteps: int
    eps: float = 1e-4
    reaction: tuple = (0, 0.0, 1.0)
    dim: int = 2
    rtol: float = 1e-8
    maxit: int = 500
    store: str = "f32"
    leaf: int = 8
    tag: object = None


@dataclass
class Result:
    u: np.ndarray            # final state, shape n^dim (FP64)
    iters: np.ndarray        # PCG iterations of every step
    relres: np.ndarray       # final relative residual of every step
    t_arrival: float         # perf_counter times
    t_admit: float
    t_ready: float
    t_done: float
    device_bytes: int        # HBM the solve held while resident
    tag: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def estimate_bytes(n: int, dim: int, store: str) -> int:
    """Upper estimate of the device memory one solve needs while its factor is built.

    The build keeps the factor's blocks in FP64 (up to about 48 entries per DOF for the 2D
    workloads at eps = 1e-4 and 3x that in 3D) besides their stored copy, plus the PCG
    workspace and coefficients (about 12 FP64 vectors).  The dense top of the apply holds at
    most 10M entries, and fewer than (N/4)^2 (N/4 bounds the separator DOFs of the levels it
    covers), formed through about six FP64 matrices of its size."""
    N = n ** dim
    entries = 48 if dim == 2 else 144
    eb = {"f64": 8, "f32": 4, "bf16": 2}[store]
    top = min(10 << 20, (N // 4) ** 2)
    return int(N * (entries * (8 + eb) + 12 * 8) + top * (eb + 48) + (8 << 20))


@dataclass
class _Job:
    req: Request
    fut: Future
    t_arrival: float
    est: int
    held: int = 0
    t_admit: float = 0.0
    t_ready: float = 0.0
    handle: object = None
    u: object = None
    stream: object = None
    step: int = 0
    iters: list = field(default_factory=list)
    relres: list = field(default_factory=list)


class Server:
    """Serve Request objects with at most `max_slots` resident solves within `hbm_budget_bytes`.

    `lanes` scheduler threads each advance their own batch of resident solves (solves of similar
    size share a lane) with the batched step entry point, concurrently with each other.
    submit() returns a concurrent.futures.Future resolved with a Result (or the error); its
    cancel() withdraws the request until the future is resolved."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 32, builders: int = 2,
                 device: int = 0, paused: bool = False, lanes: int = 1, dense_top: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        # the factors' dense top (hif_factor_ex): off by default, since forming it costs more
        # build time than a request's few steps win back
        self.dense_top = dense_top
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self._cv = threading.Condition()
        self._waiting: collections.deque[_Job] = collections.deque()
        self._ready: list[_Job] = []
        self._held = 0       # bytes reserved by admitted solves
        self._slots = 0      # admitted solves (building, ready or active)
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_slots)]
        # the batched step of a lane runs all its solves on one stream (the lane's)
        self._free_streams = list(range(self.max_slots))
        self._builders = ThreadPoolExecutor(max_workers=max(1, builders),
                                            thread_name_prefix="hif-build")
        # finished solves are released on a thread of their own (hif_destroy waits for the
        # device once), so that releases never hold up builds
        self._freer = ThreadPoolExecutor(max_workers=1, thread_name_prefix="hif-free")
        self._tls = threading.local()
        self._closing = False
        self._paused = bool(paused)  # admit and build, but run no rounds until resume()
        self.rounds = 0
        self.batch_sizes: list[int] = []
        self.step_seconds = 0.0  # time spent in the batched step calls
        self.build_seconds = 0.0  # builder-thread time in factor builds
        self.free_seconds = 0.0   # builder-thread time releasing finished solves
        self.cancelled = 0        # requests withdrawn by Future.cancel()
        self.peak_held = 0
        self._error: BaseException | None = None
        self.lanes = max(1, int(lanes))
        self._lane_streams = [torch.cuda.Stream(device=self.device) for _ in range(self.lanes)]
        self._threads = [threading.Thread(target=self._run_lane, args=(k,),
                                          name=f"hif-serve-{k}", daemon=True)
                         for k in range(self.lanes)]
        for t in self._threads:
            t.start()

    # -- client side -------------------------------------------------------------------------
    def submit(self, req: Request, t_arrival: float | None = None) -> Future:
        fut: Future = Future()
        if req.dim not in (2, 3) or req.n < 1 or req.nsteps < 1:
            fut.set_exception(ValueError("bad request: need dim in {2,3}, n >= 1, nsteps >= 1"))
            return fut
        if req.a_cells.shape != (req.n + 1,) * req.dim or req.u0.size != req.n ** req.dim:
            fut.set_exception(ValueError("a_cells must have (n+1)^dim and u0 n^dim values"))
            return fut
        est = estimate_bytes(req.n, req.dim, req.store)
        if est > self.budget:
            fut.set_exception(MemoryError(
                f"request needs about {est} bytes of HBM, more than the budget {self.budget}"))
            return fut
        job = _Job(req, fut, time.perf_counter() if t_arrival is None else t_arrival, est)
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            self._waiting.append(job)
            self._cv.notify_all()
        return fut

    def resume(self):
        """Start the batch rounds of a server created with paused=True."""
        with self._cv:
            self._paused = False
            self._cv.notify_all()

    def ready_count(self) -> int:
        """Solves whose factor is built and that wait for their first round."""
        with self._cv:
            return len(self._ready)

    def close(self, wait: bool = True):
        """Stop accepting requests; finish (wait=True) every admitted and waiting request."""
        with self._cv:
            self._closing = True
            self._paused = False
            self._cv.notify_all()
        if wait:
            for t in self._threads:
                t.join()
        self._builders.shutdown(wait=wait)
        self._freer.shutdown(wait=wait)
        if self._error is not None:
            raise self._error

    def stats(self) -> dict:
        b = np.array(self.batch_sizes or [0])
        return {"rounds": self.rounds, "mean_batch": float(b.mean()), "max_batch": int(b.max()),
                "step_call_s": self.step_seconds, "build_thread_s": self.build_seconds,
                "free_thread_s": self.free_seconds, "cancelled": self.cancelled,
                "peak_held_bytes": int(self.peak_held), "budget_bytes": self.budget,
                "max_slots": self.max_slots}

    # -- builder threads ---------------------------------------------------------------------
    def _build_stream(self):
        import torch
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self._tls.stream = torch.cuda.Stream(device=self.device)
        return s

    def _build(self, job: _Job):
        t0 = time.perf_counter()
        try:
            return self._build_body(job)
        finally:
            dt = time.perf_counter() - t0
            with self._cv:
                self.build_seconds += dt

    def _build_body(self, job: _Job):
        import torch
        r = job.req
        s = self._build_stream()
        with torch.cuda.stream(s):
            a = torch.as_tensor(np.ascontiguousarray(r.a_cells, dtype=np.float64)).to(
                self.device, non_blocking=False)
            u = torch.as_tensor(np.ascontiguousarray(r.u0, dtype=np.float64).ravel()).to(
                self.device, non_blocking=False)
            h = hifcn.factor(a, r.dt, r.n, r.dim, r.eps, store=r.store, leaf=r.leaf, stream=s,
                             dense_top=self.dense_top)
            s.synchronize()  # u is ready for the slot's stream, a may be released
            del a
        return h, u

    def _destroy(self, handle):
        t0 = time.perf_counter()
        handle.close()
        dt = time.perf_counter() - t0
        with self._cv:
            self.free_seconds += dt

    # -- scheduler ---------------------------------------------------------------------------
    def _admit_locked(self):
        if any(j.fut.cancelled() for j in self._waiting):  # withdrawn before admission
            keep: collections.deque[_Job] = collections.deque()
            for j in self._waiting:
                if j.fut.cancelled():
                    self.cancelled += 1
                else:
                    keep.append(j)
            self._waiting = keep
        while self._waiting and self._slots < self.max_slots:
            job = self._waiting[0]
            if self._held + job.est > self.budget:
                break  # first come, first served: later requests wait behind this one
            self._waiting.popleft()
            self._slots += 1
            self._held += job.est
            job.held = job.est
            self.peak_held = max(self.peak_held, self._held)
            job.t_admit = time.perf_counter()
            job.stream = self._streams[self._free_streams.pop()]
            f = self._builders.submit(self._build, job)
            f.add_done_callback(lambda f, job=job: self._built(job, f))

    def _built(self, job: _Job, f):
        with self._cv:
            try:
                job.handle, job.u = f.result()
            except BaseException as e:  # factor failed: report it and give the slot back
                self._release_locked(job)
                _resolve(job.fut, exc=e)
                self._cv.notify_all()
                return
            if job.fut.cancelled():  # withdrawn while it was built
                self._cancel_locked(job)
                self._cv.notify_all()
                return
            if self._error is not None:  # a lane failed meanwhile: no lane will run this one
                self._abandon_locked(job, self._error)
                self._cv.notify_all()
                return
            actual = int(job.handle.info()["device_bytes"])
            self._held += actual - job.held
            job.held = actual
            self.peak_held = max(self.peak_held, self._held)
            job.t_ready = time.perf_counter()
            self._ready.append(job)
            self._cv.notify_all()

    def _release_locked(self, job: _Job):
        self._release_slot_locked(job)
        self._release_bytes_locked(job)

    def _release_slot_locked(self, job: _Job):
        self._slots -= 1
        self._free_streams.append(self._streams.index(job.stream))

    def _release_bytes_locked(self, job: _Job):
        self._held -= job.held
        job.held = 0

    def _abandon_locked(self, job: _Job, exc: BaseException):
        """Fail an admitted job that will not run (its handle is freed, its slot returned)."""
        _resolve(job.fut, exc=exc)
        if job.handle is not None:
            try:
                job.handle.close()
            except Exception:  # noqa: BLE001 - already failing; the slot is returned anyway
                pass
            job.handle, job.u = None, None
        if job.stream is not None:
            self._release_locked(job)
            job.stream = None

    def _cancel_locked(self, job: _Job):
        """Release a withdrawn solve: its slot at once, its memory once the handle is freed."""
        self.cancelled += 1
        h, job.handle, job.u = job.handle, None, None
        self._release_slot_locked(job)
        if h is None:
            self._release_bytes_locked(job)
            return
        done = self._freer.submit(self._destroy, h)
        done.add_done_callback(lambda _f, job=job: self._freed(job))

    def _finish(self, job: _Job, status: int):
        r = job.req
        if status == hifcn.HIF_OK:
            u = job.u.cpu().numpy().reshape((r.n,) * r.dim)
            res = Result(u, np.array(job.iters, np.int32), np.array(job.relres), job.t_arrival,
                         job.t_admit, job.t_ready, time.perf_counter(), job.held, r.tag)
        h, job.handle, job.u = job.handle, None, None
        # the slot is free at once; the memory counts against the budget until it is released
        # (off the batch loop: the release waits for the device)
        with self._cv:
            self._release_slot_locked(job)
            self._cv.notify_all()
        done = self._freer.submit(self._destroy, h)
        done.add_done_callback(lambda _f, job=job: self._freed(job))
        if status == hifcn.HIF_OK:
            _resolve(job.fut, result=res)
        else:
            _resolve(job.fut, exc=hifcn.HifError(status, f"PCG did not converge at step "
                                                         f"{job.step} of {r.nsteps}"))

    def _freed(self, job: _Job):
        with self._cv:
            self._release_bytes_locked(job)
            self._cv.notify_all()

    @staticmethod
    def _lane_of(job: "_Job", lanes: int) -> int:
        """Solves of similar size share a lane (rounds in lockstep wait for their slowest
        member, so mixing a 64^2 and a 512^2 solve would hold the small one back)."""
        N = job.req.n ** job.req.dim
        return (N.bit_length() // 2) % lanes

    def _run_lane(self, lane: int):
        active: list[_Job] = []
        try:
            while True:
                with self._cv:
                    if self._error is not None:  # another lane failed: fail this lane's solves
                        for j in active:
                            self._abandon_locked(j, self._error)
                        active.clear()
                        self._cv.notify_all()
                        return
                    self._admit_locked()
                    for j in [j for j in self._ready if j.fut.cancelled()]:
                        self._ready.remove(j)
                        self._cancel_locked(j)
                    for j in [j for j in active if j.fut.cancelled()]:
                        active.remove(j)
                        self._cancel_locked(j)
                    if not self._paused:
                        mine = [j for j in self._ready if self._lane_of(j, self.lanes) == lane]
                        for j in mine:
                            self._ready.remove(j)
                        active.extend(mine)
                    if not active:
                        if self._closing and not self._waiting and self._slots == 0:
                            self._cv.notify_all()
                            return
                        self._cv.wait(timeout=0.02)
                        continue
                    batch = list(active)
                t0 = time.perf_counter()
                its, rel, sts = hifcn.cn_batch_step(
                    [j.handle for j in batch], [j.u for j in batch],
                    [j.req.reaction for j in batch], [j.req.rtol for j in batch],
                    [j.req.maxit for j in batch], [self._lane_streams[lane]] * len(batch))
                dt_step = time.perf_counter() - t0
                with self._cv:
                    self.step_seconds += dt_step
                    self.rounds += 1
                    self.batch_sizes.append(len(batch))
                finished = []
                for j, it, rr, st in zip(batch, its, rel, sts):
                    j.step += 1
                    j.iters.append(int(it))
                    j.relres.append(float(rr))
                    if st != hifcn.HIF_OK or j.step == j.req.nsteps:
                        finished.append((j, int(st)))
                for j, st in finished:
                    active.remove(j)
                    self._finish(j, st)
        except BaseException as e:  # fail every outstanding request rather than hang them
            with self._cv:
                if self._error is None:
                    self._error = e
                for j in list(self._waiting):  # not admitted: nothing held
                    _resolve(j.fut, exc=e)
                self._waiting.clear()
                for j in self._ready + active:
                    self._abandon_locked(j, e)
                self._ready.clear()
                active.clear()
                self._cv.notify_all()


def _resolve(fut: Future, result=None, exc: BaseException | None = None):
    """Resolve a request's future unless the client cancelled it meanwhile."""
    try:
        if exc is not None:
            fut.set_exception(exc)
        else:
            fut.set_result(result)
    except InvalidStateError:  # cancelled (or already resolved): nothing to report
        pass


def percentiles(latencies, qs=(50, 99)) -> dict:
    """p50/p99 (nearest-rank) of a list of latencies in seconds."""
    x = np.sort(np.asarray(latencies, dtype=np.float64))
    out = {}
    for q in qs:
        k = max(0, int(np.ceil(q / 100.0 * x.size)) - 1)
        out[f"p{q}"] = float(x[k]) if x.size else None
    return out
