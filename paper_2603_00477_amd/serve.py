"""Continuous-batching server for stencil jobs on one GPU.

Requests (stencil jobs of mixed shape, size and step count) arrive at any
time.  A scheduler thread:

  * admits queued jobs in arrival order while their device footprint (two
    resident grids plus the plan's operand blocks) fits the HBM budget; a job
    larger than the whole budget is rejected;
  * keeps admitted grids resident on the device;
  * runs in rounds: each round issues one pass (min(T, steps left) steps) of
    every active job through one stencil_run_batch call, so jobs that arrive
    while others run join the next round and their work shares launches with
    the jobs already running;
  * completes a job when the event recorded after its last round has fired,
    hands its output tensor to the caller and frees the rest of its budget;
    the output grid stays counted against the budget until the caller drops
    its last reference to it (a weak-reference finalizer returns the bytes),
    so results held by callers bound admission like running jobs do.

Latency = completion time - arrival time.  Results are bit-identical to
running each job alone with the same plan: the same kernels run on the same
data in the same pass order.

The executor does the device work; `GpuExecutor` drives the HIP library.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import threading
import time
import weakref
from typing import Any, Callable, Optional

import numpy as np


@dataclasses.dataclass
class Job:
    shape: str
    d: int
    r: int
    weights: Any
    dims: tuple
    steps: int
    dtype: str = "f32"
    boundary: str = "dirichlet"
    halo: float = 0.0
    T: Optional[int] = None          # None: choose by the model
    path: Optional[str] = None       # None: the plan's resolved path
    data: Any = None                 # host/device tensor or callable(device) -> device tensor
    arrival: Optional[float] = None  # server clock; None = time of submit()
    id: Any = None


@dataclasses.dataclass
class Done:
    job: Job
    output: Any
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    __slots__ = ("job", "fut", "state", "left", "arrival", "admitted", "bytes")

    def __init__(self, job, fut, state, arrival, admitted, nbytes):
        self.job = job
        self.fut = fut
        self.state = state
        self.left = int(job.steps)
        self.arrival = arrival
        self.admitted = admitted
        self.bytes = nbytes


class GpuExecutor:
    """Device work of the server, through the HIP library.

    Path, fusion depth T and VALU rows per workgroup come from the library's
    model-seeded autotuner (stencil_plan_autotune: candidates ranked by the
    roofline model, the best few timed on the job's own grid), run once per
    problem class (shape, d, r, dtype, boundary and the grid side rounded to
    a power of two) on the first job of the class and applied to the later
    ones; a job that names T or a path keeps it.

    Jobs are spread over `streams` HIP streams (default priority) by kernel
    variant: all jobs of one variant share a stream, so their passes of a
    round go out as one batched launch, while other variants' launches can
    overlap with them on the device; grids of 2^24 points or more take the
    streams in turn, so that a large pass does not hold back the small jobs
    of its variant (measured on the 4096-job stream at 0.8 load: p99 112 ms
    against 162 ms with every job on its variant's stream and 135 ms with 2D
    jobs on one stream and 3D jobs in turn).  A job stays on its stream, so
    its passes run in order."""

    def __init__(self, device="cuda", stream=None, streams=4, autotune=True, tune_candidates=3,
                 stream_policy="size"):
        import torch

        import paper_2603_00477_amd as stl

        self.torch = torch
        self.stl = stl
        self.device = torch.device(device)
        first = stream or torch.cuda.Stream(device=self.device)
        self.streams = [first] + [torch.cuda.Stream(device=self.device) for _ in range(max(0, streams - 1))]
        self.stream = first
        self.autotune = bool(autotune)
        self.stream_policy = stream_policy
        self._rr = 0
        self.tune_candidates = int(tune_candidates)
        self.choices = {}  # problem class -> (path, T, rows, GStencil/s measured when tuned)

    @staticmethod
    def problem_class(job):
        side = max(int(x) for x in job.dims)
        return (job.shape, job.d, job.r, job.dtype, job.boundary, int(round(np.log2(max(side, 1)))))

    def footprint(self, job) -> int:
        return 2 * self.output_bytes(job) + (1 << 20)

    def output_bytes(self, job) -> int:
        """Device bytes of the result grid handed to the caller."""
        D = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16x3": 4}[job.dtype]
        return int(np.prod(job.dims)) * D

    def _stream_index(self, info) -> int:
        """Stream of a job.  "variant": all jobs of a kernel variant share a
        stream (their passes batch); "dim": 2D jobs on stream 0 (batched),
        3D jobs round-robin over the others (overlapping launches);
        "size": like "variant" for grids under 2^24 points, large grids
        round-robin over the streams (a large pass does not hold back the
        small jobs batched with it)."""
        n = len(self.streams)
        if n == 1:
            return 0
        key = (info["shape"], info["d"], info["r"], info["T"], info["dtype"], info["path"])
        npts = int(np.prod(info["dims"]))
        if self.stream_policy == "dim":
            if info["d"] == 2:
                return 0
            self._rr += 1
            return 1 + self._rr % (n - 1)
        if self.stream_policy == "size" and npts >= (1 << 24):
            self._rr += 1
            return self._rr % n
        return hash(key) % n

    def prepare(self, job):
        torch = self.torch
        stl = self.stl
        plan = stl.Plan(job.shape, job.d, job.r, job.weights, job.dims, T=job.T or 1, dtype=job.dtype,
                        boundary=job.boundary, path=job.path, halo=job.halo)
        tdt = stl.torch_dtype(job.dtype)
        key = self.problem_class(job)
        tune = self.autotune and job.T is None and job.path is None
        choice = self.choices.get(key) if tune else None
        if choice is not None:
            path, T, rows, _ = choice
            plan.set(stl._abi.OPT_T, T)
            plan.set(stl._abi.OPT_PATH, path)
            plan.set(stl._abi.OPT_TILE_ROWS, rows)
        with torch.cuda.stream(self.stream):
            if callable(job.data):
                a = job.data(self.device)
            elif isinstance(job.data, torch.Tensor):
                a = job.data.to(self.device, non_blocking=True)
            else:
                a = torch.as_tensor(np.asarray(job.data)).to(self.device)
            a = a.to(tdt).contiguous()
            b = torch.empty_like(a)
        if tune and choice is None:
            # first job of its class: time the model's best candidates on it
            # (the probe runs overwrite b only)
            g = plan.autotune(a, b, 8, max_candidates=self.tune_candidates, stream=self.stream)
            i = plan.info()
            self.choices[key] = (i["path"], i["T"], i.get("tile_rows", 0), g)
        info = plan.info()
        si = self._stream_index(info)
        if si != 0:
            # the grid was written on stream 0: the job's own stream waits for it
            self.streams[si].wait_stream(self.stream)
        return {"plan": plan, "a": a, "b": b, "T": info["T"], "stream": si}

    def run_round(self, states, steps):
        """One pass of every state (one batched call per stream used);
        returns the events that fire when the passes are done."""
        torch = self.torch
        by = {}
        for s, k in zip(states, steps):
            by.setdefault(s["stream"], []).append((s, k))
        for s in states:  # argument checks before any launch
            s["plan"]._check_tensor(s["a"], "in")
            s["plan"]._check_tensor(s["b"], "out")
        events, launched = [], []
        for si, items in sorted(by.items()):
            st = [s for s, _ in items]
            try:
                self.stl.run_batch([s["plan"] for s in st], [s["a"] for s in st], [s["b"] for s in st],
                                   [k for _, k in items], stream=self.streams[si])
            except Exception as e:
                # passes of earlier groups are queued: report them so that
                # the caller does not run them a second time
                e.launched, e.handle = launched, events
                raise
            for s in st:
                s["a"], s["b"] = s["b"], s["a"]
            launched.extend(st)
            ev = torch.cuda.Event()
            ev.record(self.streams[si])
            events.append(ev)
        return events

    def run_job(self, state, steps):
        """All `steps` of one job in one stencil_run call on its stream (the
        one-plan-per-call form); returns an event handle."""
        torch = self.torch
        st = self.streams[state["stream"]]
        state["plan"].run(state["a"], state["b"], steps, stream=st)
        state["a"], state["b"] = state["b"], state["a"]
        ev = torch.cuda.Event()
        ev.record(st)
        return [ev]

    def pass_steps(self, state, left) -> int:
        return min(state["T"], left)

    def done(self, handle) -> bool:
        return all(e.query() for e in handle)

    def wait(self, handle):
        for e in handle:
            e.synchronize()

    def result(self, state):
        return state["a"]

    def release(self, state):
        state["plan"].close()
        state["b"] = None


class _Joined(list):
    """Several executor handles of one round (a round that had to be split);
    the round is complete when every part is."""


class StencilServer:
    def __init__(self, executor, hbm_budget: int, max_inflight_rounds: int = 2,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.used = 0   # bytes of admitted jobs and of results callers still hold
        self.held = 0   # of which: results handed back and not yet released
        self.clock = clock
        self.max_inflight = max(1, int(max_inflight_rounds))
        self._queue = collections.deque()
        self._active = []
        self._inflight = collections.deque()  # (handle, [finished _Active])
        self._cv = threading.Condition()
        self._stop = False
        self._thread = None
        self.rounds = 0
        self.done = []

    # ---- client side
    def submit(self, job: Job) -> cf.Future:
        fut = cf.Future()
        arrival = job.arrival if job.arrival is not None else self.clock()
        with self._cv:
            if self._stop:
                raise RuntimeError("server stopped")
            self._queue.append((job, fut, arrival))
            self._cv.notify()
        return fut

    def start(self):
        self._thread = threading.Thread(target=self._loop, name="stencil-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True):
        with self._cv:
            if not drain:
                while self._queue:
                    job, fut, _ = self._queue.popleft()
                    fut.cancel()
            self._stop = True
            self._cv.notify()
        if self._thread:
            self._thread.join()

    # ---- scheduler
    def _h_done(self, h) -> bool:
        return all(self.ex.done(x) for x in h) if isinstance(h, _Joined) else self.ex.done(h)

    def _h_wait(self, h):
        for x in (h if isinstance(h, _Joined) else [h]):
            self.ex.wait(x)

    def _admit(self):
        while self._queue:
            job, fut, arrival = self._queue[0]
            if fut.cancelled():
                self._queue.popleft()
                continue
            try:
                need = self.ex.footprint(job)
            except Exception as e:  # invalid job description
                self._queue.popleft()
                fut.set_exception(e)
                continue
            if need > self.budget:
                self._queue.popleft()
                fut.set_exception(MemoryError(
                    f"job needs {need} bytes, more than the whole HBM budget {self.budget}"))
                continue
            if self.used + need > self.budget:
                return  # wait for running jobs to free memory (FIFO, no overtaking)
            self._queue.popleft()
            try:
                state = self.ex.prepare(job)
            except Exception as e:
                fut.set_exception(e)
                continue
            self.used += need
            self._active.append(_Active(job, fut, state, arrival, self.clock(), need))

    def _finish(self, a: _Active, now: float):
        out = self.ex.result(a.state)
        self.ex.release(a.state)
        held = 0
        if out is not None and hasattr(self.ex, "output_bytes"):
            held = min(a.bytes, int(self.ex.output_bytes(a.job)))
            try:
                weakref.finalize(out, self._output_dropped, held)
            except TypeError:  # an output type without weak references is not tracked
                held = 0
        self.used -= a.bytes - held
        self.held += held
        # the server keeps timing records only; the output goes to the caller
        self.done.append(Done(a.job, None, a.arrival, a.admitted, now))
        a.fut.set_result(Done(a.job, out, a.arrival, a.admitted, now))

    def _output_dropped(self, nbytes: int):
        """Finalizer of a result grid: the caller released it."""
        with self._cv:
            self.used -= nbytes
            self.held -= nbytes
            self._cv.notify()

    def _reap_ready(self):
        """Finish the jobs of every completed round at the head of the queue
        (never waits; called with the lock held)."""
        while self._inflight and self._h_done(self._inflight[0][0]):
            _, fin = self._inflight.popleft()
            now = self.clock()
            for a in fin:
                self._finish(a, now)

    def _fail(self, a: _Active, e: Exception):
        self._active.remove(a)
        self.ex.release(a.state)
        self.used -= a.bytes
        a.fut.set_exception(e)

    def _loop(self):
        while True:
            wait_on = None
            with self._cv:
                self._reap_ready()
                self._admit()
                runnable = [a for a in self._active if a.left > 0]
                if not runnable and not self._inflight:
                    if self._stop and not self._queue:
                        return
                    self._cv.wait(timeout=0.001)
                    continue
                if not runnable or len(self._inflight) >= self.max_inflight:
                    wait_on = self._inflight[0][0]
            if wait_on is not None:
                self._h_wait(wait_on)  # outside the lock: clients can submit/stop meanwhile
                continue
            steps = [self.ex.pass_steps(a.state, a.left) for a in runnable]
            try:
                h = self.ex.run_round([a.state for a in runnable], steps)
            except Exception as exc:
                # isolate: run each job's pass alone; only jobs that fail
                # again are failed, the others keep their pass.  Passes the
                # executor reports as already queued are not run again.
                queued = getattr(exc, "launched", None) or []
                ok, ok_steps = [], []
                hs = list(getattr(exc, "handle", None) or [])
                for a, s in zip(runnable, steps):
                    if any(a.state is q for q in queued):
                        ok.append(a)
                        ok_steps.append(s)
                        continue
                    try:
                        hs.append(self.ex.run_round([a.state], [s]))
                        ok.append(a)
                        ok_steps.append(s)
                    except Exception as e:
                        with self._cv:
                            self._fail(a, e)
                runnable, steps = ok, ok_steps
                if not hs:
                    continue
                h = _Joined(hs) if len(hs) > 1 else hs[0]
            self.rounds += 1
            with self._cv:
                fin = []
                for a, s in zip(runnable, steps):
                    a.left -= s
                    if a.left <= 0:
                        self._active.remove(a)
                        fin.append(a)
                self._inflight.append((h, fin))


def latency_stats(done):
    lat = np.array([d.latency for d in done], dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "n": 0}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "n": int(lat.size)}


def run_fifo(executor, jobs, clock=time.perf_counter, t0=None, keep_outputs=True):
    """Baseline: one plan per call.  Jobs run alone in arrival order, each as
    a single library call over all its steps (executor.run_job), and each is
    synchronised before the next starts."""
    t0 = clock() if t0 is None else t0
    done = []
    for job in sorted(jobs, key=lambda j: j.arrival):
        now = clock()
        if job.arrival + t0 > now:
            time.sleep(job.arrival + t0 - now)
        st = executor.prepare(job)
        executor.wait(executor.run_job(st, int(job.steps)))
        fin = clock()
        done.append(Done(job, executor.result(st) if keep_outputs else None, job.arrival + t0,
                         job.arrival + t0, fin))
        executor.release(st)
    return done
