"""Scheduler logic of the continuous-batching server, run on the CPU with a
simulated executor (no arithmetic: it only accounts for passes and time).
Failures are forced from the host."""
import threading
import time

import pytest

from paper_2603_00477_amd.serve import Job, StencilServer, latency_stats, run_fifo


class FakeExecutor:
    def __init__(self, pass_time=0.002, T=2, fail_prepare=(), fail_round_with=None):
        self.pass_time = pass_time
        self.T = T
        self.fail_prepare = set(fail_prepare)
        self.fail_round_with = fail_round_with
        self.rounds = []
        self.live = 0
        self.peak = 0
        self.lock = threading.Lock()
        self.order = []
        self.device_free_at = 0.0  # rounds execute one after another, like a stream
        self.whole_jobs = []

    def footprint(self, job):
        if job.dims is None:
            raise ValueError("bad job")
        return int(job.dims[0])

    def prepare(self, job):
        if job.id in self.fail_prepare:
            raise RuntimeError(f"prepare failed for {job.id}")
        with self.lock:
            self.live += self.footprint(job)
            self.peak = max(self.peak, self.live)
        self.order.append(job.id)
        return {"job": job, "passes": 0, "bytes": self.footprint(job)}

    def pass_steps(self, st, left):
        return min(self.T, left)

    def run_round(self, states, steps):
        ids = [s["job"].id for s in states]
        if self.fail_round_with is not None and self.fail_round_with in ids:
            raise RuntimeError("device error")
        self.rounds.append(ids)
        for s in states:
            s["passes"] += 1
        start = max(time.perf_counter(), self.device_free_at)
        self.device_free_at = start + self.pass_time * len(states)
        return self.device_free_at

    def run_job(self, st, steps):
        """One call over all of a job's steps (the one-plan-per-call form)."""
        self.whole_jobs.append((st["job"].id, steps))
        st["passes"] += -(-steps // self.T)
        start = max(time.perf_counter(), self.device_free_at)
        self.device_free_at = start + self.pass_time * (-(-steps // self.T))
        return self.device_free_at

    def done(self, h):
        return time.perf_counter() >= h

    def wait(self, h):
        dt = h - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def result(self, st):
        return ("out", st["job"].id, st["passes"])

    def release(self, st):
        with self.lock:
            self.live -= st["bytes"]


def _job(i, size=10, steps=5, **kw):
    return Job(shape="box", d=2, r=1, weights=None, dims=(size, size), steps=steps, id=i, **kw)


def test_all_jobs_complete_with_right_pass_count():
    ex = FakeExecutor()
    srv = StencilServer(ex, hbm_budget=100).start()
    futs = [srv.submit(_job(i, steps=1 + i % 7)) for i in range(30)]
    res = [f.result(timeout=30) for f in futs]
    srv.stop()
    for i, d in enumerate(res):
        assert d.output == ("out", i, -(-(1 + i % 7) // 2))
        assert d.latency >= 0 and d.finished >= d.admitted >= d.arrival - 1e-9
    assert ex.peak <= 100
    assert ex.live == 0 and srv.used == 0
    assert latency_stats(srv.done)["n"] == 30


def test_budget_limits_residency_and_fifo_admission():
    ex = FakeExecutor(pass_time=0.003)
    srv = StencilServer(ex, hbm_budget=25).start()
    futs = [srv.submit(_job(i, size=10, steps=4)) for i in range(10)]
    for f in futs:
        f.result(timeout=30)
    srv.stop()
    assert ex.peak <= 25
    assert ex.order == list(range(10))  # admitted in arrival order
    assert max(len(r) for r in ex.rounds) == 2  # at most two resident at once


def test_oversize_job_rejected_others_run():
    ex = FakeExecutor()
    srv = StencilServer(ex, hbm_budget=50).start()
    big = srv.submit(_job("big", size=60))
    ok = srv.submit(_job("ok", size=10))
    with pytest.raises(MemoryError):
        big.result(timeout=10)
    assert ok.result(timeout=10).output[1] == "ok"
    srv.stop()


def test_invalid_and_failing_jobs_isolated():
    ex = FakeExecutor(fail_prepare={"p"}, fail_round_with="r")
    srv = StencilServer(ex, hbm_budget=1000).start()
    bad = srv.submit(Job(shape="box", d=2, r=1, weights=None, dims=None, steps=3, id="bad"))
    p = srv.submit(_job("p"))
    time.sleep(0.05)
    r = srv.submit(_job("r", steps=2))
    after = srv.submit(_job("after", steps=3))
    with pytest.raises(ValueError):
        bad.result(timeout=10)
    with pytest.raises(RuntimeError):
        p.result(timeout=10)
    with pytest.raises(RuntimeError):
        r.result(timeout=10)
    assert after.result(timeout=10).output[1] == "after"
    srv.stop()
    assert srv.used == 0


class PartialExecutor(FakeExecutor):
    """A round whose later part fails after its first job's pass was queued
    (as a multi-stream executor reports it)."""

    def run_round(self, states, steps):
        ids = [s["job"].id for s in states]
        if self.fail_round_with in ids and len(states) > 1:
            first = states[0]
            h = FakeExecutor.run_round(self, [first], steps[:1])
            e = RuntimeError("device error in a later group")
            e.launched, e.handle = [first], [h]
            raise e
        return FakeExecutor.run_round(self, states, steps)


def test_partially_launched_round_is_not_run_twice():
    ex = PartialExecutor(pass_time=0.002, T=1, fail_round_with="r")
    srv = StencilServer(ex, hbm_budget=1000)
    ok = srv.submit(_job("ok", steps=4))
    r = srv.submit(_job("r", steps=3))
    srv.start()
    assert ok.result(timeout=10).output == ("out", "ok", 4)  # exactly one pass per step
    with pytest.raises(RuntimeError):
        r.result(timeout=10)
    srv.stop()
    assert srv.used == 0


def test_continuous_batching_late_arrivals_join_running_rounds():
    ex = FakeExecutor(pass_time=0.002, T=1)
    srv = StencilServer(ex, hbm_budget=1000).start()
    long = srv.submit(_job("long", steps=60))
    time.sleep(0.03)
    late = [srv.submit(_job(f"late{i}", steps=2)) for i in range(5)]
    res_late = [f.result(timeout=10) for f in late]
    res_long = long.result(timeout=10)
    srv.stop()
    # the late jobs finished while the long job was still running ...
    assert max(d.finished for d in res_late) < res_long.finished
    # ... and shared rounds with it
    assert any("long" in r and any(str(x).startswith("late") for x in r) for r in ex.rounds)


def test_stop_without_drain_cancels_queued():
    ex = FakeExecutor(pass_time=0.01, T=1)
    srv = StencilServer(ex, hbm_budget=10).start()
    first = srv.submit(_job("a", size=10, steps=20))
    queued = [srv.submit(_job(f"q{i}", size=10)) for i in range(3)]
    time.sleep(0.02)
    srv.stop(drain=False)
    assert first.result(timeout=10).output[1] == "a"
    assert all(q.cancelled() for q in queued)


def test_fifo_baseline_runs_jobs_alone():
    ex = FakeExecutor(pass_time=0.001)
    jobs = [_job(i, steps=3) for i in range(5)]
    for i, j in enumerate(jobs):
        j.arrival = 0.001 * i
    done = run_fifo(ex, jobs)
    assert [d.job.id for d in done] == list(range(5))
    # one library call per job over all its steps, no rounds
    assert ex.whole_jobs == [(i, 3) for i in range(5)] and ex.rounds == []
    assert [d.output for d in done] == [("out", i, 2) for i in range(5)]


class Output:
    """A result grid stand-in that supports weak references."""

    def __init__(self, job_id, passes):
        self.id, self.passes = job_id, passes


class HoldingExecutor(FakeExecutor):
    """Reports the size of each job's result grid, so the server keeps it
    counted against the budget until the caller drops it."""

    def output_bytes(self, job):
        return int(job.dims[0]) // 2

    def result(self, st):
        return Output(st["job"].id, st["passes"])


def test_outputs_held_by_callers_count_against_the_budget():
    import gc

    ex = HoldingExecutor(pass_time=0.001)
    srv = StencilServer(ex, hbm_budget=25).start()
    a = srv.submit(_job("a", size=10, steps=2)).result(timeout=10)
    b = srv.submit(_job("b", size=10, steps=2)).result(timeout=10)
    # two outputs of 5 bytes held: 10 of 25 used, a job of footprint 10 fits ...
    assert srv.used == 10 and srv.held == 10
    c = srv.submit(_job("c", size=10, steps=2)).result(timeout=10)
    assert srv.used == 15
    # ... but not one of footprint 16: admission blocks while the outputs are held
    blocked = srv.submit(_job("d", size=16, steps=2))
    time.sleep(0.1)
    assert not blocked.done() and "d" not in ex.order
    del a
    gc.collect()
    time.sleep(0.1)
    assert not blocked.done()  # 15 - 5 = 10 used: 10 + 16 > 25 still
    del b
    gc.collect()
    d = blocked.result(timeout=10)
    assert d.output.id == "d" and srv.used == 5 + 8
    del c, d, blocked  # the future holds the result too
    gc.collect()
    srv.stop()
    assert srv.used == 0 and srv.held == 0
