"""Serving loop on the CPU: admission by device-memory budget, continuous
batching and result routing, driven by a fake executor with scripted
latencies (no GPU)."""
import threading
import time
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2606_26547_amd.serve import (AdmissionError, Request, Scheduler, Server, closed_loop, poisson_arrivals,
                                        request_sizes)


class FakeExecutor:
    """Completes a batch `latency(batch)` seconds after launch; the 'labels'
    of a query are a deterministic function of its features."""

    def __init__(self, latency=lambda b: 0.002, fail_model=None, fail_results_model=None):
        self.models = [SimpleNamespace(F=16) for _ in range(3)]
        self.fail_results_model = fail_results_model
        self.released = 0
        self.latency = latency
        self.launched = []
        self.fail_model = fail_model
        self.lock = threading.Lock()
        self.concurrent = 0
        self.max_concurrent = 0

    def launch(self, b):
        if self.fail_model is not None and b.requests[0].model == self.fail_model:
            raise ValueError("bad model")
        with self.lock:
            self.launched.append(b)
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        b.handle = time.perf_counter() + self.latency(b)

    def ready(self, b):
        return time.perf_counter() >= b.handle

    def release(self, b):
        self.released += 1

    def results(self, b):
        with self.lock:
            self.concurrent -= 1
        if self.fail_results_model is not None and b.requests[0].model == self.fail_results_model:
            raise RuntimeError("device error")
        if b.requests[0].kind == "configs":
            return [np.array([len(b.requests[0].cfgs)])]
        return [r.X.astype(np.int64).sum(1) % 7 for r in b.requests]


def req(model, n, seed=0, **kw):
    X = np.random.default_rng(seed).integers(-127, 128, size=(n, 16)).astype(np.int8)
    return Request(model=model, X=X, **kw)


def test_scheduler_admission_respects_budget_and_fifo():
    s = Scheduler(budget=1000, bytes_of=lambda r: r.n * 10, max_batch=1000)
    rs = [req(0, 30, i) for i in range(5)]            # 300 bytes each
    for r in rs:
        s.submit(r)
    b = s.next_batches()
    assert len(b) == 1 and [r.n for r in b[0].requests] == [30, 30, 30]   # 900 of 1000 admitted
    assert s.used == 900 and len(s.waiting) == 2
    s.done(b[0])
    b2 = s.next_batches()
    assert [r for r in b2[0].requests] == rs[3:]
    with pytest.raises(AdmissionError):
        s.submit(req(0, 200))                           # 2000 bytes > budget
    assert s.blocked == 1                               # rs[3] waited at the head of the queue once


def test_closed_loop_keeps_requests_outstanding():
    """Saturation driver: a fixed number of requests stays in flight, each
    completion submits the next; every completed query is counted."""

    class Src:
        def queries(self, n, stream):
            return np.random.default_rng(stream).integers(-127, 128, size=(n, 16)).astype(np.int8), None

    ex = FakeExecutor(latency=lambda b: 0.003)
    srv = Server(ex, budget=10 ** 9, bytes_of=lambda r: r.n)
    q, wall = closed_loop(srv, [Src(), Src(), Src()], concurrency=8, duration=0.3, seed=1, tuned=False, max_n=64)
    srv.close()
    assert wall >= 0.3 and q > 0
    done = sum(c[3] for c in srv.completed)
    assert done >= q                                    # the drained tail completes too
    assert ex.max_concurrent <= 3 * 2                   # three model lanes, depth 2


def test_scheduler_batches_per_lane_with_depth_and_max_batch():
    s = Scheduler(budget=10 ** 9, bytes_of=lambda r: r.n, max_batch=100, depth=2)
    for i in range(6):
        s.submit(req(i % 2, 40, i))
    s.submit(req(0, 40, 99, tuned=True))
    bs = s.next_batches()
    keys = sorted(b.key for b in bs)
    assert keys == [(0, False), (0, True), (1, False)]
    for b in bs:
        assert b.n <= 100
    bs2 = s.next_batches()                              # depth 2: one more batch per busy lane
    assert sorted(b.key for b in bs2) == [(0, False), (1, False)]
    assert s.next_batches() == []                       # both lanes at depth, nothing admitted left
    assert all(s.inflight[k] <= 2 for k in s.inflight)


def test_continuous_batching_joins_running_lane():
    ex = FakeExecutor(latency=lambda b: 0.05)
    srv = Server(ex, budget=10 ** 9, max_batch=10 ** 6, depth=1, bytes_of=lambda r: r.n)
    f0 = srv.submit(req(0, 10, 0))
    time.sleep(0.01)                                    # batch 0 is running
    later = [srv.submit(req(0, 5, i + 1)) for i in range(4)]
    for f in [f0] + later:
        f.result(timeout=5)
    srv.close()
    sizes = [b.n for b in ex.launched]
    assert sizes[0] == 10 and sizes[1] == 20            # the four late requests ran as one batch


def test_results_routed_to_their_requests_and_latency_reported():
    ex = FakeExecutor(latency=lambda b: 0.001 * (1 + b.n / 1000))
    srv = Server(ex, budget=5000, max_batch=300, bytes_of=lambda r: r.n)
    sizes = request_sizes(60, seed=3, max_n=200)
    futs, reqs = [], []
    for i, n in enumerate(sizes):
        r = req(i % 3, int(n), seed=i)
        reqs.append(r)
        futs.append(srv.submit(r))
    for r, f in zip(reqs, futs):
        assert np.array_equal(f.result(timeout=10), r.X.astype(np.int64).sum(1) % 7)
    srv.close()
    rep = srv.latency_report()
    assert rep["requests"] == 60 and rep["queries"] == int(sizes.sum())
    assert rep["p99_ms"] >= rep["p50_ms"] > 0
    assert srv.sched.peak_used <= 5000 and srv.sched.used == 0


def test_config_jobs_run_alone_and_failures_are_isolated():
    ex = FakeExecutor(fail_model=2)
    srv = Server(ex, budget=10 ** 9, bytes_of=lambda r: r.n)
    good = srv.submit(req(0, 8))
    bad = srv.submit(req(2, 8))
    job = srv.submit(req(1, 50, kind="configs", cfgs=[(1024, 1, 0, "int8")] * 3, truth=np.zeros(50)))
    assert good.result(timeout=5).shape == (8,)
    assert job.result(timeout=5)[0] == 3
    with pytest.raises(ValueError):
        bad.result(timeout=5)
    srv.close()
    assert all(len(b.requests) == 1 for b in ex.launched if b.requests[0].kind == "configs")


def test_config_jobs_share_one_lane_of_bounded_depth():
    """Configuration jobs queue on one lane: at most `depth` of them hold a
    staging slot at a time, however many arrive together, and all finish."""
    ex = FakeExecutor(latency=lambda b: 0.01)
    srv = Server(ex, budget=10 ** 9, bytes_of=lambda r: r.n, depth=2)
    jobs = [srv.submit(req(m % 3, 20, seed=m, kind="configs", cfgs=[(1024, 1, 0, "int8")] * (m + 1),
                           truth=np.zeros(20))) for m in range(12)]
    assert [j.result(timeout=10)[0] for j in jobs] == list(range(1, 13))
    srv.close()
    assert ex.max_concurrent <= 2


def test_malformed_requests_are_rejected_at_submit():
    ex = FakeExecutor()
    srv = Server(ex, budget=10 ** 9, bytes_of=lambda r: r.n)
    bad = [Request(model=0, X=np.zeros((4, 15), np.int8)),                      # wrong width
           Request(model=0, X=np.zeros((4, 16), np.float32)),                   # wrong dtype
           Request(model=7, X=np.zeros((4, 16), np.int8)),                      # no such model
           Request(model=0, X=np.zeros((0, 16), np.int8)),                      # empty
           Request(model=1, X=np.zeros((5, 16), np.int8), kind="configs",
                   cfgs=[(1024, 1, 0, "int8")], truth=np.zeros(4)),             # truth length
           Request(model=1, X=np.zeros((5, 16), np.int8), kind="configs", cfgs=[], truth=np.zeros(5))]
    futs = [srv.submit(r) for r in bad]
    for f in futs:
        with pytest.raises(AdmissionError):
            f.result(timeout=5)
    good = srv.submit(req(0, 8))
    assert good.result(timeout=5).shape == (8,)
    srv.close()
    assert len(ex.launched) == 1 and srv.sched.used == 0


def test_failed_completion_fails_its_requests_and_the_loop_goes_on():
    ex = FakeExecutor(fail_results_model=1)
    srv = Server(ex, budget=10 ** 9, bytes_of=lambda r: r.n)
    bad = srv.submit(req(1, 8))
    with pytest.raises(RuntimeError):
        bad.result(timeout=5)
    good = srv.submit(req(0, 8))                        # the loop thread is still alive
    assert good.result(timeout=5).shape == (8,)
    srv.close()
    assert ex.released == 1 and srv.sched.used == 0


def test_tight_budget_still_completes_everything():
    ex = FakeExecutor(latency=lambda b: 0.002)
    srv = Server(ex, budget=100, max_batch=1000, bytes_of=lambda r: r.n)
    futs = [srv.submit(req(i % 2, 40, i)) for i in range(20)]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert srv.sched.peak_used <= 100


def test_arrival_process_and_sizes():
    t = poisson_arrivals(2000.0, 1.0, seed=1)
    assert 1800 < t.size < 2200 and np.all(np.diff(t) > 0)
    n = request_sizes(10000, seed=2)
    assert n.min() >= 1 and n.max() <= 4096
    assert 300 < n.mean() < 700                          # log-uniform on [1, 4096]: mean ~ 492


def test_automatic_gc_is_off_while_serving_and_restored():
    """Automatic cyclic collection stops while servers run (the loop collects
    the young generations itself) and comes back after the last one closes."""
    import gc
    assert gc.isenabled()
    a = Server(FakeExecutor(), budget=10 ** 9, bytes_of=lambda r: r.n)
    b = Server(FakeExecutor(), budget=10 ** 9, bytes_of=lambda r: r.n)
    assert not gc.isenabled()
    assert a.submit(req(0, 4)).result(timeout=5).shape == (4,)
    a.close()
    assert not gc.isenabled()                       # b still runs
    b.close()
    b.close()                                       # a second close changes nothing
    assert gc.isenabled()


def test_gpu_executor_staging_copy():
    """The executor's staging copy writes each request at its offset, as
    one plain copy would, and leaves the pad columns (which the kernels
    ignore) alone."""
    import torch

    from paper_2606_26547_amd.serve import GpuExecutor
    ex = GpuExecutor.__new__(GpuExecutor)          # no device needed for the host copy
    ex.torch = torch
    g = np.random.default_rng(0)
    reqs = [SimpleNamespace(n=n, X=g.integers(-127, 128, size=(n, 37)).astype(np.int8)) for n in (1, 250, 9, 1000)]
    offs = list(np.cumsum([0] + [r.n for r in reqs])[:-1])
    b = SimpleNamespace(requests=reqs, offsets=offs, n=sum(r.n for r in reqs))
    hxt = torch.full((b.n, 64), 7, dtype=torch.int8)
    ex._stage(hxt, b, 37, 64)
    ref = np.full((b.n, 64), 7, np.int8)
    ref[:, :37] = np.concatenate([r.X for r in reqs])
    assert np.array_equal(hxt.numpy(), ref)
