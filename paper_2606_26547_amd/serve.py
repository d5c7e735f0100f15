"""Continuous-batching serving loop over resident HDC models.

Requests are either inference (classify n query vectors with one model under
its plain or tuned configuration) or configuration-evaluation jobs (run a
list of approximation configurations on labelled queries in one persistent
launch: the tuner's inner loop, Sec. 3 / 4.1 of the paper).

Structure
---------
* ``Scheduler``: admission and batching only (no device code), so it can be
  tested on the CPU with a fake executor.  A request is admitted when its
  device bytes fit in the HBM budget left after the resident models; admitted
  inference requests for the same (model, configuration) are packed into a
  batch of at most ``max_batch`` queries the next time that lane is free —
  requests that arrive while earlier batches run join the next batch
  (continuous batching, not a queue of whole requests).  Bytes are released
  when the batch completes.
* ``GpuExecutor``: one HIP stream per model plus one for configuration jobs;
  a batch is an async H2D copy from pinned staging, one fused-classifier
  launch (``hdc_classify_prepared``) and an async D2H copy of the labels,
  closed by an event.  Batches of different models overlap on the device;
  configuration jobs run on a capped number of workgroups beside them.
* ``Server``: the scheduler thread that drives both and completes futures
  with per-request latency (arrival -> labels on the host).
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import threading
import time
from concurrent.futures import Future

import numpy as np

# Largest configuration job a slot holds results for (the sweep's own limit).
MAX_JOB_CONFIGS = 4096


# ---------------------------------------------------------------- requests
@dataclasses.dataclass
class Request:
    model: int
    X: np.ndarray                      # [n][F] int8 queries
    tuned: bool = False
    kind: str = "infer"                # "infer" | "configs"
    cfgs: list | None = None           # configs job: [(d_trunc, stride, start, dtype)]
    truth: np.ndarray | None = None    # configs job: labels
    t_arrival: float = 0.0
    future: Future = dataclasses.field(default_factory=Future)
    rid: int = 0

    @property
    def n(self) -> int:
        return int(self.X.shape[0])


@dataclasses.dataclass
class Batch:
    key: tuple                          # (model, tuned) or ("configs",)
    requests: list
    offsets: list
    n: int
    nbytes: int
    handle: object = None


class AdmissionError(ValueError):
    pass


class Scheduler:
    """Admission by device-memory budget and continuous batching per lane.

    ``bytes_of(request)`` gives the device bytes a request holds while it is
    in flight; ``budget`` is what is left of the HBM budget after the
    resident models.  A lane is (model, tuned) for inference, and one lane
    holds the configuration jobs (one job per batch: they run one after the
    other on the executor's configuration stream anyway, so more in flight
    would only hold staging slots); each lane has at most ``depth`` batches
    in flight."""

    def __init__(self, budget: int, bytes_of, max_batch: int = 16384, depth: int = 2):
        self.budget = int(budget)
        self.bytes_of = bytes_of
        self.max_batch = int(max_batch)
        self.depth = int(depth)
        self.used = 0
        self.waiting = collections.deque()          # arrived, not yet admitted (FIFO)
        self.admitted = collections.defaultdict(collections.deque)   # lane -> requests
        self.inflight = collections.defaultdict(int)                  # lane -> batches in flight
        self.peak_used = 0
        self.blocked = 0                            # requests that waited for budget at the queue head

    def lane(self, r: Request):
        return ("configs",) if r.kind == "configs" else (r.model, bool(r.tuned))

    def submit(self, r: Request):
        need = self.bytes_of(r)
        if need > self.budget:
            raise AdmissionError("request needs %d device bytes, budget is %d" % (need, self.budget))
        self.waiting.append(r)

    def admit(self):
        """Admit waiting requests in arrival order while they fit."""
        while self.waiting:
            r = self.waiting[0]
            need = self.bytes_of(r)
            if self.used + need > self.budget:
                if not getattr(r, "blocked", False):
                    r.blocked = True
                    self.blocked += 1
                break
            self.waiting.popleft()
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            self.admitted[self.lane(r)].append(r)

    def next_batches(self) -> list[Batch]:
        """Form one batch for every lane that has admitted work and a free slot."""
        self.admit()
        out = []
        for lane, q in self.admitted.items():
            if not q or self.inflight[lane] >= self.depth:
                continue
            reqs, offs, n, nb = [], [], 0, 0
            while q and (not reqs or n + q[0].n <= self.max_batch) and q[0].kind == "infer":
                r = q.popleft()
                reqs.append(r)
                offs.append(n)
                n += r.n
                nb += self.bytes_of(r)
            if not reqs:                                    # a configuration job runs alone
                r = q.popleft()
                reqs, offs, n, nb = [r], [0], r.n, self.bytes_of(r)
            self.inflight[lane] += 1
            out.append(Batch(lane, reqs, offs, n, nb))
        return out

    def done(self, b: Batch):
        self.inflight[b.key] -= 1
        self.used -= b.nbytes

    def idle(self) -> bool:
        return not self.waiting and not any(self.admitted.values()) and not any(self.inflight.values())


# ---------------------------------------------------------------- executor
class GpuExecutor:
    """Resident models and per-model streams; runs batches asynchronously.

    Every batch, inference or configuration job, runs out of a staging slot
    (pinned host + device buffers for the queries, labels or truth, and the
    per-configuration results, sized for ``max_batch`` queries of the widest
    model).  The pool is allocated up front for every batch the scheduler
    can have in flight (``depth`` per model lane and per configuration job
    in flight, plus headroom), because a pinned allocation of a new slot
    takes milliseconds and stalls every request behind it; it still grows
    if more are ever needed.  The queries are copied into the slot's pinned
    buffer, then one H2D copy, the launch and one D2H copy are queued on the
    lane's stream and closed by the slot's event."""

    def __init__(self, models, device="cuda", max_batch: int = 16384, job_workgroups: int = 64,
                 slots: int | None = None, depth: int = 2):
        import torch

        from . import hdc
        self.torch, self.hdc = torch, hdc
        self.dev = device
        self.max_batch = max_batch
        # configuration jobs run persistent kernels: cap their workgroups so
        # that inference batches on the other streams still find free units
        self.job_workgroups = job_workgroups
        self.models = []
        self.streams = []
        for m in models:
            self.models.append(m)
            self.streams.append(torch.cuda.Stream(device=device))
        self.cfg_stream = torch.cuda.Stream(device=device)
        self.resident_bytes = sum(m.resident_bytes for m in models)
        self.ld_max = max(m.P.shape[1] for m in models)
        self.free = collections.deque()
        self.nslots = 0
        if slots is None:
            # every lane of one mode (plain or tuned) and the configuration lane
            slots = depth * (len(models) + 1) + 2
        for _ in range(slots):
            self.free.append(self._new_slot())

    def warm(self, job_cfgs=None, tune_tiles: bool = False):
        """Run every kernel the server will use once (each model's plain and
        tuned classifier, and its configuration sweep when ``job_cfgs(m)``
        is given), so that first-launch costs stay out of request latency.
        With ``tune_tiles`` the tile autotuner first picks the tiles of each
        model's classifier (at a mid-size batch) and sweep buckets; the
        choices are returned."""
        torch, hdc = self.torch, self.hdc
        choices = []
        if tune_tiles:
            from . import autotune as AT
            shapes, seen = [], set()
            for i, m in enumerate(self.models):
                for sh in [AT.Shape("classify", m.F, m.K, m.D, 2048, compute=m.plain.compute)] + \
                        ([AT.Shape("sweep", m.F, m.K, m.D, 512, cfgs=job_cfgs(i))] if job_cfgs else []):
                    key = (sh.kind, sh.F, sh.K, sh.D, sh.compute)
                    if key not in seen:
                        seen.add(key)
                        shapes.append(sh)
            choices = AT.autotune(shapes, reps=3)
            table = AT.TileTable.from_choices(choices)
            for m in self.models:
                m.plain.tile = table.get("classify", "int8", m.plain.compute, m.F, m.K)
                if m.tuned.compute == m.plain.compute:
                    m.tuned.tile = m.plain.tile
                m.sweep_tile = table.get("sweep", "int8", "int8", m.F, m.K)
        for i, m in enumerate(self.models):
            X = torch.zeros((64, m.P.shape[1]), dtype=torch.int8, device=self.dev)
            m.plain(X, m.F, m.plain.P)
            m.tuned(X, m.F, m.tuned.P)
            if job_cfgs is not None:
                y = torch.zeros(64, dtype=torch.int32, device=self.dev)
                hdc.eval_configs(X, m.F, y, m.P, m.D, m.C, job_cfgs(i), ws=m.sweep_ws,
                                 max_workgroups=self.job_workgroups, tile=m.sweep_tile)
        torch.cuda.synchronize()
        return choices

    def _new_slot(self):
        torch = self.torch
        self.nslots += 1
        n, ld = self.max_batch, self.ld_max
        return {"hx": torch.empty(n * ld, dtype=torch.int8, pin_memory=True),
                "dx": torch.empty(n * ld, dtype=torch.int8, device=self.dev),
                "hl": torch.empty(n, dtype=torch.int32, pin_memory=True),   # labels / truth
                "dl": torch.empty(n, dtype=torch.int32, device=self.dev),
                # per-configuration results (hdc_config_result records)
                "hc": torch.empty(MAX_JOB_CONFIGS * 16, dtype=torch.uint8, pin_memory=True),
                "ev": torch.cuda.Event()}

    def _stage(self, hxt, b: Batch, F: int, ld: int):
        """Copy the batch's queries into the slot's page-locked rows, on the
        scheduling thread.  The pad columns [F, ld) keep whatever the slot
        held: the kernels read them but ignore them.  (Handing large copies
        to torch's multithreaded copy raised the closed-loop capacity by half
        but its worker threads starved the loop: the open-loop p99 went from
        0.7 ms to 1.4-20 ms.)"""
        hx = hxt.numpy()
        for r, off in zip(b.requests, b.offsets):
            hx[off:off + r.n, :F] = r.X

    @staticmethod
    def request_bytes(r: Request, F: int) -> int:
        ld = max(64, (F + 63) // 64 * 64)
        return r.n * (ld + 4) + (1 << 12)

    def launch(self, b: Batch):
        torch, hdc = self.torch, self.hdc
        r0 = b.requests[0]
        m = self.models[r0.model]
        if b.n > self.max_batch:
            raise ValueError("batch of %d queries exceeds max_batch %d" % (b.n, self.max_batch))
        if r0.kind == "configs" and len(r0.cfgs) > MAX_JOB_CONFIGS:
            raise ValueError("configuration job of %d configurations exceeds %d" % (len(r0.cfgs), MAX_JOB_CONFIGS))
        slot = self.free.popleft() if self.free else self._new_slot()
        try:
            self._enqueue(b, m, slot)
        except BaseException:
            # nothing of this batch reached the device queue in a state
            # that still uses the slot: hand it back before failing
            self.free.append(slot)
            raise

    def _enqueue(self, b: Batch, m, slot):
        torch, hdc = self.torch, self.hdc
        r0 = b.requests[0]
        ld = m.P.shape[1]
        hxt = slot["hx"][:b.n * ld].view(b.n, ld)
        self._stage(hxt, b, m.F, ld)
        if r0.kind == "configs":
            nc = len(r0.cfgs)
            slot["hl"].numpy()[:b.n] = r0.truth
            with torch.cuda.stream(self.cfg_stream):
                dx = slot["dx"][:b.n * ld].view(b.n, ld)
                dx.copy_(hxt, non_blocking=True)
                truth = slot["dl"][:b.n]
                truth.copy_(slot["hl"][:b.n], non_blocking=True)
                hdc.eval_configs(dx, m.F, truth, m.P, m.D, m.C, r0.cfgs, ws=m.sweep_ws,
                                 max_workgroups=self.job_workgroups, tile=m.sweep_tile, out=slot["hc"])
                slot["ev"].record(self.cfg_stream)
            b.handle = ("configs", slot, nc)
            return
        stream = self.streams[r0.model]
        with torch.cuda.stream(stream):
            dx = slot["dx"][:b.n * ld].view(b.n, ld)
            dx.copy_(hxt, non_blocking=True)
            prep = m.tuned if r0.tuned else m.plain
            prep(dx, m.F, prep.P, slot["dl"][:b.n])
            slot["hl"][:b.n].copy_(slot["dl"][:b.n], non_blocking=True)
            slot["ev"].record(stream)
        b.handle = ("infer", slot)

    def ready(self, b: Batch) -> bool:
        return b.handle[1]["ev"].query()

    def release(self, b: Batch):
        """Return a launched batch's slot after its work failed (the slot is
        reused only once its event has completed)."""
        if b.handle is not None:
            slot = b.handle[1]
            try:
                slot["ev"].synchronize()
            finally:
                self.free.append(slot)
            b.handle = None

    def results(self, b: Batch):
        h = b.handle
        slot = h[1]
        slot["ev"].synchronize()
        try:
            if h[0] == "configs":
                out = [self.hdc.result_view(slot["hc"], h[2])["correct"].copy()]
            else:
                res = slot["hl"].numpy()
                out = [res[off:off + r.n].copy() for r, off in zip(b.requests, b.offsets)]
        finally:
            b.handle = None
            self.free.append(slot)
        return out


class ResidentModel:
    """A model kept on the device: projection, class hypervectors and the
    prepared class operands of its plain and tuned configurations."""

    def __init__(self, P: np.ndarray, X_train: np.ndarray, y_train: np.ndarray, K: int,
                 tuned_cfg=None, device="cuda", max_job_cfgs: int = 64):
        import torch

        from . import hdc
        self.D, self.F, self.K = int(P.shape[0]), int(P.shape[1]), int(K)
        self.P = hdc.pad_cols(P, device)
        # int8 and E4M3 configurations classify on the shifted projection
        # (weights p + 1, the same labels) where its kernels take the
        # model's shape: compute type -> that form of the projection
        self.shifted = {t: hdc.shift_projection(self.P, self.F, compute=ts) for t, ts in hdc.SHIFTED.items()
                        if hdc.shift_supported("classify", self.F, self.K, ts)}
        Xtr = hdc.pad_cols(X_train, device)
        H = hdc.encode(Xtr, self.F, self.P, self.D)
        self.C, _ = hdc.bundle(H, self.D, torch.as_tensor(y_train, dtype=torch.int32).to(device), self.K)
        del H, Xtr
        self.plain = self.prepared((self.D, 1, 0, "int8"))
        self.sweep_tile = 0       # work-item shape of configuration jobs (0: built-in)
        self.tuned_cfg = tuned_cfg or (self.D, 1, 0, "int8")
        self.tuned = self.prepared(self.tuned_cfg)
        # workspace of configuration jobs (up to max_job_cfgs configurations)
        need = int(hdc.lib().hdc_eval_configs_workspace_bytes(max_job_cfgs, self.F, self.D, self.K))
        self.sweep_ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
        self.resident_bytes = (self.P.numel() + sum(p.numel() for p in self.shifted.values())
                               + self.C.numel() * 8 + self.plain.ws.numel() + self.tuned.ws.numel()
                               + self.sweep_ws.numel())

    def prepared(self, cfg, tile: int = 0):
        """The prepared classifier of configuration ``cfg``; its attribute P
        is the projection it reads (the shifted one for int8 / E4M3 where the
        model has it).  ``tile`` applies to int8 configurations."""
        from . import hdc
        d, k, s, t = cfg
        if t in self.shifted:
            prep = hdc.Prepared(self.C, self.D, hdc.SHIFTED[t], s, d, k, tile=tile if t == "int8" else 0)
            prep.P = self.shifted[t]
        else:
            prep = hdc.Prepared(self.C, self.D, t, s, d, k, tile=tile if t == "int8" else 0)
            prep.P = self.P
        return prep

    def set_tuned(self, cfg):
        self.tuned_cfg = cfg
        self.tuned = self.prepared(cfg, tile=self.plain.tile)


# ---------------------------------------------------------------- server
# Automatic cyclic collection is off while any server runs (see Server).
_gc_lock = threading.Lock()
_gc_servers = 0
_gc_was_enabled = True


def _gc_hold():
    global _gc_servers, _gc_was_enabled
    with _gc_lock:
        if _gc_servers == 0:
            _gc_was_enabled = gc.isenabled()
            gc.disable()
        _gc_servers += 1


def _gc_release():
    global _gc_servers
    with _gc_lock:
        _gc_servers -= 1
        if _gc_servers == 0 and _gc_was_enabled:
            gc.enable()


class Server:
    """Scheduler thread: admits, batches, launches and completes requests."""

    def __init__(self, executor, budget: int, max_batch: int = 16384, depth: int = 2,
                 bytes_of=None, poll_s: float = 1e-5):
        self.ex = executor
        if bytes_of is None:
            bytes_of = lambda r: GpuExecutor.request_bytes(r, executor.models[r.model].F)  # noqa: E731
        self.sched = Scheduler(budget, bytes_of, max_batch, depth)
        self.lock = threading.Lock()
        self.running = []
        self.stop_flag = False
        self.poll_s = poll_s
        self.next_id = 0
        self.completed = []                 # (rid, kind, model, n, latency_s)
        # longest pass of the scheduling loop, and passes over 10 ms (a
        # stalled loop delays every request behind it)
        self.max_loop_s = 0.0
        self.loop_stalls = 0
        self.closed = False
        # The cyclic collector.  Everything allocated so far (models, pools,
        # staging) lives as long as the server: it is moved out of the
        # collector's view.  While the server runs, the interpreter's
        # automatic collections are off: under a steady request stream they
        # reach the oldest generation every few seconds, and a pass over
        # every live request, future and result there stopped the loop for
        # hundreds of milliseconds.  The loop collects the young generations
        # itself instead (their size is bounded by the work of the last
        # interval, so each pass is short); when the last running server is
        # closed, the automatic collector is turned back on if it was on.
        gc.collect()
        gc.freeze()
        _gc_hold()
        self.gc_young_s, self.gc_mid_s = 0.05, 1.0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def validate(self, r: Request):
        """Reject a malformed request before it is admitted: queries must be
        an [n][F] int8 array of the model's feature width, and a
        configuration job needs one true label per query."""
        models = self.ex.models
        if not 0 <= r.model < len(models):
            raise AdmissionError("model %d does not exist" % r.model)
        F = models[r.model].F
        X = r.X
        if not isinstance(X, np.ndarray) or X.dtype != np.int8 or X.ndim != 2 or X.shape[1] != F:
            raise AdmissionError("queries must be an int8 array of shape [n][%d]" % F)
        if X.shape[0] < 1:
            raise AdmissionError("a request needs at least one query")
        if r.kind == "configs":
            if not r.cfgs or len(r.cfgs) > MAX_JOB_CONFIGS:
                raise AdmissionError("a configuration job needs 1..%d configurations" % MAX_JOB_CONFIGS)
            if r.truth is None or np.asarray(r.truth).shape != (X.shape[0],):
                raise AdmissionError("a configuration job needs one true label per query")
        elif r.kind != "infer":
            raise AdmissionError("unknown request kind %r" % r.kind)

    def submit(self, r: Request) -> Future:
        with self.lock:
            r.t_arrival = r.t_arrival or time.perf_counter()
            r.rid = self.next_id
            self.next_id += 1
            try:
                self.validate(r)
                self.sched.submit(r)
            except AdmissionError as e:
                r.future.set_exception(e)
        return r.future

    def _loop(self):
        t_prev = time.perf_counter()
        t_young = t_mid = t_prev
        while True:
            t_now = time.perf_counter()
            gap = t_now - t_prev
            t_prev = t_now
            if gap > self.max_loop_s:
                self.max_loop_s = gap
            if gap > 0.01:
                self.loop_stalls += 1
            if t_now - t_mid > self.gc_mid_s:
                gc.collect(1)
                t_mid = t_young = t_now
            elif t_now - t_young > self.gc_young_s:
                gc.collect(0)
                t_young = t_now
            with self.lock:
                batches = self.sched.next_batches()
                stopping = self.stop_flag and self.sched.idle() and not self.running
            if stopping:
                return
            for b in batches:
                try:
                    self.ex.launch(b)
                    self.running.append(b)
                except Exception as e:   # a malformed request fails alone
                    for r in b.requests:
                        r.future.set_exception(e)
                    with self.lock:
                        self.sched.done(b)
            still = []
            for b in self.running:
                try:
                    if not self.ex.ready(b):
                        still.append(b)
                        continue
                    res = self.ex.results(b)
                except Exception as e:   # a failed batch fails its own requests only
                    try:
                        self.ex.release(b)
                    except Exception:
                        pass
                    with self.lock:
                        self.sched.done(b)
                    for r in b.requests:
                        if not r.future.done():
                            r.future.set_exception(e)
                    continue
                now = time.perf_counter()
                with self.lock:
                    self.sched.done(b)
                for r, v in zip(b.requests, res):
                    self.completed.append((r.rid, r.kind, r.model, r.n, now - r.t_arrival))
                    r.future.set_result(v)
            self.running = still
            if not batches and still:
                time.sleep(self.poll_s)
            elif not batches and not still:
                time.sleep(self.poll_s)

    def close(self, timeout: float = 60.0):
        self.stop_flag = True
        self.thread.join(timeout)
        if not self.closed:
            self.closed = True
            _gc_release()

    def latency_report(self, kind="infer"):
        lat = np.array([c[4] for c in self.completed if c[1] == kind])
        if lat.size == 0:
            return {}
        return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "queries": int(sum(c[3] for c in self.completed if c[1] == kind))}


def open_loop(server: Server, sources, rate: float, duration: float, seed: int, tuned: bool,
              job_frac: float = 0.05, job_cfgs=None, job_queries: int = 512, max_n: int = 4096):
    """Drive ``server`` with an open-loop Poisson stream: arrivals are
    submitted at their scheduled times regardless of completions (so queueing
    shows up in the latency instead of being hidden).  ``sources[m]`` has
    ``queries(n, stream) -> (X, y)``.  Returns the futures with their requests."""
    from .datagen import rng
    t_arr = poisson_arrivals(rate, duration, seed)
    sizes = request_sizes(t_arr.size, seed, max_n)
    g = rng(seed, 13)
    models = g.integers(0, len(sources), size=t_arr.size)
    is_job = g.random(t_arr.size) < job_frac
    pool = {}
    for m, src in enumerate(sources):                   # pre-drawn query pools per model
        pool[m] = src.queries(max_n, 100 + m)
    out = []
    t0 = time.perf_counter()
    for i, ta in enumerate(t_arr):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        m = int(models[i])
        X, y = pool[m]
        if is_job[i]:
            n = min(job_queries, X.shape[0])
            r = Request(model=m, X=X[:n], kind="configs", cfgs=job_cfgs(m), truth=y[:n])
        else:
            n = int(sizes[i])
            off = int(g.integers(0, X.shape[0] - n + 1))
            r = Request(model=m, X=X[off:off + n], tuned=tuned)
        r.t_arrival = t0 + ta
        out.append((r, server.submit(r)))
    return out


def closed_loop(server: Server, sources, concurrency: int, duration: float, seed: int, tuned: bool,
                max_n: int = 4096, fixed_n: int | None = None):
    """Drive ``server`` at saturation: ``concurrency`` inference requests
    (log-uniform sizes up to ``max_n``, or all of ``fixed_n`` queries; random
    models) are kept outstanding for ``duration`` seconds, a new one
    submitted as each completes.  Returns (completed queries, wall seconds)."""
    import concurrent.futures as cf

    from .datagen import rng
    g = rng(seed, 14)
    pool = {m: src.queries(max_n, 200 + m)[0] for m, src in enumerate(sources)}

    def new_request():
        m = int(g.integers(0, len(sources)))
        n = fixed_n if fixed_n else int(np.floor(np.exp(g.uniform(0, np.log(max_n + 1)))).clip(1, max_n))
        off = int(g.integers(0, max_n - n + 1))
        return server.submit(Request(model=m, X=pool[m][off:off + n], tuned=tuned)), n

    out = dict(new_request() for _ in range(concurrency))
    done_q, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < duration:
        finished, _ = cf.wait(list(out), timeout=1.0, return_when=cf.FIRST_COMPLETED)
        for f in finished:
            f.result()
            done_q += out.pop(f)
            fut, n = new_request()
            out[fut] = n
    wall = time.perf_counter() - t0
    for f in list(out):
        f.result(timeout=300)
    return done_q, wall


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds) of a Poisson process."""
    from .datagen import rng
    g = rng(seed, 11)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def request_sizes(count: int, seed: int, max_n: int = 4096) -> np.ndarray:
    """Log-uniform request sizes in [1, max_n]."""
    from .datagen import rng
    g = rng(seed, 12)
    return np.floor(np.exp(g.uniform(0, np.log(max_n + 1), size=count))).astype(int).clip(1, max_n)
