"""Request loop for denoising jobs of different cube sizes.

Jobs arrive over time (cube, radii, range, omega, tolerance, cap). The
server keeps every admitted job's primal/dual state on the device in the
job's own workspace. It admits waiting jobs first come, first served while
their HBM footprint (workspace + cube) fits the budget. It advances all
admitted jobs together in rounds of batched iterations (geo_batch_step: one
launch sequence per iteration for every job, replayed from a HIP graph). A
job leaves when its stopping rule (eq. (28)) holds or its cap is reached:
u, s and t are copied to the host and its memory is released. Every job's
iterates are exactly those of the same job run alone, because batching
changes no per-cube arithmetic. A job whose iterates turn non-finite is
retired with an error and no result; the others go on.

Copies overlap the rounds. A helper thread copies the cubes of the first
jobs in line into pinned host memory; at admission the cube goes to the device and its state
is initialised on a second stream (default priority), which the next round
waits for on the device only. A finished job's u, s, t are read out of its
workspace on the round's stream and copied to pinned host memory on the
second stream while the next rounds run; a second helper thread stamps the
moment each copy completes and moves the result out of pinned memory.

Timing is wall clock: a job's latency runs from its arrival to the moment
its result is on the host.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import threading
import time
from collections import deque

import numpy as np

from . import (GEO_ENONFINITE, GEO_STORE_F32, Workspace, dims_of, geo_batch_step,
               geo_batch_table_size, geo_state_get, geo_state_init, geo_workspace_size, params)

MAX_BATCH = 64  # cubes of one batched launch (the library's limit)


@dataclasses.dataclass
class Job:
    job_id: int
    v: np.ndarray                 # BSQ cube (N3, N1, N2), host, float32
    eps: float
    alpha: float
    beta: float
    mu_lo: float = 0.0
    mu_hi: float = 1.0
    omega: float = 0.03
    tol: float = 1e-4
    cap: int = 5000
    arrival: float = 0.0          # seconds on the server clock
    # filled by the server
    admitted: float = float("nan")
    finished: float = float("nan")
    iters: int = 0
    converged: bool = False
    error: str | None = None      # set when the job was retired without a result
    u: np.ndarray | None = None
    s: np.ndarray | None = None
    t: np.ndarray | None = None


def _pin(v: np.ndarray):
    """The cube in pinned host memory (runs on the helper thread)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).pin_memory()


class _Active:
    """An admitted job: its cube and workspace on the device, initialised on
    `copy` (a stream) from `pinned` (its cube in pinned host memory); `ready`
    is the event the first round waits for."""

    def __init__(self, job: Job, dual_storage: int, copy=None, pinned=None):
        import torch
        self.job = job
        self.done = 0
        with torch.cuda.stream(copy) if copy is not None else _null():
            src = pinned if pinned is not None else torch.from_numpy(
                np.ascontiguousarray(job.v, dtype=np.float32))
            self.vd = src.to("cuda", non_blocking=pinned is not None)
            self.dims = dims_of(self.vd.shape)
            self.p = params(job.eps, job.alpha, job.beta, job.mu_lo, job.mu_hi, job.omega,
                            max_iter=job.cap, tol=job.tol, dual_storage=dual_storage)
            self.ws = Workspace(geo_workspace_size(self.dims, self.p))
            geo_state_init(self.dims, self.p, self.vd, self.ws, stream=copy)
            self.ready = torch.cuda.Event()
            self.ready.record(copy if copy is not None else torch.cuda.current_stream())
        if copy is not None:
            # allocated on the copy stream, used on the rounds' stream
            main = torch.cuda.current_stream()
            self.vd.record_stream(main)
            self.ws.tensor.record_stream(main)
        self.pinned = pinned  # kept until the copy has run
        self.waited = False


class _null:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


def footprint(shape, dual_storage: int = GEO_STORE_F32) -> int:
    """HBM bytes one job holds while admitted: its workspace and its cube."""
    n3, n1, n2 = shape
    p = params(1.0, 1.0, 1.0, dual_storage=dual_storage)
    return geo_workspace_size(dims_of(shape), p) + 4 * n1 * n2 * n3


class Server:
    """Admission by HBM footprint, rounds of `round_iters` batched iterations.

    active_voxels caps the work in flight: a waiting job is admitted only while
    the admitted cubes hold fewer voxels than that (the first one always). The
    GPU is full well before the HBM budget is, so admitting more only spreads
    the same throughput over more jobs and delays every one of them. None
    admits by footprint alone. overlap: copies and state set-up on a second
    stream, beside the rounds (on a host without a GPU the server keeps the
    admission logic only). keep_results: a finished job keeps its u, s, t in
    host memory (job.u, job.s, job.t); False drops them once their copy to
    the host has completed (a long stream's results would not fit in host
    memory: about 3 x 45 MB for each 11M-voxel job)."""

    def __init__(self, hbm_budget: int, round_iters: int = 25, dual_storage: int = GEO_STORE_F32,
                 use_graph: bool = True, clock=time.perf_counter, active_voxels: int | None = None,
                 overlap: bool = True, keep_results: bool = True):
        self.budget = int(hbm_budget)
        self.keep_results = keep_results
        self.active_voxels = active_voxels
        self.round_iters = int(round_iters)
        self.dual_storage = dual_storage
        self.use_graph = use_graph
        self.clock = clock
        self.t0 = clock()
        self.waiting: deque[Job] = deque()
        self.active: list[_Active] = []
        self.used = 0
        self.voxel_iters = 0
        self._tables = {}
        self.overlap = overlap and _gpu()
        self._copy = None
        self._pins = {}
        self._outbox: list = []  # (job, host tensors, device tensors, event)
        self._out_lock = threading.Lock()
        self._pool = cf.ThreadPoolExecutor(1) if self.overlap else None
        self._stamper = None
        self._stop = threading.Event()

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, job: Job):
        need = footprint(job.v.shape, self.dual_storage)
        if need > self.budget:
            raise ValueError(f"job {job.job_id} needs {need} B, more than the HBM budget")
        self.waiting.append(job)
        self._prefetch()

    def _prefetch(self, ahead: int = 4):
        """Pinned copies for the first `ahead` jobs in line (not for the whole
        queue: under overload it holds most of the stream)."""
        if not self.overlap:
            return
        for job in list(self.waiting)[:ahead]:
            if job.job_id not in self._pins:
                self._pins[job.job_id] = self._pool.submit(_pin, job.v)

    def idle(self) -> bool:
        with self._out_lock:
            out = bool(self._outbox)
        return not self.waiting and not self.active and not out

    def _copy_stream(self):
        import torch
        if self._copy is None:
            self._copy = torch.cuda.Stream()  # default priority
        return self._copy

    def _admit(self):
        while self.waiting and len(self.active) < MAX_BATCH:
            job = self.waiting[0]
            need = footprint(job.v.shape, self.dual_storage)
            if self.used + need > self.budget:
                break
            held = sum(a.vd.numel() for a in self.active)
            if self.active_voxels is not None and self.active and held >= self.active_voxels:
                break
            pin = self._pins.get(job.job_id)
            if pin is not None and not pin.done() and self.active:
                break  # FIFO: wait for its pinned copy rather than stall the GPU
            self.waiting.popleft()
            job.admitted = self.now()
            if self.overlap:
                if job.job_id not in self._pins:
                    self._pins[job.job_id] = self._pool.submit(_pin, job.v)
                pinned = self._pins.pop(job.job_id).result()
                self.active.append(_Active(job, self.dual_storage, self._copy_stream(), pinned))
            else:
                self.active.append(_Active(job, self.dual_storage))
            self.used += need

    def _table(self, n: int) -> Workspace:
        if n not in self._tables:
            self._tables[n] = Workspace(geo_batch_table_size(n))
        return self._tables[n]

    def _stamp_loop(self):
        """Helper thread: stamps each finished job when its copy to the host
        has completed."""
        while not self._stop.is_set():
            with self._out_lock:
                box = list(self._outbox)
            for item in box:
                job, host, _, ev = item
                if ev.query():
                    job.finished = self.now()
                    # into pageable memory: the pinned buffers go back to the
                    # pinned-memory cache for the next jobs
                    if self.keep_results:
                        for name, x in host.items():
                            setattr(job, name, x.numpy().copy())
                    with self._out_lock:
                        self._outbox.remove(item)
            time.sleep(0.0005)

    def _retire(self, a: _Active, converged: bool):
        import torch
        job = a.job
        job.iters, job.converged = a.done, converged
        self.used -= footprint(job.v.shape, self.dual_storage)
        dev = {}
        for name in ("u", "s", "t"):
            x = torch.empty_like(a.vd)
            geo_state_get(a.dims, a.p, a.ws, name, a.vd, x)
            dev[name] = x
        if not self.overlap:
            for name, x in dev.items():
                h = x.cpu().numpy()
                if self.keep_results:
                    setattr(job, name, h)
            job.finished = self.now()
            return [job]
        copy = self._copy_stream()
        main = torch.cuda.current_stream()
        got = torch.cuda.Event()
        got.record(main)
        copy.wait_event(got)
        host = {}
        with torch.cuda.stream(copy):
            for name, x in dev.items():
                h = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
                h.copy_(x, non_blocking=True)
                x.record_stream(copy)
                host[name] = h
            done = torch.cuda.Event()
            done.record(copy)
        with self._out_lock:
            self._outbox.append((job, host, dev, done))
        if self._stamper is None:
            self._stamper = threading.Thread(target=self._stamp_loop, daemon=True)
            self._stamper.start()
        return []

    def step(self) -> list[Job]:
        """Admit what fits, run one round, retire finished jobs. Returns the
        jobs whose result (or error) is final now: all of them without
        overlap; with overlap only those retired with an error, the others'
        copies to the host complete in the background (see drain())."""
        import torch
        self._admit()
        self._prefetch()
        if not self.active:
            return []
        act = self.active
        main = torch.cuda.current_stream()
        for a in act:
            if not a.waited:
                main.wait_event(a.ready)
                a.waited = True
        n_iter = min(self.round_iters, min(a.job.cap - a.done for a in act))
        _, res = geo_batch_step([a.dims for a in act], [a.p for a in act], [a.vd for a in act],
                                [a.ws for a in act], self._table(len(act)), n_iter,
                                use_graph=self.use_graph, raise_nonfinite=False)
        finished, keep = [], []
        for a, r in zip(act, res):
            a.done += r.iters
            self.voxel_iters += r.iters * a.vd.numel()
            if r.status == GEO_ENONFINITE:
                # retired without a result; the rest of the batch goes on
                job = a.job
                job.iters, job.converged = a.done, False
                job.error = "non-finite iterates"
                job.finished = self.now()
                self.used -= footprint(job.v.shape, self.dual_storage)
                finished.append(job)
            elif r.converged or a.done >= a.job.cap:
                finished.extend(self._retire(a, bool(r.converged)))
            else:
                keep.append(a)
        self.active = keep
        return finished

    def drain(self):
        """Waits for every copy to the host in flight."""
        while True:
            with self._out_lock:
                if not self._outbox:
                    break
            time.sleep(0.001)

    def close(self):
        self._stop.set()
        if self._stamper is not None:
            self._stamper.join()
        if self._pool is not None:
            self._pool.shutdown(wait=True)


def _gpu() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:  # noqa: BLE001 - no torch: host-only use
        return False


def run_stream(jobs: list[Job], hbm_budget: int, round_iters: int = 25,
               dual_storage: int = GEO_STORE_F32, use_graph: bool = True,
               active_voxels: int | None = None, overlap: bool = True,
               on_progress=None, progress_every_s: float = 30.0, keep_results: bool = True) -> dict:
    """Serve `jobs` (sorted by arrival, seconds from the start) in real time:
    each job is submitted when the clock reaches its arrival. Returns the
    finished jobs and the latency and throughput figures (busy_s: wall time
    with at least one job admitted). on_progress (optional) is called about
    every progress_every_s seconds with a dict of the stream's state."""
    srv = Server(hbm_budget, round_iters, dual_storage, use_graph, active_voxels=active_voxels,
                 overlap=overlap, keep_results=keep_results)
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    busy = 0.0
    next_report = progress_every_s
    try:
        while pending or srv.waiting or srv.active:
            now = srv.now()
            while pending and pending[0].arrival <= now:
                srv.submit(pending.popleft())
            if on_progress is not None and now >= next_report:
                next_report = now + progress_every_s
                on_progress({"t_s": now, "arrived": len(jobs) - len(pending),
                             "waiting": len(srv.waiting), "active": len(srv.active),
                             "finished": sum(j.finished == j.finished for j in jobs)})  # not NaN
            if not srv.waiting and not srv.active:
                time.sleep(max(0.0, pending[0].arrival - srv.now()))
                continue
            t = srv.now()
            srv.step()
            busy += srv.now() - t
        srv.drain()
    finally:
        srv.close()
    span = srv.now()
    done = sorted(jobs, key=lambda j: j.job_id)
    ok = [j for j in done if j.error is None]
    lat = np.array([j.finished - j.arrival for j in ok])
    return {
        "jobs": done,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "span_s": span,
        "busy_s": busy,
        "requests_per_s": len(done) / span,
        "voxel_iterations_per_s": srv.voxel_iters / span,
        "busy_voxel_iterations_per_s": srv.voxel_iters / busy if busy > 0 else 0.0,
        "voxel_iterations": srv.voxel_iters,
        "mean_iterations": float(np.mean([j.iters for j in done])),
        "converged": int(sum(j.converged for j in done)),
        "errors": int(sum(j.error is not None for j in done)),
    }
