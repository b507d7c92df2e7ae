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
changes no per-cube arithmetic.

Timing is wall clock: a job's latency runs from its arrival to the moment
its result is on the host.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np

from . import (GEO_STORE_F32, Workspace, dims_of, geo_batch_step, geo_batch_table_size,
               geo_state_get, geo_state_init, geo_workspace_size, params)

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
    u: np.ndarray | None = None
    s: np.ndarray | None = None
    t: np.ndarray | None = None


class _Active:
    def __init__(self, job: Job, dual_storage: int):
        import torch
        self.job = job
        self.vd = torch.from_numpy(np.ascontiguousarray(job.v, dtype=np.float32)).cuda()
        self.dims = dims_of(self.vd.shape)
        self.p = params(job.eps, job.alpha, job.beta, job.mu_lo, job.mu_hi, job.omega,
                        max_iter=job.cap, tol=job.tol, dual_storage=dual_storage)
        self.ws = Workspace(geo_workspace_size(self.dims, self.p))
        geo_state_init(self.dims, self.p, self.vd, self.ws)
        self.done = 0


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
    admits by footprint alone."""

    def __init__(self, hbm_budget: int, round_iters: int = 25, dual_storage: int = GEO_STORE_F32,
                 use_graph: bool = True, clock=time.perf_counter, active_voxels: int | None = None):
        self.budget = int(hbm_budget)
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

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, job: Job):
        need = footprint(job.v.shape, self.dual_storage)
        if need > self.budget:
            raise ValueError(f"job {job.job_id} needs {need} B, more than the HBM budget")
        self.waiting.append(job)

    def idle(self) -> bool:
        return not self.waiting and not self.active

    def _admit(self):
        while self.waiting and len(self.active) < MAX_BATCH:
            job = self.waiting[0]
            need = footprint(job.v.shape, self.dual_storage)
            if self.used + need > self.budget:
                break
            held = sum(a.vd.numel() for a in self.active)
            if self.active_voxels is not None and self.active and held >= self.active_voxels:
                break
            self.waiting.popleft()
            job.admitted = self.now()
            self.active.append(_Active(job, self.dual_storage))
            self.used += need

    def _table(self, n: int) -> Workspace:
        if n not in self._tables:
            self._tables[n] = Workspace(geo_batch_table_size(n))
        return self._tables[n]

    def step(self) -> list[Job]:
        """Admit what fits, run one round, retire finished jobs (returned)."""
        import torch
        self._admit()
        if not self.active:
            return []
        act = self.active
        n_iter = min(self.round_iters, min(a.job.cap - a.done for a in act))
        _, res = geo_batch_step([a.dims for a in act], [a.p for a in act], [a.vd for a in act],
                                [a.ws for a in act], self._table(len(act)), n_iter,
                                use_graph=self.use_graph)
        finished, keep = [], []
        for a, r in zip(act, res):
            a.done += r.iters
            self.voxel_iters += r.iters * a.vd.numel()
            if r.converged or a.done >= a.job.cap:
                job = a.job
                out = {}
                for name in ("u", "s", "t"):
                    x = torch.empty_like(a.vd)
                    geo_state_get(a.dims, a.p, a.ws, name, a.vd, x)
                    out[name] = x
                for name, x in out.items():
                    setattr(job, name, x.cpu().numpy())
                job.iters, job.converged = a.done, bool(r.converged)
                job.finished = self.now()
                self.used -= footprint(job.v.shape, self.dual_storage)
                finished.append(job)
            else:
                keep.append(a)
        self.active = keep
        return finished


def run_stream(jobs: list[Job], hbm_budget: int, round_iters: int = 25,
               dual_storage: int = GEO_STORE_F32, use_graph: bool = True,
               active_voxels: int | None = None) -> dict:
    """Serve `jobs` (sorted by arrival, seconds from the start) in real time:
    each job is submitted when the clock reaches its arrival. Returns the
    finished jobs and the latency and throughput figures."""
    srv = Server(hbm_budget, round_iters, dual_storage, use_graph, active_voxels=active_voxels)
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    done: list[Job] = []
    while pending or not srv.idle():
        now = srv.now()
        while pending and pending[0].arrival <= now:
            srv.submit(pending.popleft())
        if srv.idle():
            time.sleep(max(0.0, pending[0].arrival - srv.now()))
            continue
        done.extend(srv.step())
    span = srv.now()
    lat = np.array([j.finished - j.arrival for j in done])
    return {
        "jobs": done,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "span_s": span,
        "requests_per_s": len(done) / span,
        "voxel_iterations_per_s": srv.voxel_iters / span,
        "mean_iterations": float(np.mean([j.iters for j in done])),
        "converged": int(sum(j.converged for j in done)),
    }
