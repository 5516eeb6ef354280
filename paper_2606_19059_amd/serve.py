"""Continuous-batching server for independent spectral Ewald requests on one GPU.

Requests (a suspension: positions, forces, box, tolerance) arrive over time.  The server
keeps plans (parameters and tables, keyed by box / tolerance / precision / size class) and per-slot
workspaces (cell lists, grids, sorted particles) resident on the device, and admits a
waiting request as soon as a slot is free and its HBM footprint -- workspace plus its
input and output arrays -- fits in what the in-flight requests leave of the budget.
Each admitted request runs on its slot's stream (default priority), so the work of
requests admitted while others are on the GPU overlaps on the device.  Latency is
measured from arrival to the completion of the request's stream work.

All evaluation goes through the C ABI of the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import Plan


def precision_for(tol: float) -> str:
    """FP32 bulk for tolerances it reaches (>= 1e-6 here), FP64 below."""
    return "fp32" if tol >= 1e-6 else "fp64"


@dataclasses.dataclass
class Job:
    rid: int
    arrival: float            # seconds after the server clock started
    box: tuple
    tol: float
    x: "object"               # (3, n) float64 host (pinned) or device tensor
    f: "object"
    n: int
    precision: str = ""
    # filled by the server
    admitted: float = math.nan
    done: float = math.nan
    u: "object" = None
    slot: int = -1
    footprint: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Slot:
    def __init__(self, idx, device):
        import torch

        self.idx = idx
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.workspace = None
        self.job = None
        self.event = None

    def ensure_workspace(self, nbytes, device):
        import torch

        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = None
            self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.workspace


class Server:
    """Admission by HBM footprint onto a pool of streams; plans and workspaces stay resident."""

    def __init__(self, n_slots: int = 4, hbm_budget: int | None = None, device: str = "cuda:0",
                 plan_n_max: int = 1 << 30):
        import torch

        self.device = torch.device(device)
        self.slots = [_Slot(i, self.device) for i in range(n_slots)]
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.in_flight_bytes = 0
        self.plans: dict = {}
        self.plan_n_max = plan_n_max  # largest request size served
        self.clock0 = None
        self.max_in_flight_bytes = 0  # statistics of the last run()
        self.memory_waits = 0

    # -- plans and footprints -------------------------------------------------------------

    @staticmethod
    def size_class(n: int) -> int:
        """Plans are shared by requests whose n rounds up to the same power of two (>= 1024)."""
        return max(1024, 1 << max(0, int(n) - 1).bit_length())

    def _key(self, job):
        return (tuple(float(b) for b in job.box), float(job.tol), job.precision, self.size_class(job.n))

    def plan_for(self, job):
        """Cached plan per (box, tol, precision, size class): its grid, split and cutoff come
        from the plan cost model for that many particles.  Plans are never replaced while the
        server lives (in-flight work uses them)."""
        key = self._key(job)
        pl = self.plans.get(key)
        if pl is None:
            n_cls = min(self.size_class(job.n), self.plan_n_max)
            pl = Plan(job.box, job.tol, precision=job.precision, n_max=n_cls)
            self.plans[key] = pl
        return pl

    def footprint(self, job) -> int:
        """Workspace bytes of the request's plan + its input/output arrays (3 x (3, n) float64)."""
        return int(self.plan_for(job).workspace_bytes(job.n)) + 3 * 24 * job.n

    # -- scheduling -------------------------------------------------------------------------

    def now(self):
        return time.perf_counter() - self.clock0

    def _admit(self, job, slot):
        import torch

        pl = self.plan_for(job)
        ws = slot.ensure_workspace(pl.workspace_bytes(job.n), self.device)
        job.admitted = self.now()
        job.slot = slot.idx
        with torch.cuda.stream(slot.stream):
            x = job.x.to(self.device, non_blocking=True) if not job.x.is_cuda else job.x
            f = job.f.to(self.device, non_blocking=True) if not job.f.is_cuda else job.f
            u = torch.empty_like(x)
            pl.eval(x, f, out=u, workspace=ws, stream=slot.stream)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        job.u = u
        job._keep = (x, f)  # inputs stay alive until the stream is done with them
        slot.job, slot.event = job, ev
        self.in_flight_bytes += job.footprint
        self.max_in_flight_bytes = max(self.max_in_flight_bytes, self.in_flight_bytes)

    def _retire(self, slot):
        job = slot.job
        job.done = self.now()
        job._keep = None
        self.in_flight_bytes -= job.footprint
        slot.job, slot.event = None, None
        return job

    def run(self, jobs, poll_s: float = 2e-5):
        """Serve `jobs` (sorted by arrival time, in seconds from now); returns them completed."""
        for j in jobs:
            if not j.precision:
                j.precision = precision_for(j.tol)
            j.footprint = self.footprint(j)
            if j.footprint > self.budget:
                raise ValueError("request %d needs %d bytes, above the HBM budget %d" % (j.rid, j.footprint, self.budget))
        waiting = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        done = []
        self.max_in_flight_bytes = 0
        self.memory_waits = 0
        self.clock0 = time.perf_counter()
        while waiting or any(s.job is not None for s in self.slots):
            for s in self.slots:
                if s.job is not None and s.event.query():
                    done.append(self._retire(s))
            t = self.now()
            while waiting and waiting[0].arrival <= t:
                job = waiting[0]
                slot = next((s for s in self.slots if s.job is None), None)
                if slot is None:
                    break
                if self.in_flight_bytes + job.footprint > self.budget:
                    self.memory_waits += 1
                    break
                waiting.popleft()
                self._admit(job, slot)
            if poll_s > 0:
                time.sleep(poll_s)
        return done


def summarize(done):
    lat = np.array([j.latency for j in done]) * 1e3
    n_total = sum(j.n for j in done)
    span = max(j.done for j in done) - min(j.arrival for j in done)
    return {
        "requests": len(done),
        "particles": n_total,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "particles_per_s": n_total / span if span > 0 else float("nan"),
        "wall_s": span,
    }


def make_jobs(requests, pin=True):
    """Jobs from workloads.Request descriptions (inputs generated on the host, pinned)."""
    import torch

    jobs = []
    for r in requests:
        x, f = r.make()
        xt, ft = torch.from_numpy(x), torch.from_numpy(f)
        if pin:
            xt, ft = xt.pin_memory(), ft.pin_memory()
        jobs.append(Job(r.rid, r.arrival_s, r.box, r.tol, xt, ft, x.shape[1]))
    return jobs
