"""Continuous-batching server for independent spectral Ewald requests on one GPU.

Requests (a suspension: positions, forces, box, tolerance) arrive over time.  The server
keeps plans (parameters and tables, keyed by box / tolerance / precision / size class)
resident, and serves requests out of one device arena of a fixed size (the HBM budget):
an admitted request gets one block of it for its workspace (cell lists, grids, sorted
particles) and its device input and output arrays, and returns the block when it
retires.  The arena is the server's only device allocation, so the budget is the bound on
its device memory, and the serving loop allocates nothing on the device.

Admission.  A request that has arrived is admitted when a slot (a stream, default
priority) is free and the arena has room for its block.  When the oldest waiting request
does not fit, younger ones that fit may pass it, at most `max_bypass` times; after that
nothing passes it until it is admitted (no starvation).  Requests carry an optional
deadline for admission and can be cancelled while waiting; malformed requests are
refused with a message and never reach the device.

Each admitted request runs on its slot's stream: host-to-device copy of x and f (pinned
host memory), the evaluation, device-to-host copy of u.  Work of requests admitted while
others run overlaps on the device.  Events on the slot stream time each request's
evaluation on the device clock (against one reference event), so the overlap of requests
is measured, not inferred from host times.  Latency runs from arrival to the completion
of the request's stream work (its result in host memory).

All evaluation goes through the C ABI of the HIP library; this module only schedules.
"""
from __future__ import annotations

import bisect
import dataclasses
import math
import time

import numpy as np

from . import MAX_BATCH, EwaldError, Plan

_ALIGN = 256


def precision_for(tol: float) -> str:
    """FP32 bulk for tolerances it reaches (>= 1e-6 here), FP64 below."""
    return "fp32" if tol >= 1e-6 else "fp64"


@dataclasses.dataclass
class Job:
    rid: int
    arrival: float            # seconds after the server clock started
    box: tuple
    tol: float
    x: "object"               # (3, n) float64 host tensor (pinned for asynchronous copies)
    f: "object"
    n: int
    precision: str = ""
    deadline: float = math.inf  # latest admission time (seconds after the clock started)
    # filled by the server
    admitted: float = math.nan
    done: float = math.nan
    u: "object" = None        # (3, n) float64 host result (a pinned buffer given here is reused)
    slot: int = -1
    footprint: int = 0
    error: str = ""           # why the request was refused, dropped or cancelled ("" = served)
    cancelled: bool = False
    bypassed: int = 0
    dev_start_ms: float = math.nan  # evaluation start / end on the device clock
    dev_end_ms: float = math.nan
    batch: int = 0                  # requests in the evaluation that served this one

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    def cancel(self):
        """Cancel the request: dropped if still waiting, its result discarded if in flight."""
        self.cancelled = True


def _round_up(v, a=_ALIGN):
    return (int(v) + a - 1) // a * a


class Arena:
    """First-fit sub-allocator over one device buffer (byte offsets, 256-byte aligned)."""

    def __init__(self, nbytes: int, device):
        import torch

        self.size = max(_ALIGN, int(nbytes) // _ALIGN * _ALIGN)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]  # sorted, disjoint, coalesced (offset, length)

    def alloc(self, nbytes: int):
        need = _round_up(nbytes)
        for k, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + need, ln - need)
                return off
        return None

    def release(self, off: int, nbytes: int):
        ln = _round_up(nbytes)
        k = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(k, (off, ln))
        # coalesce with the neighbours
        if k + 1 < len(self.free) and self.free[k][0] + self.free[k][1] == self.free[k + 1][0]:
            self.free[k] = (off, self.free[k][1] + self.free[k + 1][1])
            self.free.pop(k + 1)
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == self.free[k][0]:
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            self.free.pop(k)

    def free_bytes(self) -> int:
        return sum(ln for _, ln in self.free)

    def view(self, off: int, nbytes: int):
        return self.buf[off:off + nbytes]


class _Slot:
    def __init__(self, idx, device):
        import torch

        self.idx = idx
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.job = None
        self.block = None  # (offset, bytes) in the arena
        self.ev_start = torch.cuda.Event(enable_timing=True)
        self.ev_end = torch.cuda.Event(enable_timing=True)
        self.ev_done = torch.cuda.Event()


class Server:
    """Admission by HBM footprint onto a pool of streams, out of one device arena."""

    def __init__(self, n_slots: int = 4, hbm_budget: int | None = None, device: str = "cuda:0",
                 plan_n_max: int = 1 << 30, max_bypass: int = 8, batching: bool = True):
        import torch

        self.device = torch.device(device)
        self.slots = [_Slot(i, self.device) for i in range(n_slots)]
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.arena = Arena(self.budget, self.device)
        self.plans: dict = {}
        self.plan_n_max = plan_n_max  # largest request size served
        self.max_bypass = int(max_bypass)
        self.batching = bool(batching)  # small requests with one plan evaluated together
        self.clock0 = None
        self.ev0 = torch.cuda.Event(enable_timing=True)
        # statistics of the last run()
        self.max_in_flight_bytes = 0
        self.in_flight_bytes = 0
        self.memory_waits = 0
        self.bypasses = 0
        self.batches = 0  # evaluations launched in the last run() (a batch of small requests is one)

    # -- plans and footprints -------------------------------------------------------------

    SMALL_N = 16384  # requests up to this size share one plan per (box, tol) and are batched

    @staticmethod
    def size_class(n: int) -> int:
        """Plans are shared by requests whose n rounds up to the same power of two; every
        request of up to SMALL_N particles is in the smallest class (so that small requests
        with the same box and tolerance can be evaluated together in one batch)."""
        return max(Server.SMALL_N, 1 << max(0, int(n) - 1).bit_length())

    def _key(self, job):
        return (tuple(float(b) for b in job.box), float(job.tol), job.precision, self.size_class(job.n))

    def plan_for(self, job):
        """Cached plan per (box, tol, precision, size class): its grid, split and cutoff come
        from the plan cost model for that many particles.  Plans are never replaced while the
        server lives (in-flight work uses them)."""
        if not job.precision:
            job.precision = precision_for(job.tol)
        key = self._key(job)
        pl = self.plans.get(key)
        if pl is None:
            n_cls = min(self.size_class(job.n), self.plan_n_max)
            pl = Plan(job.box, job.tol, precision=job.precision, n_max=n_cls)
            self.plans[key] = pl
        return pl

    def layout(self, group):
        """Byte offsets of a group's block (one request, or small requests sharing a plan):
        workspace, then x, f, u ((3, N) float64 each, the requests' columns side by side)."""
        if not isinstance(group, (list, tuple)):
            group = [group]
        pl = self.plan_for(group[0])
        n = sum(j.n for j in group)
        wsb = pl.workspace_bytes(n) if len(group) == 1 else pl.workspace_bytes_batch([j.n for j in group])
        ws = _round_up(wsb)
        arr = _round_up(24 * n)
        return ws, arr, ws + 3 * arr

    def footprint(self, job) -> int:
        """Device bytes the request holds while in flight: workspace + x, f and u."""
        return self.layout(job)[2]

    @staticmethod
    def validate(job) -> str:
        """Why the request is malformed ("" if it is not)."""
        import torch

        if not (isinstance(job.box, (tuple, list)) and len(job.box) == 3
                and all(isinstance(b, (int, float)) and math.isfinite(b) and b > 0 for b in job.box)):
            return "box must be three positive finite lengths"
        if not (isinstance(job.tol, float) and 1e-12 <= job.tol <= 1e-2):
            return "tol must be in [1e-12, 1e-2]"
        for name in ("x", "f"):
            a = getattr(job, name)
            if not isinstance(a, torch.Tensor) or a.dtype != torch.float64 or a.dim() != 2 or a.shape[0] != 3:
                return "%s must be a (3, n) float64 tensor" % name
            if a.is_cuda:
                return "%s must be in host memory" % name
        if job.x.shape != job.f.shape or job.x.shape[1] != job.n:
            return "x and f must both be (3, n) with n = %d" % job.n
        if job.n < 1:
            return "n must be positive"
        if not (bool(torch.isfinite(job.x).all()) and bool(torch.isfinite(job.f).all())):
            return "x and f must be finite"
        return ""

    # -- scheduling -------------------------------------------------------------------------

    def now(self):
        return time.perf_counter() - self.clock0

    def _admit(self, group, slot, off, total):
        """Enqueue a group on a slot's stream: copies in, one evaluation (ewald_eval_batch for
        several small requests), copies out.  Returns the requests that failed to enqueue."""
        import torch

        pl = self.plan_for(group[0])
        ws_b, arr_b, _ = self.layout(group)
        n = sum(j.n for j in group)
        blk = self.arena.view(off, total)
        ws = blk[:ws_b]
        x, f, u = [blk[ws_b + k * arr_b: ws_b + k * arr_b + 24 * n].view(torch.float64).view(3, n) for k in range(3)]
        cols = []
        c = 0
        for j in group:
            cols.append((c, c + j.n))
            c += j.n
            j.admitted = self.now()
            j.slot = slot.idx
            j.batch = len(group)
            if j.u is None or tuple(j.u.shape) != (3, j.n) or j.u.is_cuda:
                j.u = torch.empty((3, j.n), dtype=torch.float64, pin_memory=True)
        with torch.cuda.stream(slot.stream):
            for j, (a, b) in zip(group, cols):
                x[:, a:b].copy_(j.x, non_blocking=True)
                f[:, a:b].copy_(j.f, non_blocking=True)
            slot.ev_start.record(slot.stream)
            try:
                if len(group) == 1:
                    pl.eval(x, f, out=u, workspace=ws, stream=slot.stream)
                else:
                    pl.eval_batch(x, f, [j.n for j in group], out=u, workspace=ws, stream=slot.stream)
            except EwaldError as e:
                # nothing of the evaluation was enqueued: the group fails alone; its block
                # returns to the arena once the stream has finished the copies into it
                slot.ev_done.record(slot.stream)
                slot.ev_done.synchronize()
                self.arena.release(off, total)
                for j in group:
                    j.error = "evaluation failed: %s" % e
                    j.done = self.now()
                    j.u = None
                return list(group)
            slot.ev_end.record(slot.stream)
            for j, (a, b) in zip(group, cols):
                j.u.copy_(u[:, a:b], non_blocking=True)
            slot.ev_done.record(slot.stream)
        slot.job, slot.block = list(group), (off, total)
        self.in_flight_bytes += total
        self.max_in_flight_bytes = max(self.max_in_flight_bytes, self.in_flight_bytes)
        return []

    def _retire(self, slot):
        out = []
        for job in slot.job:
            job.done = self.now()
            job.dev_start_ms = self.ev0.elapsed_time(slot.ev_start)
            job.dev_end_ms = self.ev0.elapsed_time(slot.ev_end)
            if job.cancelled:
                job.error = "cancelled"
                job.u = None
            out.append(job)
        self.arena.release(*slot.block)
        self.in_flight_bytes -= slot.block[1]
        slot.job, slot.block = None, None
        return out

    def _group(self, ready, lead):
        """The lead request and, when it is small, the other waiting requests with its plan
        (up to the library's batch limit), in arrival order."""
        group = [ready[lead]]
        if self.batching and ready[lead].n <= self.SMALL_N:
            key = self._key(ready[lead])
            for i, j in enumerate(ready):
                if len(group) >= MAX_BATCH:
                    break
                if i != lead and j.n <= self.SMALL_N and self._key(j) == key:
                    group.append(j)
        return group

    def run(self, jobs, poll_s: float = 2e-5):
        """Serve `jobs` (arrival times in seconds from now); returns every job, served ones
        first in completion order, then the refused, expired or cancelled ones (`error`)."""
        import torch

        done, dropped = [], []
        pending = []
        for j in jobs:
            j.error = ""
            msg = self.validate(j)
            if not msg:
                if not j.precision:
                    j.precision = precision_for(j.tol)
                try:
                    j.footprint = self.footprint(j)
                except Exception as e:  # the library refused the plan
                    msg = "plan: %s" % e
            if not msg and j.footprint > self.arena.size:
                msg = "needs %d bytes, above the HBM budget %d" % (j.footprint, self.arena.size)
            if msg:
                j.error = msg
                dropped.append(j)
            else:
                pending.append(j)
        pending.sort(key=lambda j: j.arrival)
        ready = []
        k = 0
        self.max_in_flight_bytes = self.in_flight_bytes = 0
        self.memory_waits = self.bypasses = self.batches = 0
        self.clock0 = time.perf_counter()
        self.ev0.record(torch.cuda.current_stream(self.device))
        self.ev0.synchronize()
        while k < len(pending) or ready or any(s.job is not None for s in self.slots):
            for s in self.slots:
                if s.job is not None and s.ev_done.query():
                    done.extend(self._retire(s))
            t = self.now()
            while k < len(pending) and pending[k].arrival <= t:
                ready.append(pending[k])
                k += 1
            # cancelled or expired requests leave the queue without touching the device
            keep = []
            for j in ready:
                if j.cancelled or t > j.deadline:
                    j.error = "cancelled" if j.cancelled else "deadline passed before admission"
                    dropped.append(j)
                else:
                    keep.append(j)
            ready = keep
            while ready:
                slot = next((s for s in self.slots if s.job is None), None)
                if slot is None:
                    break
                pick, off = None, self.arena.alloc(ready[0].footprint)
                if off is not None:
                    pick = 0
                elif ready[0].bypassed < self.max_bypass:
                    for i in range(1, len(ready)):
                        if ready[i].footprint < ready[0].footprint:
                            off = self.arena.alloc(ready[i].footprint)
                            if off is not None:
                                pick = i
                                ready[0].bypassed += 1
                                self.bypasses += 1
                                break
                if pick is None:
                    self.memory_waits += 1
                    break
                # small requests sharing the lead's plan join it in one batched evaluation
                # while their joint block fits
                group = self._group(ready, pick)
                total = ready[pick].footprint
                if len(group) > 1:
                    self.arena.release(off, ready[pick].footprint)
                    while True:
                        total = self.layout(group)[2]
                        off = self.arena.alloc(total)
                        if off is not None or len(group) == 1:
                            break
                        group.pop()
                    if off is None:  # the lead alone fitted a moment ago
                        total = ready[pick].footprint
                        off = self.arena.alloc(total)
                ids = set(id(j) for j in group)
                ready = [j for j in ready if id(j) not in ids]
                dropped.extend(self._admit(group, slot, off, total))
                self.batches += 1
            if poll_s > 0:
                time.sleep(poll_s)
        return done + dropped


def device_overlap(done):
    """Concurrency of the served requests' evaluations on the device clock: the summed
    evaluation time over the time during which at least one evaluation ran (1 = no
    overlap), and the number of request pairs whose evaluations overlapped."""
    iv = sorted((j.dev_start_ms, j.dev_end_ms) for j in done if not j.error and math.isfinite(j.dev_start_ms))
    if not iv:
        return {"concurrency": float("nan"), "overlapping_pairs": 0, "busy_ms": 0.0}
    busy, cur_s, cur_e = 0.0, iv[0][0], iv[0][1]
    for s, e in iv[1:]:
        if s > cur_e:
            busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    busy += cur_e - cur_s
    total = sum(e - s for s, e in iv)
    pairs = 0
    for a in range(len(iv)):
        for b in range(a + 1, len(iv)):
            if iv[b][0] >= iv[a][1]:
                break
            pairs += 1
    return {"concurrency": total / busy if busy > 0 else float("nan"), "overlapping_pairs": pairs,
            "busy_ms": busy}


def summarize(done):
    served = [j for j in done if not j.error]
    lat = np.array([j.latency for j in served]) * 1e3
    n_total = sum(j.n for j in served)
    span = max(j.done for j in served) - min(j.arrival for j in served)
    out = {
        "requests": len(served),
        "dropped": len(done) - len(served),
        "particles": n_total,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "particles_per_s": n_total / span if span > 0 else float("nan"),
        "wall_s": span,
    }
    small = [j for j in served if j.n <= 10_000]
    if small:
        out["small_requests"] = len(small)
        out["small_p50_ms"] = float(np.percentile(np.array([j.latency for j in small]) * 1e3, 50))
    out.update(device_overlap(served))
    return out


def make_jobs(requests, pin=True):
    """Jobs from workloads.Request descriptions (inputs generated on the host, pinned)."""
    import torch

    jobs = []
    for r in requests:
        x, f = r.make()
        xt, ft = torch.from_numpy(x), torch.from_numpy(f)
        if pin:
            xt, ft = xt.pin_memory(), ft.pin_memory()
        j = Job(r.rid, r.arrival_s, r.box, r.tol, xt, ft, x.shape[1])
        # the result's host buffer, pinned ahead of time (allocating it would add to latency)
        j.u = torch.empty((3, j.n), dtype=torch.float64, pin_memory=pin)
        jobs.append(j)
    return jobs
