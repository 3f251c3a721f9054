"""Continuous-batching request loop for projection steps of uneven grid sizes.

Requests (one projection step each: ppe_solve + ppe_correct) arrive over
time.  The scheduler
  * admits a request when its memory (its seven resident input fields and
    four output fields, plus the workspace of a plan it would need that is
    not cached yet) fits the HBM budget, rejecting a request that could never
    fit (PPE_ERR_NOMEM); an admitted request's inputs are made resident then
    (Backend.stage) and released when it completes;
  * keeps plans cached per (stream slot, shape, batch size), evicting unused
    plans least-recently-used when the budget is tight;
  * whenever a stream slot is free, launches the oldest ready request together
    with up to `max_group` ready requests of the same shape in ONE batched
    ppe_solve / ppe_correct (every kernel handles all of them per launch);
  * overlaps groups on `n_slots` HIP streams and completes them by polling
    their events, recording latency = completion - arrival.

Every arithmetic step runs in libppe.so; this module only schedules.  The
backend is pluggable, so the scheduling logic is tested on the CPU with a
fake backend and a fake clock.
"""

from __future__ import annotations

import collections
import dataclasses
import heapq
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

PPE_OK = 0
PPE_ERR_NOMEM = -2

Shape = Tuple[int, int, int]


@dataclasses.dataclass
class Request:
    rid: int
    shape: Shape                   # (nx, ny, nz)
    inputs: object                 # backend-specific handle to the seven resident input fields
    rho0: float
    dt: float
    arrival: float                 # seconds on the server clock
    lengths: Tuple[float, float, float] = (2 * math.pi, 2.0, 2 * math.pi)
    ybc: int = 0                   # y boundaries (0 walls, 1 symmetry bottom + outflow top)
    # filled by the server
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None
    status: Optional[int] = None
    info: Optional[dict] = None
    outputs: object = None
    group: Optional[int] = None    # launch group id
    # where the inputs come from when they are not resident yet: the backend
    # copies them into request-owned device memory at admission (None: the
    # caller's `inputs` are used as they are)
    source: object = None

    @property
    def npts(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def plan_key(self):
        """Requests with equal keys can share a plan and a batched launch."""
        return (self.shape, tuple(self.lengths), self.ybc)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    s = sorted(xs)
    if not s:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(s))))
    return s[k - 1]


class Backend:
    """Interface the scheduler drives."""

    def output_bytes(self, shape: Shape) -> int:
        raise NotImplementedError

    def input_bytes(self, shape: Shape) -> int:
        """Device bytes of a request's inputs: u*, w*, rho, p^n, p^{n-1}, S on
        cells and v* on the ny + 1 v faces, float64 (the interface's layouts)."""
        nx, ny, nz = shape
        return 8 * (6 * nx * ny * nz + nx * (ny + 1) * nz)

    def stage(self, req: "Request") -> None:
        """Make an admitted request's inputs resident (default: they are)."""

    def release(self, req: "Request") -> None:
        """Free what stage() allocated for a request that has completed."""

    def plan_bytes(self, shape: Shape, batch: int) -> int:
        raise NotImplementedError

    def make_plan(self, slot: int, shape: Shape, batch: int, lengths, ybc: int = 0) -> object:
        raise NotImplementedError

    def free_plan(self, plan: object) -> None:
        raise NotImplementedError

    def launch(self, slot: int, plan: object, reqs: List[Request]) -> object:
        """Enqueue one batched solve + correct for `reqs` on stream `slot`."""
        raise NotImplementedError

    def poll(self, handle: object) -> bool:
        raise NotImplementedError

    def collect(self, handle: object, reqs: List[Request]) -> None:
        """After poll() is True: fill req.info / req.status / req.outputs."""
        raise NotImplementedError


class Server:
    def __init__(self, backend: Backend, budget_bytes: int, n_slots: int = 4, max_group: int = 8,
                 clock: Callable[[], float] = time.perf_counter, idle: Optional[Callable[[], None]] = None,
                 max_points: Optional[int] = None):
        self.b = backend
        self.budget = int(budget_bytes)
        self.n_slots = int(n_slots)
        self.max_group = int(max_group)
        # cap on the grid points of one group (at least one request): a large
        # instance already fills the GPU, and a group of them only makes the
        # requests queued behind it wait longer
        self.max_points = None if max_points is None else int(max_points)
        self.clock = clock
        self.idle = idle
        self.used = 0                                 # bytes held by admitted requests and cached plans
        self.plans: "collections.OrderedDict[Tuple[int, Shape, int], Tuple[object, int]]" = collections.OrderedDict()
        self.plan_busy: Dict[Tuple[int, Shape, int], bool] = {}
        self.ready: Deque[Request] = collections.deque()
        self.inflight: Dict[int, Tuple[object, List[Request], int]] = {}   # slot -> (handle, reqs, group)
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.groups = 0
        self.t0 = None

    # -- memory ---------------------------------------------------------------
    def _evict(self, need: int) -> bool:
        """Free unused cached plans (LRU first) until `need` more bytes fit."""
        if self.used + need <= self.budget:
            return True
        for key in list(self.plans.keys()):
            if self.used + need <= self.budget:
                break
            if self.plan_busy.get(key):
                continue
            plan, nbytes = self.plans.pop(key)
            self.plan_busy.pop(key, None)
            self.b.free_plan(plan)
            self.used -= nbytes
        return self.used + need <= self.budget

    def _bytes(self, req: Request) -> int:
        """Memory a request holds from admission to completion: inputs and outputs."""
        return self.b.output_bytes(req.shape) + self.b.input_bytes(req.shape)

    def _admit(self, req: Request) -> bool:
        need = self._bytes(req)
        worst = need + self.b.plan_bytes(req.shape, 1)
        if worst > self.budget:
            req.status = PPE_ERR_NOMEM
            req.done = self.clock()
            self.rejected.append(req)
            return True  # consumed (rejected)
        if not self._evict(need):
            return False
        self.used += need
        req.admitted = self.clock()
        self.b.stage(req)
        self.ready.append(req)
        return True

    def _plan(self, slot: int, req: Request, batch: int):
        key = (slot, req.plan_key, batch)
        if key in self.plans:
            self.plans.move_to_end(key)
            return key, self.plans[key][0]
        nbytes = self.b.plan_bytes(req.shape, batch)
        if not self._evict(nbytes):
            return None, None
        plan = self.b.make_plan(slot, req.shape, batch, req.lengths, req.ybc)
        self.plans[key] = (plan, nbytes)
        self.used += nbytes
        return key, plan

    # -- scheduling -------------------------------------------------------------
    def _launch_ready(self):
        for slot in range(self.n_slots):
            if not self.ready:
                return
            if slot in self.inflight:
                continue
            head = self.ready[0]
            cap = self.max_group
            if self.max_points is not None:
                cap = max(1, min(cap, self.max_points // math.prod(head.shape)))
            same = [r for r in self.ready if r.plan_key == head.plan_key][:cap]
            # batch sizes are powers of two so that few plans serve every group
            g = 1 << (len(same).bit_length() - 1)
            group = same[:g]
            key, plan = self._plan(slot, head, g)
            if plan is None and g > 1:
                g = 1
                group = same[:1]
                key, plan = self._plan(slot, head, 1)
            if plan is None:
                if not self.inflight:
                    # nothing will free memory: the head request cannot be served
                    self.ready.popleft()
                    head.status = PPE_ERR_NOMEM
                    head.done = self.clock()
                    self.used -= self._bytes(head)
                    self.b.release(head)
                    self.rejected.append(head)
                    continue
                # no room for the plan now: retry once requests complete
                return
            for r in group:
                self.ready.remove(r)
                r.launched = self.clock()
                r.group = self.groups
            self.plan_busy[key] = True
            handle = self.b.launch(slot, plan, group)
            self.inflight[slot] = (handle, group, key)
            self.groups += 1

    def _complete(self):
        for slot in list(self.inflight.keys()):
            handle, group, key = self.inflight[slot]
            if not self.b.poll(handle):
                continue
            now = self.clock()
            self.b.collect(handle, group)
            for r in group:
                r.done = now
                self.used -= self._bytes(r)
                self.b.release(r)
                self.finished.append(r)
            self.plan_busy[key] = False
            del self.inflight[slot]

    def run(self, requests: Sequence[Request], time_limit: float = 3600.0) -> dict:
        """Serve `requests` (arrival times relative to the start) to completion."""
        self.t0 = self.clock()
        pending = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(pending)
        for r in requests:
            r.arrival += self.t0
        waiting: Deque[Request] = collections.deque()
        while pending or waiting or self.ready or self.inflight:
            now = self.clock()
            while pending and self.t0 + pending[0][0] <= now:
                waiting.append(heapq.heappop(pending)[2])
            while waiting and self._admit(waiting[0]):
                waiting.popleft()
            self._complete()
            self._launch_ready()
            if self.clock() - self.t0 > time_limit:
                raise TimeoutError("serving loop exceeded its time limit")
            if self.idle is not None:
                self.idle()
        return self.metrics(requests)

    def metrics(self, requests: Sequence[Request]) -> dict:
        served = [r for r in requests if r.status is not None and r.status != PPE_ERR_NOMEM and r.done]
        lat = [r.latency for r in served]
        if not served:
            return {"served": 0}
        t_end = max(r.done for r in served)
        span = t_end - self.t0
        pts = sum(r.npts for r in served)
        return {
            "served": len(served),
            "rejected": len(self.rejected),
            "groups": self.groups,
            "span_s": span,
            "requests_per_s": len(served) / span if span > 0 else float("inf"),
            "points_per_s": pts / span if span > 0 else float("inf"),
            "p50_ms": 1e3 * percentile(lat, 50),
            "p99_ms": 1e3 * percentile(lat, 99),
            "mean_ms": 1e3 * sum(lat) / len(lat),
            "max_group": max(sum(1 for r in served if r.group == g) for g in {r.group for r in served}),
        }


# ---------------------------------------------------------------------------
# Arrival processes
# ---------------------------------------------------------------------------

def poisson_arrivals(n: int, rate: float, seed: int) -> List[float]:
    """n arrival times (s) of a Poisson process of `rate` per second."""
    import numpy as np

    rng = np.random.default_rng(seed)
    if rate == float("inf"):
        return [0.0] * n
    gaps = rng.exponential(1.0 / rate, size=n)
    return list(np.cumsum(gaps) - gaps[0])


# ---------------------------------------------------------------------------
# GPU backend (libppe.so through the binding)
# ---------------------------------------------------------------------------

class GpuBackend(Backend):
    """Batched ppe_solve + ppe_correct on `n_slots` torch streams."""

    def __init__(self, n_slots: int = 4, precision: int = 1, tol: float = 1e-12, max_refine: int = 1,
                 device: int = 0, keep_outputs: bool = False):
        import torch

        from . import binding

        self.torch = torch
        self.binding = binding
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_slots)]
        self.stage_stream = torch.cuda.Stream(self.device)  # input copies at admission
        self.precision, self.tol, self.max_refine = precision, tol, max_refine
        self.keep_outputs = keep_outputs
        self._ws: Dict[Tuple[Shape, int], int] = {}

    def output_bytes(self, shape: Shape) -> int:
        nx, ny, nz = shape
        return 8 * (3 * nx * ny * nz + nx * (ny + 1) * nz)   # p, u, w and v

    def plan_bytes(self, shape: Shape, batch: int) -> int:
        key = (shape, batch)
        if key not in self._ws:
            d = self.binding.make_desc(*shape, precision=self.precision, tol=self.tol,
                                       max_refine=self.max_refine, batch=batch)
            self._ws[key] = self.binding.workspace_bytes(d)
        return self._ws[key]

    def stage(self, req):
        """Copy the request's source fields into device memory it owns (on
        the staging stream; its launch waits for the copy)."""
        if req.source is None or req.inputs is not None:
            return
        torch = self.torch
        keys = list(req.source.keys())
        srcs = [req.source[k] for k in keys]
        with torch.cuda.stream(self.stage_stream):
            # one allocation for all the fields and one multi-tensor copy: the
            # serving loop is a single host thread, so per-field calls would
            # bound its request rate
            flat = torch.empty(sum(t.numel() for t in srcs), dtype=srcs[0].dtype, device=srcs[0].device)
            dsts, off = [], 0
            for t in srcs:
                dsts.append(flat[off:off + t.numel()].view(t.shape))
                off += t.numel()
            torch._foreach_copy_(dsts, srcs)
            ev = torch.cuda.Event()
            ev.record(self.stage_stream)
        req.inputs = dict(zip(keys, dsts))
        req.staged = ev
        req.staged_flat = flat

    def release(self, req):
        if req.source is not None:
            req.inputs = None
            req.staged = None
            req.staged_flat = None

    def make_plan(self, slot, shape, batch, lengths, ybc=0):
        nx, ny, nz = shape
        return self.binding.Plan(nx, ny, nz, *lengths, precision=self.precision, tol=self.tol,
                                 max_refine=self.max_refine, batch=batch, stream=self.streams[slot], ybc=ybc)

    def free_plan(self, plan):
        plan.close()

    def launch(self, slot, plan, reqs):
        torch = self.torch
        st = self.streams[slot]
        for r in reqs:
            ev = getattr(r, "staged", None)
            if ev is not None:
                st.wait_event(ev)
                r.staged_flat.record_stream(st)  # allocated on the staging stream, used on this one
        with torch.cuda.stream(st):
            fields = [r.inputs for r in reqs]
            outs = []
            for f in fields:
                outs.append({"p": torch.empty_like(f["rho"]), "u": torch.empty_like(f["us"]),
                             "v": torch.empty_like(f["vs"]), "w": torch.empty_like(f["ws"])})
            _, info = self.binding.step(plan, fields, [r.rho0 for r in reqs], [r.dt for r in reqs], outs)
            # the records travel to pinned host memory on the same stream, so
            # completion needs no synchronisation with other streams
            info_host = torch.empty(info.shape, dtype=info.dtype, pin_memory=True)
            info_host.copy_(info, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, outs, info_host)

    def poll(self, handle):
        return handle[0].query()

    def collect(self, handle, reqs):
        ev, outs, info_host = handle
        recs = self.binding.decode_info(info_host)
        for r, o, rec in zip(reqs, outs, recs):
            r.outputs = o if self.keep_outputs else None
            r.info = rec
            r.status = rec["status"]


def group_by_shape(reqs: Sequence[Request], max_batch: int) -> List[List[Request]]:
    """Requests of one plan key (shape, lengths, y boundaries) in groups of at
    most max_batch, in first-seen order."""
    by: "collections.OrderedDict[tuple, List[Request]]" = collections.OrderedDict()
    for r in reqs:
        by.setdefault(r.plan_key, []).append(r)
    out = []
    for lst in by.values():
        for i in range(0, len(lst), max_batch):
            out.append(lst[i:i + max_batch])
    return out


def solve_batch(backend: GpuBackend, reqs: Sequence[Request], max_batch: int = 64) -> dict:
    """All requests at once: one plan and one batched launch sequence per shape
    group, groups spread over the backend's streams.  Returns timing."""
    torch = backend.torch
    groups = group_by_shape(reqs, max_batch)
    plans = [backend.make_plan(i % len(backend.streams), g[0].shape, len(g), g[0].lengths, g[0].ybc)
             for i, g in enumerate(groups)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    handles = [backend.launch(i % len(backend.streams), pl, g) for i, (pl, g) in enumerate(zip(plans, groups))]
    torch.cuda.synchronize()
    span = time.perf_counter() - t0
    for h, g in zip(handles, groups):
        backend.collect(h, g)
    for pl in plans:
        backend.free_plan(pl)
    pts = sum(r.npts for r in reqs)
    return {"groups": len(groups), "span_s": span, "points_per_s": pts / span, "requests": len(reqs)}
