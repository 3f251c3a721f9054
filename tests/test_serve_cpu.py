"""Serving scheduler on the CPU: a fake backend and a fake clock.

Checks admission by memory budget, rejection of requests that can never fit,
same-shape grouping in power-of-two launches, plan caching and eviction,
FIFO order, fault isolation (a failing request does not affect others) and
the p50/p99 arithmetic.
"""
import math

import pytest

from paper_2103_01874_amd.serve import (PPE_ERR_NOMEM, Backend, Request, Server, group_by_shape, percentile,
                                        poisson_arrivals)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self, dt=1e-4):
        self.t += dt


class FakeBackend(Backend):
    """Service time = 1 ms per million points per group (batched work adds up)."""

    def __init__(self, clock, plan_cost=1000, bad=()):
        self.clock = clock
        self.plan_cost = plan_cost
        self.made = []
        self.freed = []
        self.launches = []
        self.bad = set(bad)
        self.staged = []
        self.released = []

    def stage(self, req):
        self.staged.append(req.rid)

    def release(self, req):
        self.released.append(req.rid)

    def output_bytes(self, shape):
        nx, ny, nz = shape
        return 8 * (3 * nx * ny * nz + nx * (ny + 1) * nz)

    def plan_bytes(self, shape, batch):
        return self.plan_cost * batch

    def make_plan(self, slot, shape, batch, lengths, ybc=0):
        p = (slot, shape, batch, len(self.made), tuple(lengths), ybc)
        self.made.append(p)
        return p

    def free_plan(self, plan):
        self.freed.append(plan)

    def launch(self, slot, plan, reqs):
        assert plan[1] == reqs[0].shape and plan[2] == len(reqs)
        assert all(r.plan_key == (plan[1], plan[4], plan[5]) for r in reqs)
        self.launches.append((slot, [r.rid for r in reqs]))
        work = sum(r.npts for r in reqs) / 1e6 * 1e-3
        return self.clock() + work

    def poll(self, handle):
        return self.clock() >= handle

    def collect(self, handle, reqs):
        for r in reqs:
            r.status = -5 if r.rid in self.bad else 0
            r.info = {"status": r.status}


def mk(rid, shape, t):
    return Request(rid=rid, shape=shape, inputs=None, rho0=1.0, dt=1e-3, arrival=t)


def run(reqs, budget=10**12, slots=2, max_group=8, max_points=None, **kw):
    clk = FakeClock()
    be = FakeBackend(clk, **kw)
    srv = Server(be, budget, n_slots=slots, max_group=max_group, clock=clk, idle=clk.tick, max_points=max_points)
    m = srv.run(reqs)
    return srv, be, m


def test_percentiles_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert math.isnan(percentile([], 50))


def test_same_shape_requests_share_one_launch():
    reqs = [mk(i, (32, 32, 32), 0.0) for i in range(8)] + [mk(8 + i, (64, 64, 64), 0.0) for i in range(3)]
    srv, be, m = run(reqs, slots=2)
    assert m["served"] == 11
    sizes = sorted(len(l[1]) for l in be.launches)
    # 8 small ones in one group; 3 large ones as a power-of-two group of 2 plus 1
    assert sizes == [1, 2, 8]
    for slot, ids in be.launches:
        assert len({reqs[i].shape for i in ids}) == 1


def test_fifo_head_goes_first():
    reqs = [mk(0, (64, 64, 64), 0.0), mk(1, (32, 32, 32), 0.0), mk(2, (64, 64, 64), 0.0)]
    srv, be, m = run(reqs, slots=1)
    assert be.launches[0][1] == [0, 2]
    assert be.launches[1][1] == [1]


def request_bytes(shape):
    be = FakeBackend(FakeClock())
    return be.output_bytes(shape) + be.input_bytes(shape)


def test_budget_limits_admission_and_rejects_impossible():
    big = (256, 128, 256)
    small = (32, 32, 32)
    budget = request_bytes(small) * 3 + 10**5
    reqs = [mk(0, big, 0.0)] + [mk(1 + i, small, 0.0) for i in range(6)]
    srv, be, m = run(reqs, budget=budget, slots=1, plan_cost=10)
    assert reqs[0].status == PPE_ERR_NOMEM
    assert m["rejected"] == 1 and m["served"] == 6
    # never more than three small requests admitted at once
    assert max(len(ids) for _, ids in be.launches) <= 2


def test_plan_cache_reuses_and_evicts():
    reqs = [mk(i, (32, 32, 32), 0.01 * i) for i in range(5)]
    srv, be, m = run(reqs, slots=1)
    # requests arrive one by one and finish before the next: one plan reused
    assert len(be.made) == 1
    shapes = [(32, 32, 32), (64, 32, 32), (32, 64, 32)]
    reqs = [mk(i, shapes[i % 3], 0.01 * i) for i in range(6)]
    budget = max(request_bytes(s) for s in shapes) + 1500  # room for one plan at a time
    srv, be, m = run(reqs, budget=budget, slots=1, plan_cost=1000)
    assert m["served"] == 6
    assert len(be.freed) >= 4  # plans evicted to make room


def test_failure_is_isolated():
    reqs = [mk(i, (32, 32, 32), 0.0) for i in range(4)]
    srv, be, m = run(reqs, bad={2})
    assert [r.status for r in reqs] == [0, 0, -5, 0]


def test_latency_and_throughput_accounting():
    reqs = [mk(i, (100, 100, 100), 0.002 * i) for i in range(10)]  # 1 ms of work each, arrivals every 2 ms
    srv, be, m = run(reqs, slots=1)
    assert m["served"] == 10
    lat = [r.latency for r in reqs]
    assert all(0.0009 < x < 0.0013 for x in lat)
    assert abs(m["p50_ms"] - 1e3 * percentile(lat, 50)) < 1e-9
    assert m["points_per_s"] > 0


def test_grouping_helper_and_arrivals():
    reqs = [mk(i, (32 if i % 2 else 64, 32, 32), 0.0) for i in range(7)]
    gs = group_by_shape(reqs, 2)
    assert [len(g) for g in gs] == [2, 2, 2, 1]
    a = poisson_arrivals(1000, 100.0, 1)
    assert a[0] == 0.0 and all(x <= y for x, y in zip(a, a[1:]))
    assert 8.0 < a[-1] < 12.0


def test_boundaries_and_lengths_split_groups():
    """Same shape but other y boundaries or lengths never share a plan or a launch."""
    reqs = [mk(i, (32, 32, 32), 0.0) for i in range(6)]
    reqs[1].ybc = 1
    reqs[3].ybc = 1
    reqs[4].lengths = (1.0, 1.0, 1.0)
    srv, be, m = run(reqs, slots=1)
    assert m["served"] == 6
    keys = {(p[1], p[4], p[5]) for p in be.made}
    assert len(keys) == 3
    for _, rids in be.launches:
        assert len({reqs[r].plan_key for r in rids}) == 1
    groups = group_by_shape(reqs, 8)
    assert sorted(len(g) for g in groups) == [1, 2, 3]


def test_points_cap_limits_large_groups_only():
    """max_points bounds a group's grid points (at least one request): large
    shapes go out in small groups, small shapes still fill max_group."""
    reqs = [mk(i, (32, 32, 32), 0.0) for i in range(8)] + [mk(8 + i, (128, 64, 128), 0.0) for i in range(4)]
    srv, be, m = run(reqs, slots=1, max_points=2 * 128 * 64 * 128)
    assert m["served"] == 12
    groups = [sorted(reqs[i].shape for i in ids) for _, ids in be.launches]
    assert sorted(len(g) for g in groups if g[0] == (32, 32, 32)) == [8]
    assert sorted(len(g) for g in groups if g[0] == (128, 64, 128)) == [2, 2]
    # a cap below one request still launches it alone
    srv, be, m = run([mk(0, (128, 64, 128), 0.0)], slots=1, max_points=10)
    assert m["served"] == 1 and [len(ids) for _, ids in be.launches] == [1]
    # the first large requests finish before the rest of their shape: lower mean latency
    reqs2 = [mk(i, (128, 64, 128), 0.0) for i in range(4)] + [mk(4, (32, 32, 32), 0.0)]
    _, _, capped = run(reqs2, slots=1, max_points=2 * 128 * 64 * 128)
    reqs3 = [mk(i, (128, 64, 128), 0.0) for i in range(4)] + [mk(4, (32, 32, 32), 0.0)]
    _, _, whole = run(reqs3, slots=1)
    assert capped["mean_ms"] < whole["mean_ms"]


def test_input_fields_are_charged_at_admission():
    """The seven resident input fields (6 cell fields and v* on ny + 1 faces)
    count against the budget: a budget that holds a request's four outputs
    and its plan but not its inputs rejects it with PPE_ERR_NOMEM."""
    shape = (64, 32, 48)
    be = FakeBackend(FakeClock())
    nx, ny, nz = shape
    assert be.input_bytes(shape) == 8 * (6 * nx * ny * nz + nx * (ny + 1) * nz)
    assert be.input_bytes(shape) > be.output_bytes(shape)
    budget = be.output_bytes(shape) + be.input_bytes(shape) // 2 + 10 * 1000
    reqs = [mk(0, shape, 0.0)]
    srv, be, m = run(reqs, budget=budget, slots=1, plan_cost=1000)
    assert reqs[0].status == PPE_ERR_NOMEM and m["served"] == 0
    assert be.staged == [] and be.launches == []
    # with room for the inputs too it is served, staged once and released once
    reqs = [mk(0, shape, 0.0)]
    srv, be, m = run(reqs, budget=request_bytes(shape) + 1000, slots=1, plan_cost=1000)
    assert reqs[0].status == 0 and m["served"] == 1
    assert be.staged == [0] and be.released == [0]
    assert srv.used == 1000  # only the cached plan is left


def test_inputs_limit_how_many_requests_are_resident():
    """Eight equal requests, a budget for three requests' inputs and outputs
    (and their plans): at most three are admitted at a time, every request
    is released exactly once, and the memory in use returns to the plans."""
    shape = (32, 32, 32)
    budget = 3 * request_bytes(shape) + 4 * 1000
    reqs = [mk(i, shape, 0.0) for i in range(8)]
    srv, be, m = run(reqs, budget=budget, slots=2, plan_cost=1000)
    assert m["served"] == 8 and m["rejected"] == 0
    assert sorted(be.staged) == list(range(8)) and sorted(be.released) == list(range(8))
    assert sum(len(ids) for _, ids in be.launches) == 8
    assert max(len(ids) for _, ids in be.launches) <= 2
    assert srv.used == sum(nbytes for _, nbytes in srv.plans.values())
