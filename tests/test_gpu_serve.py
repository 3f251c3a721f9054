"""Batched and served projection steps on the GPU.

Each result must be the same alone and in the mix: batching changes only
which instances share a launch, never the per-instance arithmetic, so the
comparison is bitwise.  A request with a non-finite input is flagged
(PPE_ERR_NONFINITE) without disturbing the others.
"""
import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import binding, synth
from paper_2103_01874_amd.serve import GpuBackend, Request, Server, poisson_arrivals, solve_batch

pytestmark = pytest.mark.gpu

SHAPES = [(32, 16, 24), (24, 12, 18), (48, 8, 16)]


def make_requests(n, seed, shapes=SHAPES, bad=()):
    import torch
    reqs = []
    for i in range(n):
        pr = synth.mixed_instance(seed + i, shape=shapes[i % len(shapes)])
        if i in bad:
            pr.S = pr.S.copy()
            pr.S[0, 0, 0] = np.nan
        f = binding.to_device(pr)
        r = Request(rid=i, shape=(pr.nx, pr.ny, pr.nz), inputs=f, rho0=pr.rho0, dt=pr.dt, arrival=0.0)
        r.problem = pr
        reqs.append(r)
    return reqs


def alone(r, precision=1):
    import torch
    pr = r.problem
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=precision, tol=1e-12, max_refine=1)
    outs, info = binding.step(plan, [r.inputs], [pr.rho0], [pr.dt])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in outs[0].items()}
    rec = binding.decode_info(info)[0]
    plan.close()
    return res, rec


def same(r, res):
    for k in ("p", "u", "v", "w"):
        a = r.outputs[k].cpu().numpy()
        assert np.array_equal(a, res[k], equal_nan=True), (r.rid, k)


def test_batched_mixed_shapes_match_alone_and_oracle():
    reqs = make_requests(8, 500)
    be = GpuBackend(n_slots=3, precision=1, keep_outputs=True)
    stats = solve_batch(be, reqs)
    assert stats["groups"] == 3
    for r in reqs:
        res, rec = alone(r)
        same(r, res)
        assert r.info == rec
        assert rec["status"] == 0 and rec["res_rel"] <= 1e-12
        pr = r.problem
        g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
        ref = O.ppe_step(g, pr.rho0, pr.dt, *pr.fields())
        ep = np.linalg.norm(res["p"] - ref["p"]) / np.linalg.norm(ref["p"])
        assert ep <= 1e-12


def test_served_results_equal_alone():
    reqs = make_requests(12, 700)
    arr = poisson_arrivals(len(reqs), 2000.0, 3)
    for r, a in zip(reqs, arr):
        r.arrival = a
    be = GpuBackend(n_slots=2, precision=1, keep_outputs=True)
    srv = Server(be, budget_bytes=8 << 30, n_slots=2, max_group=4)
    m = srv.run(reqs, time_limit=60)
    assert m["served"] == len(reqs)
    assert m["p99_ms"] >= m["p50_ms"] > 0
    for r in reqs:
        res, rec = alone(r)
        same(r, res)
        assert r.status == 0


def test_nonfinite_request_is_isolated():
    reqs = make_requests(6, 900, shapes=[(32, 16, 24)], bad={2})
    be = GpuBackend(n_slots=1, precision=1, keep_outputs=True)
    stats = solve_batch(be, reqs)
    assert stats["groups"] == 1
    for r in reqs:
        if r.rid == 2:
            assert r.status == -5
        else:
            assert r.status == 0
            res, rec = alone(r)
            same(r, res)


def test_staged_inputs_are_charged_and_equal_alone():
    """Requests that arrive with a source instead of resident inputs: the
    backend copies the seven fields into memory of the request's own at
    admission (charged against the budget with the outputs) and releases it
    on completion; every result equals the same request solved alone.  A
    budget that holds two requests' inputs and outputs (and the plans) keeps
    at most two admitted at a time."""
    torch = __import__("torch")
    prs = [synth.mixed_instance(1500 + i, shape=(32, 16, 24)) for i in range(6)]
    src = [binding.to_device(p) for p in prs]
    be = GpuBackend(n_slots=2, precision=1, keep_outputs=True)
    per_req = be.output_bytes((32, 16, 24)) + be.input_bytes((32, 16, 24))
    budget = 2 * per_req + 4 * be.plan_bytes((32, 16, 24), 2)
    reqs = []
    for i, p in enumerate(prs):
        r = Request(rid=i, shape=(32, 16, 24), inputs=None, source=src[i], rho0=p.rho0, dt=p.dt, arrival=0.0)
        r.problem = p
        reqs.append(r)
    srv = Server(be, budget_bytes=budget, n_slots=2, max_group=2)
    m = srv.run(reqs, time_limit=60)
    assert m["served"] == 6 and m["rejected"] == 0
    assert all(r.inputs is None for r in reqs)  # released
    assert srv.used == sum(nbytes for _, nbytes in srv.plans.values())
    for r in reqs:
        r.inputs = src[r.rid]  # (alone() solves from the source fields)
        res, rec = alone(r)
        same(r, res)
        assert r.info == rec and r.status == 0
