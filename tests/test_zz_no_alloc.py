"""ppe_solve_noalloc (the allocation-free entry point) against the plan path.

Two calls in a row on one GPU, the second with a smaller grid, each against
ppe_plan + ppe_solve + ppe_correct on the same inputs (1e-12 relative in l2
and pointwise, the info records to rounding) and against the oracle.  The
static workspace keeps the first call's contents when the second runs.
Grids beyond the workspace, and descriptors it does not serve, are refused
before anything is enqueued.
"""
import numpy as np
import pytest

import parity_util as PU
from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu

FP64, MIXED = binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED


def _torch():
    import torch
    return torch


def new_outputs(fields, fill=None):
    torch = _torch()
    outs = [{"p": torch.empty_like(f["rho"]), "u": torch.empty_like(f["us"]), "v": torch.empty_like(f["vs"]),
             "w": torch.empty_like(f["ws"])} for f in fields]
    if fill is not None:
        for o in outs:
            for t in o.values():
                t.fill_(fill)
    return outs


def plan_path(probs, fields, precision, max_refine):
    torch = _torch()
    pr = probs[0]
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=precision, tol=1e-12,
                        max_refine=max_refine, batch=len(probs), ybc=pr.ybc)
    outs, info = binding.step(plan, fields, [q.rho0 for q in probs], [q.dt for q in probs])
    torch.cuda.synchronize()
    res = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    recs = binding.decode_info(info)
    plan.close()
    return res, recs


def noalloc_path(probs, fields, precision, max_refine, project=True):
    torch = _torch()
    pr = probs[0]
    outs = new_outputs(fields)
    info = torch.zeros(8 * len(probs), dtype=torch.float64, device=fields[0]["rho"].device)
    st = binding.solve_noalloc(pr.nx, pr.ny, pr.nz, fields, [q.rho0 for q in probs], [q.dt for q in probs], outs,
                               info, lx=pr.lx, ly=pr.ly, lz=pr.lz, precision=precision, tol=1e-12,
                               max_refine=max_refine, ybc=pr.ybc, project=project)
    assert st == binding.PPE_OK, st
    torch.cuda.synchronize()
    res = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    return res, binding.decode_info(info)


def compare(probs, fields, precision, max_refine):
    ref, rrecs = plan_path(probs, fields, precision, max_refine)
    got, grecs = noalloc_path(probs, fields, precision, max_refine)
    for pr, a, b, ra, rb in zip(probs, got, ref, grecs, rrecs):
        e = {"p": PU.rel(a["p"], b["p"]), "inf_p": PU.rel_inf(a["p"], b["p"])}
        for k, s in (("u", "us"), ("v", "vs"), ("w", "ws")):
            da, db = a[k] - getattr(pr, s), b[k] - getattr(pr, s)
            e[k] = PU.rel(da, db)
            e["inf_" + k] = PU.rel_inf(da, db)
        print(f"noalloc {pr.nx}x{pr.ny}x{pr.nz} prec={precision}: {e} iters {ra['iters']}/{rb['iters']} "
              f"eps_div {ra['res_rel']:.2e}/{rb['res_rel']:.2e}", flush=True)
        assert max(e["p"], e["inf_p"], e["u"], e["v"], e["w"]) <= 1e-12, e
        assert max(e["inf_u"], e["inf_v"], e["inf_w"]) <= 1e-11, e
        assert ra["status"] == rb["status"] == 0 and ra["iters"] == rb["iters"]
        assert ra["rho0_used"] == rb["rho0_used"]
        assert ra["compat_defect"] == rb["compat_defect"]  # the same assembly pass and sums
        assert ra["res_rel"] <= 1e-12 and rb["res_rel"] <= 1e-12
        PU.check(pr, a, ra, PU.oracle_step(pr), label="noalloc ")


def test_noalloc_two_calls_fp64_then_smaller():
    """192x96x192 (the largest batched grid, 57 MiB of the 64 MiB workspace),
    then a smaller ragged batch of two."""
    big = [synth.mixed_instance(11000, shape=(192, 96, 192))]
    compare(big, [binding.to_device(p) for p in big], FP64, 0)
    small = [synth.random_problem(36, 20, 24, seed=11001 + i) for i in range(2)]
    compare(small, [binding.to_device(p) for p in small], FP64, 0)


def test_noalloc_two_calls_mixed_then_smaller():
    """FP32 spectra with refinement: 128x64x128, then a batch of three smaller
    half jets (outflow top)."""
    big = [synth.mixed_instance(12000, shape=(128, 64, 128))]
    compare(big, [binding.to_device(p) for p in big], MIXED, 2)
    small = [synth.jet_problem(32, 16, 24, seed=12001 + i, rho_l=100.0 * (3 + i)) for i in range(3)]
    compare(small, [binding.to_device(p) for p in small], MIXED, 2)


def test_noalloc_pressure_only_and_refusals():
    torch = _torch()
    pr = synth.sheet_problem(48, 24, 32, seed=13000, nmodes=3)
    f = [binding.to_device(pr)]
    ref, _ = plan_path([pr], f, FP64, 0)
    got, recs = noalloc_path([pr], f, FP64, 0, project=False)
    assert PU.rel(got[0]["p"], ref[0]["p"]) <= 1e-12 and recs[0]["status"] == 0
    # refusals: nothing is enqueued, the outputs keep their fill
    cases = [((256, 128, 256), binding.PPE_ERR_NOMEM), ((16, 300, 8), binding.PPE_ERR_UNSUPPORTED)]
    for shape, code in cases:
        q = synth.random_problem(*shape, seed=13001)
        fq = [binding.to_device(q)]
        outs = new_outputs(fq, fill=7.0)
        info = torch.full((8,), 7.0, dtype=torch.float64, device=fq[0]["rho"].device)
        st = binding.solve_noalloc(q.nx, q.ny, q.nz, fq, [q.rho0], [q.dt], outs, info, lx=q.lx, ly=q.ly, lz=q.lz)
        torch.cuda.synchronize()
        print(f"noalloc {shape}: status {st}", flush=True)
        assert st == code
        assert all(bool((t == 7.0).all()) for t in outs[0].values()) and bool((info == 7.0).all())
        del fq, outs
