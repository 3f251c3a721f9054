"""A projection step captured as a HIP graph on the plan's stream.

ppe_solve and ppe_correct enqueue kernels only (no host synchronisation, no
memory set), so a caller with fixed field buffers can capture a step once
and replay it.  Each replay is checked against an eager step on the same
inputs, with eager work and synchronisation between the replays."""
import numpy as np
import pytest

from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
def test_captured_step_replays_equal_eager_steps(precision):
    import torch

    pr = synth.sheet_32()
    side = torch.cuda.Stream()
    f = binding.to_device(pr)
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=precision, tol=1e-12, max_refine=2,
                        stream=side)
    eager = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=precision, tol=1e-12, max_refine=2)
    outs = [{k: torch.empty_like(f[src]) for k, src in (("p", "rho"), ("u", "us"), ("v", "vs"), ("w", "ws"))}]
    info = plan.new_info()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        binding.step(plan, [f], [pr.rho0], [pr.dt], outs, info)   # warm-up outside the capture
    side.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        binding.step(plan, [f], [pr.rho0], [pr.dt], outs, info)
    torch.cuda.synchronize()
    for rep in range(4):
        # eager work between the replays: new inputs in the captured buffers
        f["us"].mul_(1.0 + 0.01 * rep)
        f["S"].add_(1e-4 * rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ref, rinfo = binding.step(eager, [f], [pr.rho0], [pr.dt])
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in outs[0].items()}
        want = {k: v.cpu().numpy() for k, v in ref[0].items()}
        for k in ("p", "u", "v", "w"):
            assert np.array_equal(got[k], want[k]), (rep, k)
        assert binding.decode_info(info) == binding.decode_info(rinfo)
    plan.close()
    eager.close()
