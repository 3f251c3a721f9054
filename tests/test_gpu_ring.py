"""Time-loop residency: the device pressure ring against explicit history
handling (bitwise) and against the oracle's time loop (1e-12), and the
per-step split defect against the oracle's Eq. (25) residuals."""
import numpy as np
import pytest

import oracle as O
import parity_util as PU
from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def step_inputs(shape, ybc, n):
    """Per-step u*, rho, S (a new seeded request each step) on a fixed grid."""
    out = []
    for t in range(n):
        if ybc == 0:
            pr = synth.sheet_problem(*shape, seed=700 + t, nmodes=3)
        else:
            pr = synth.jet_problem(*shape, seed=800 + t, nmodes=3)
        out.append(pr)
    return out


@pytest.mark.parametrize("ybc", [0, 1])
def test_ring_equals_explicit_history_and_oracle_loop(ybc):
    torch = _torch()
    shape = (32, 16, 24)
    T = 4
    steps = step_inputs(shape, ybc, T)
    pr0 = steps[0]
    plan = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, ybc=ybc)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ring = binding.Ring(plan, [dev(pr0.pn)], [dev(pr0.pnm1)])
    # explicit history on the same plan
    hn, hm = dev(pr0.pn), dev(pr0.pnm1)
    # oracle loop
    g = O.Grid(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, ybc=ybc)
    on, om = pr0.pn.copy(), pr0.pnm1.copy()
    for t, pr in enumerate(steps):
        f = binding.to_device(pr)
        u, v, w = torch.empty_like(f["us"]), torch.empty_like(f["vs"]), torch.empty_like(f["ws"])
        info, _ = ring.step([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["S"]], [u], [v], [w])
        p_ring = torch.empty_like(f["rho"])
        ring.read(0, [p_ring])
        # explicit
        p = torch.empty_like(f["rho"])
        u2, v2, w2 = torch.empty_like(u), torch.empty_like(v), torch.empty_like(w)
        info2 = plan.solve([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [hn], [hm], [f["S"]], [p])
        plan.correct([pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [hn], [hm], [p], [f["S"]], [u2], [v2],
                     [w2], info2)
        torch.cuda.synchronize()
        assert torch.equal(p_ring, p) and torch.equal(u, u2) and torch.equal(v, v2) and torch.equal(w, w2)
        hm, hn = hn, p
        # oracle
        ref = O.ppe_step(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, on, om, pr.S)
        om, on = on, ref["p"]
        e = PU.errors(pr, {"p": p.cpu().numpy(), "u": u.cpu().numpy(), "v": v.cpu().numpy(),
                           "w": w.cpu().numpy()}, ref)
        rec = binding.decode_info(info)[0]
        print(f"ybc={ybc} step {t}: {e} eps_div={rec['res_rel']:.2e}", flush=True)
        assert e["eps_p"] <= 1e-12 and e["eps_du"] <= 1e-12 and e["inf_p"] <= 1e-12 and rec["status"] == 0
        assert max(e["inf_du"], e["inf_dv"], e["inf_dw"]) <= 1e-11
    assert ring.steps == T
    prev = torch.empty_like(hn)
    ring.read(1, [prev])
    torch.cuda.synchronize()
    assert torch.equal(prev, hm)
    ring.close()
    plan.close()


@pytest.mark.parametrize("ybc", [0, 1])
def test_ring_256x128x256_against_oracle_loop(ybc):
    """The time-loop benchmark's grid: two ring steps against the oracle's
    time loop, every point."""
    torch = _torch()
    shape = (256, 128, 256)
    steps = step_inputs(shape, ybc, 2)
    pr0 = steps[0]
    plan = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, ybc=ybc)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ring = binding.Ring(plan, [dev(pr0.pn)], [dev(pr0.pnm1)])
    g = O.Grid(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, ybc=ybc)
    on, om = pr0.pn.copy(), pr0.pnm1.copy()
    for t, pr in enumerate(steps):
        f = binding.to_device(pr)
        u, v, w = torch.empty_like(f["us"]), torch.empty_like(f["vs"]), torch.empty_like(f["ws"])
        info, _ = ring.step([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["S"]], [u], [v], [w])
        p = torch.empty_like(f["rho"])
        ring.read(0, [p])
        torch.cuda.synchronize()
        ref = O.ppe_step(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, on, om, pr.S)
        om, on = on, ref["p"]
        e = PU.errors(pr, {"p": p.cpu().numpy(), "u": u.cpu().numpy(), "v": v.cpu().numpy(),
                           "w": w.cpu().numpy()}, ref)
        rec = binding.decode_info(info)[0]
        print(f"ybc={ybc} step {t}: {e} eps_div={rec['res_rel']:.2e}", flush=True)
        assert e["eps_p"] <= 1e-12 and e["eps_du"] <= 1e-12 and e["inf_p"] <= 1e-12
        assert max(e["inf_du"], e["inf_dv"], e["inf_dw"]) <= 1e-11
        assert rec["status"] == 0 and rec["res_rel"] <= 1e-12
        del f, u, v, w, p
    ring.close()
    plan.close()


def test_ring_without_previous_pressure_uses_p_n():
    torch = _torch()
    pr = synth.sheet_problem(16, 8, 12, seed=31)
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    f = binding.to_device(pr)
    ring = binding.Ring(plan, [f["pn"]])
    u, v, w = torch.empty_like(f["us"]), torch.empty_like(f["vs"]), torch.empty_like(f["ws"])
    ring.step([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["S"]], [u], [v], [w])
    p = torch.empty_like(f["rho"])
    ring.read(0, [p])
    torch.cuda.synchronize()
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    ref = O.ppe_step(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pn, pr.S)
    assert rel(p.cpu().numpy(), ref["p"]) <= 1e-12
    ring.close()
    plan.close()


@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
@pytest.mark.parametrize("ybc", [0, 1])
def test_split_defect_each_step(ybc, precision):
    """The diagnostic evaluates Eq. (25)'s residual for p_hat and for the
    split pressure after the solve: the ring's pressures and velocities are
    bitwise those of a ring without it, in both precisions (a mixed plan's
    pressure is the refined one), and the two residuals match the oracle's."""
    torch = _torch()
    shape = (24, 16, 32)
    T = 3
    steps = step_inputs(shape, ybc, T)
    pr0 = steps[0]
    kw = dict(ybc=ybc, precision=precision, tol=1e-12, max_refine=2)
    plan = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, flags=binding.PPE_FLAG_VARCOEF, **kw)
    plain = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, **kw)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ring = binding.Ring(plan, [dev(pr0.pn)], [dev(pr0.pnm1)])
    ring0 = binding.Ring(plain, [dev(pr0.pn)], [dev(pr0.pnm1)])
    g = O.Grid(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, ybc=ybc)
    on, om = pr0.pn.copy(), pr0.pnm1.copy()
    for t, pr in enumerate(steps):
        f = binding.to_device(pr)
        outs = [[torch.empty_like(f[k])] for k in ("us", "vs", "ws")]
        outs0 = [[torch.empty_like(f[k])] for k in ("us", "vs", "ws")]
        info, d = ring.step([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["S"]], *outs,
                            defect=True)
        ring0.step([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["S"]], *outs0)
        p, p0 = torch.empty_like(f["rho"]), torch.empty_like(f["rho"])
        ring.read(0, [p])
        ring0.read(0, [p0])
        torch.cuda.synchronize()
        rec = binding.decode_info(info)[0]
        ref = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, on, om, pr.S, 1)
        dd = d.cpu().numpy()
        print(f"ybc={ybc} step {t}: defect p_hat={dd[0]:.3e} split={dd[1]:.3e} (oracle {ref['res'][0]:.3e}, "
              f"{ref['res'][1]:.3e}) eps_div={rec['res_rel']:.2e}", flush=True)
        assert rec["status"] == 0 and rec["res_rel"] <= 1e-12
        assert abs(dd[0] - ref["res"][0]) <= 1e-9 * ref["res"][0]
        assert abs(dd[1] - ref["res"][1]) <= 1e-9 * ref["res"][1]
        assert torch.equal(p, p0)
        for a, b in zip(outs, outs0):
            assert torch.equal(a[0], b[0])
        assert rel(p.cpu().numpy(), ref["p"]) <= 1e-12
        om, on = on, ref["p"]
    ring.close()
    ring0.close()
    plan.close()
    plain.close()
