"""GPU parity of the split fixed-point iteration (pressure of Eq. 25).

Against the oracle's split_fixed_point (the same sequence of iterates in
exact arithmetic) after a fixed number of sweeps, and against the dense
solution of Eq. (25) once converged.  FP64 iterates are held to 1e-12
relative; the residual history to 1e-8 relative where the residual is above
1e-9 (it is formed from those iterates).  Mixed plans use an FP32 inner solve,
so their iterates differ; only the converged pressure is compared.
"""
import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def gpu_varcoef(probs, max_iters, tol, precision=binding.PPE_PREC_FP64, correct=False):
    torch = _torch()
    pr0 = probs[0]
    plan = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, precision=precision, batch=len(probs),
                        ybc=pr0.ybc, flags=binding.PPE_FLAG_VARCOEF)
    fields = [binding.to_device(pr) for pr in probs]
    g = lambda k: [f[k] for f in fields]
    p = [torch.empty_like(f["rho"]) for f in fields]
    info, hist = plan.solve_varcoef([pr.rho0 for pr in probs], [pr.dt for pr in probs], g("us"), g("vs"), g("ws"),
                                    g("rho"), g("pn"), g("pnm1"), g("S"), p, max_iters, tol, hist=True)
    torch.cuda.synchronize()
    recs = binding.decode_info(info)
    outs = None
    if correct:
        outs = [{"u": torch.empty_like(f["us"]), "v": torch.empty_like(f["vs"]), "w": torch.empty_like(f["ws"])}
                for f in fields]
        plan.correct([pr.dt for pr in probs], g("us"), g("vs"), g("ws"), g("rho"), p, p, p, g("S"),
                     [o["u"] for o in outs], [o["v"] for o in outs], [o["w"] for o in outs], info)
        torch.cuda.synchronize()
        crecs = binding.decode_info(info)
        for o, c in zip(outs, crecs):
            o["info"] = c
    H = hist.cpu().numpy().reshape(len(probs), max_iters + 1)
    res = [x.cpu().numpy() for x in p]
    if outs is not None:
        outs = [{k: (v if k == "info" else v.cpu().numpy()) for k, v in o.items()} for o in outs]
    plan.close()
    return res, recs, H, outs


def oracle_fp(pr, iters, tol=0.0):
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    return g, O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, iters, tol)


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(6, 4, 6), (12, 5, 9), (32, 16, 24)])
def test_fixed_sweeps_match_oracle_iterates(shape, ybc):
    pr = synth.random_problem(*shape, seed=5 + sum(shape), ybc=ybc)
    K = 12
    (p,), (rec,), H, _ = gpu_varcoef([pr], K, 0.0)
    _, ref = oracle_fp(pr, K)
    print(f"{shape} ybc={ybc} eps_p={rel(p, ref['p']):.2e} res0={H[0, 0]:.3e} resK={H[0, K]:.3e}", flush=True)
    assert rel(p, ref["p"]) <= 1e-12
    assert rec["iters"] == K and rec["status"] == 0   # tol 0: sweeps without a convergence test
    r = np.array(ref["res"])
    big = r > 1e-9
    assert np.all(np.abs(H[0][big] - r[big]) <= 1e-8 * r[big])
    assert rec["res_rel"] == H[0, K]


@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
@pytest.mark.parametrize("ybc", [0, 1])
def test_converged_pressure_is_the_dense_variable_coefficient_solution(ybc, precision):
    pr = synth.random_problem(6, 5, 6, seed=31, ybc=ybc)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=ybc)
    q = O.solve_variable_coefficient_dense(g, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.S)
    (p,), (rec,), H, (out,) = gpu_varcoef([pr], 600, 1e-12, precision, correct=True)
    print(f"ybc={ybc} prec={precision} iters={rec['iters']} res={rec['res_rel']:.2e} eps_q={rel(p, q):.2e}",
          flush=True)
    assert rec["status"] == 0 and rec["res_rel"] <= 1e-12
    assert rel(p, q) <= 1e-10
    k = rec["iters"]
    assert H[0, k] == rec["res_rel"] and np.all(H[0, k + 1:] == -1.0)
    # the variable-density projection u = u* - dt G q / rho_f
    rx, ry, rz = O.face_density(pr.rho)
    gx, gy, gz = O.gradient(g, q)
    u_ref = pr.us - pr.dt * gx / rx
    assert rel(out["u"] - pr.us, u_ref - pr.us) <= 1e-10
    chk = O.divergence_check(g, pr.us, pr.vs, pr.ws, pr.S, out["u"], out["v"], out["w"])
    assert chk["rel"] <= 1e-11
    # its relative divergence error is the last residual of the iteration
    assert abs(out["info"]["res_rel"] - rec["res_rel"]) <= 1e-3 * rec["res_rel"] + 1e-15


def test_one_sweep_is_the_split_solve():
    torch = _torch()
    pr = synth.sheet_problem(32, 16, 24, seed=41)
    (p,), (rec,), H, _ = gpu_varcoef([pr], 1, 0.0)
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    outs, info = binding.step(plan, [binding.to_device(pr)], [pr.rho0], [pr.dt])
    torch.cuda.synchronize()
    assert rel(p, outs[0]["p"].cpu().numpy()) <= 1e-12
    plan.close()


def test_sheet_contracts_within_the_bound_and_batches_bitwise():
    probs = [synth.sheet_problem(48, 32, 36, seed=50 + i, rho_l=640.0, rho_g=100.0 * (1 + i)) for i in range(2)]
    K = 15
    ps, recs, H, _ = gpu_varcoef(probs, K, 0.0)
    for i, pr in enumerate(probs):
        _, ref = oracle_fp(pr, K)
        assert rel(ps[i], ref["p"]) <= 1e-12
        bmax = 1.0 - pr.rho0 / pr.rho.max()
        h = H[i]
        print(f"bmax={bmax:.3f} res={h[0]:.2e}..{h[K]:.2e} ratio={h[K] / h[K - 1]:.3f}", flush=True)
        (alone,), (ra,), Ha, _ = gpu_varcoef([pr], K, 0.0)
        assert np.array_equal(alone, ps[i]) and np.array_equal(Ha[0], H[i])


def test_fixed_sweeps_sheet_256x128x256():
    """The 256x128x256 sheet of the fixed-point benchmark, in its launch
    configuration: four sweeps against the oracle's iterates, every point."""
    pr = synth.sheet_256()
    K = 4
    (p,), (rec,), H, _ = gpu_varcoef([pr], K, 0.0)
    _, ref = oracle_fp(pr, K)
    print(f"eps_p={rel(p, ref['p']):.2e} res={H[0, :K + 1]}", flush=True)
    assert rel(p, ref["p"]) <= 1e-12
    r = np.array(ref["res"])
    assert np.all(np.abs(H[0][: K + 1] - r[: K + 1]) <= 1e-8 * r[: K + 1])


def test_not_converged_status():
    pr = synth.random_problem(8, 4, 8, seed=9)
    (p,), (rec,), H, _ = gpu_varcoef([pr], 3, 1e-14)
    assert rec["status"] == binding.PPE_ERR_NOT_CONVERGED and rec["iters"] == 3
    assert rec["res_rel"] == H[0, 3] > 1e-14


def test_needs_the_residual_buffer():
    torch = _torch()
    pr = synth.random_problem(8, 4, 8, seed=3)
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)   # FP64 without the flag
    f = binding.to_device(pr)
    p = torch.empty_like(f["rho"])
    with pytest.raises(binding.PPEError):
        plan.solve_varcoef([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["pn"]],
                           [f["pnm1"]], [f["S"]], [p], 3, 1e-12)
    plan.close()
    assert binding.workspace_bytes(binding.make_desc(8, 4, 8, flags=binding.PPE_FLAG_VARCOEF)) - \
        binding.workspace_bytes(binding.make_desc(8, 4, 8)) == 8 * 8 * 4 * 8
    # a mixed plan holds only the FP32 residual of its refinement: it needs the
    # flag for the fixed-point iteration too
    mixed = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=binding.PPE_PREC_MIXED)
    with pytest.raises(binding.PPEError):
        mixed.solve_varcoef([pr.rho0], [pr.dt], [f["us"]], [f["vs"]], [f["ws"]], [f["rho"]], [f["pn"]],
                            [f["pnm1"]], [f["S"]], [p], 3, 1e-12)
    mixed.close()
