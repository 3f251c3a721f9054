"""GPU parity of the predictor, Eq. (23), against the oracle.

The increments u^p - u^n are compared (a large u^n would hide errors in the
update) at 1e-12 relative in the 2-norm and 1e-11 relative to the largest
increment pointwise; both sides take the SMART and central/upwind decisions
with the same products in FP64.  Grids whose nx is a multiple of 64 run the
LDS kernels: the slab-marching ones when the viscous-term velocity is the
advected one, else the one-slab tiles.  Those are also compared with the
one-thread-per-face kernels (PPE_TUNE_PREDICT_GLOBAL=1), which evaluate the
same expressions on the same values: to a few units in the last place of the
result (the kernels are compiled separately, and the compiler may fuse a
product and a sum into one FMA in one and not in the other).
"""
import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def random_inputs(g, seed):
    rng = np.random.default_rng(seed)
    sh, vs = g.shape, g.vshape
    C = rng.choice([0.0, 1.0], size=sh)
    m = rng.uniform(size=sh) < 0.3
    C[m] = rng.uniform(0.05, 0.95, size=int(m.sum()))
    ifc = (C > 0) & (C < 1)
    v = rng.uniform(-1, 1, vs)
    v[:, 0, :] = 0.0
    if g.ybc == 0:
        v[:, -1, :] = 0.0
    rho_n = 1.0 + 9.0 * C + 0.1 * rng.uniform(size=sh)
    return {"u": rng.uniform(-1, 1, sh), "v": v, "w": rng.uniform(-1, 1, sh), "rho_n": rho_n,
            "rho_np1": rho_n * (1.0 + 0.05 * rng.uniform(-1, 1, sh)),
            "mu": 0.01 + 0.05 * C + 0.01 * rng.uniform(size=sh), "C": C,
            "sigma": np.where(ifc, rng.uniform(0.5, 1.5, sh), 0.0),
            "kappa": np.where(ifc, rng.uniform(-3, 3, sh), 0.0), "rho_mean": 5.0, "dt": 2e-3}


def gpu_predict(g, recs):
    torch = _torch()
    plan = binding.Plan(g.nx, g.ny, g.nz, g.lx, g.ly, g.lz, batch=len(recs), ybc=g.ybc)
    dev = []
    for r in recs:
        d = {k: (torch.from_numpy(np.ascontiguousarray(v)).cuda() if isinstance(v, np.ndarray) else v)
             for k, v in r.items()}
        dev.append(d)
    up = [torch.empty(g.shape, dtype=torch.float64, device="cuda") for _ in recs]
    vp = [torch.empty(g.vshape, dtype=torch.float64, device="cuda") for _ in recs]
    wp = [torch.empty(g.shape, dtype=torch.float64, device="cuda") for _ in recs]
    plan.predict(dev, up, vp, wp)
    torch.cuda.synchronize()
    plan.close()
    return [(a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()) for a, b, c in zip(up, vp, wp)]


def oracle_predict(g, r):
    opt = {k: r[k] for k in ("uv", "vv", "wv", "fsx", "fsy", "fsz") if k in r}
    return O.predictor(g, r["dt"], r["rho_mean"], r["u"], r["v"], r["w"], r["rho_n"], r["rho_np1"], r["mu"],
                       r["C"], r["sigma"], r["kappa"], **opt)


def check(g, r, got, tag=""):
    ref = oracle_predict(g, r)
    for name, a, b, base in zip("uvw", got, ref, (r["u"], r["v"], r["w"])):
        da, db = a - base, b - base
        nrm = np.linalg.norm(db)
        e2 = np.linalg.norm(da - db) / nrm
        einf = np.abs(da - db).max() / np.abs(db).max()
        print(f"{tag} {name}: eps2={e2:.2e} epsinf={einf:.2e}", flush=True)
        assert e2 <= 1e-12 and einf <= 1e-11, (name, e2, einf)
    # wall faces keep v^n exactly
    assert np.array_equal(got[1][:, 0, :], r["v"][:, 0, :])
    if g.ybc == 0:
        assert np.array_equal(got[1][:, -1, :], r["v"][:, -1, :])


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(6, 5, 4), (8, 4, 6), (3, 6, 9), (1, 4, 2), (32, 16, 24), (48, 33, 18)])
def test_predict_random_fields(shape, ybc):
    g = O.Grid(*shape, 1.1, 0.8, 1.3, ybc=ybc)
    r = random_inputs(g, 7 * sum(shape) + ybc)
    (got,) = gpu_predict(g, [r])
    check(g, r, got, f"{shape} ybc={ybc}")


def test_predict_optional_fields_and_batch():
    g = O.Grid(16, 8, 12, 1.0, 1.0, 1.0, ybc=1)
    rng = np.random.default_rng(3)
    recs = []
    for s in range(3):
        r = random_inputs(g, 100 + s)
        r["uv"] = r["u"] + 0.1 * rng.standard_normal(g.shape)
        r["vv"] = r["v"] + 0.1 * rng.standard_normal(g.vshape)
        r["wv"] = r["w"] + 0.1 * rng.standard_normal(g.shape)
        r["fsx"] = rng.standard_normal(g.shape)
        r["fsy"] = rng.standard_normal(g.vshape)
        r["fsz"] = rng.standard_normal(g.shape)
        recs.append(r)
    got = gpu_predict(g, recs)
    for r, gg in zip(recs, got):
        check(g, r, gg, "opt")
        (alone,) = gpu_predict(g, [r])
        for a, b in zip(alone, gg):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("ybc", [0, 1])
def test_predict_sheet_256x128x256(ybc):
    pr = synth.sheet_256() if ybc == 0 else synth.jet_256()
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=ybc)
    r = synth.predictor_inputs(pr, 11)
    (got,) = gpu_predict(g, [r])
    check(g, r, got, f"sheet ybc={ybc}")


def test_predict_then_project_matches_oracle_chain():
    """Eq. (23) -> (29) -> (28): the predicted field projected on the GPU
    against the same chain in the oracle."""
    torch = _torch()
    pr = synth.sheet_problem(48, 32, 36, seed=21, nmodes=3)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    r = synth.predictor_inputs(pr, 12)
    up_o, vp_o, wp_o = oracle_predict(g, r)
    ref = O.ppe_step(g, pr.rho0, pr.dt, up_o, vp_o, wp_o, r["rho_np1"], pr.pn, pr.pnm1, pr.S)
    (up, vp, wp), = gpu_predict(g, [r])
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    f = {"us": dev(up), "vs": dev(vp), "ws": dev(wp), "rho": dev(r["rho_np1"]), "pn": dev(pr.pn),
         "pnm1": dev(pr.pnm1), "S": dev(pr.S)}
    outs, info = binding.step(plan, [f], [pr.rho0], [pr.dt])
    torch.cuda.synchronize()
    rec = binding.decode_info(info)[0]
    p = outs[0]["p"].cpu().numpy()
    assert rec["status"] == 0 and rec["res_rel"] <= 1e-12
    assert np.linalg.norm(p - ref["p"]) <= 1e-12 * np.linalg.norm(ref["p"])
    plan.close()


def test_predict_rejects_small_ny_and_bad_dt():
    torch = _torch()
    g = O.Grid(8, 3, 8)
    plan = binding.Plan(8, 3, 8)
    r = random_inputs(O.Grid(8, 3, 8), 1)
    d = {k: (torch.from_numpy(np.ascontiguousarray(v)).cuda() if isinstance(v, np.ndarray) else v) for k, v in r.items()}
    out = [torch.empty(g.shape, dtype=torch.float64, device="cuda")]
    outv = [torch.empty(g.vshape, dtype=torch.float64, device="cuda")]
    with pytest.raises(binding.PPEError):
        plan.predict([d], out, outv, out)
    plan.close()
    g = O.Grid(8, 4, 8)
    plan = binding.Plan(8, 4, 8)
    r = random_inputs(g, 2)
    r["dt"] = 0.0
    d = {k: (torch.from_numpy(np.ascontiguousarray(v)).cuda() if isinstance(v, np.ndarray) else v) for k, v in r.items()}
    out = [torch.empty(g.shape, dtype=torch.float64, device="cuda")]
    outv = [torch.empty(g.vshape, dtype=torch.float64, device="cuda")]
    with pytest.raises(binding.PPEError):
        plan.predict([d], out, outv, out)
    plan.close()


TILED = [(64, 4, 1), (64, 5, 6), (128, 33, 18), (192, 7, 3), (64, 13, 2), (128, 8, 8)]


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", TILED)
def test_tiled_kernels_against_oracle_and_per_face_kernels(shape, ybc, monkeypatch):
    """Partial y and z tiles (ny, nz not multiples of 4), one to three
    planes, the smallest ny, x halos wrapping at both ends of a single tile,
    and the optional fields on every other shape."""
    g = O.Grid(*shape, 1.1, 0.8, 1.3, ybc=ybc)
    r = random_inputs(g, 11 * sum(shape) + ybc)
    if sum(shape) % 2 == 0:
        rng = np.random.default_rng(sum(shape))
        r["uv"] = r["u"] + 0.1 * rng.standard_normal(g.shape)
        r["vv"] = r["v"] + 0.1 * rng.standard_normal(g.vshape)
        r["wv"] = r["w"] + 0.1 * rng.standard_normal(g.shape)
        r["fsx"] = rng.standard_normal(g.shape)
        r["fsy"] = rng.standard_normal(g.vshape)
        r["fsz"] = rng.standard_normal(g.shape)
    (tiled,) = gpu_predict(g, [r])
    check(g, r, tiled, f"tiled {shape} ybc={ybc}")
    monkeypatch.setenv("PPE_TUNE_PREDICT_GLOBAL", "1")
    (per_face,) = gpu_predict(g, [r])
    for name, a, b in zip("uvw", tiled, per_face):
        d = np.abs(a - b).max()
        assert d <= 4 * np.finfo(np.float64).eps * np.abs(b).max(), (name, d)


@pytest.mark.parametrize("run", [1, 3, 7])
@pytest.mark.parametrize("ybc", [0, 1])
def test_march_run_lengths(run, ybc, monkeypatch):
    """Marches of 1, 3 and 7 slabs (runs that end mid-grid and a last run
    that is shorter), each against the oracle and the per-face kernels."""
    g = O.Grid(64, 13, 12, 1.1, 0.8, 1.3, ybc=ybc)
    r = random_inputs(g, 500 + run + ybc)
    monkeypatch.setenv("PPE_TUNE_PREDICT_RUN", str(run))
    (march,) = gpu_predict(g, [r])
    check(g, r, march, f"march run={run} ybc={ybc}")
    monkeypatch.setenv("PPE_TUNE_PREDICT_GLOBAL", "1")
    (per_face,) = gpu_predict(g, [r])
    for name, a, b in zip("uvw", march, per_face):
        d = np.abs(a - b).max()
        assert d <= 4 * np.finfo(np.float64).eps * np.abs(b).max(), (name, d)


@pytest.mark.parametrize("separate_vis", [False, True])
def test_batched_lds_kernels_equal_alone(separate_vis):
    """Three instances in one launch of the march (shared viscous velocity)
    or the one-slab tiles (separate arrays): each equals its own launch
    bitwise and matches the oracle."""
    g = O.Grid(64, 9, 12, 1.0, 1.0, 1.0, ybc=1)
    rng = np.random.default_rng(41)
    recs = []
    for s in range(3):
        r = random_inputs(g, 300 + s)
        if separate_vis:
            r["uv"] = r["u"] + 0.1 * rng.standard_normal(g.shape)
            r["vv"] = r["v"] + 0.1 * rng.standard_normal(g.vshape)
            r["wv"] = r["w"] + 0.1 * rng.standard_normal(g.shape)
        recs.append(r)
    got = gpu_predict(g, recs)
    for r, gg in zip(recs, got):
        check(g, r, gg, f"batched separate={separate_vis}")
        (alone,) = gpu_predict(g, [r])
        for a, b in zip(alone, gg):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(64, 13, 12), (128, 33, 18), (192, 7, 3)])
def test_one_launch_equals_launch_per_component(shape, ybc, monkeypatch):
    """The three marches in one launch (block ranges padded to whole XCD
    rounds, counts not multiples of 8 here) against one launch per
    component: bitwise equal, two instances per launch."""
    g = O.Grid(*shape, 1.1, 0.8, 1.3, ybc=ybc)
    recs = [random_inputs(g, 700 + 3 * sum(shape) + s + ybc) for s in range(2)]
    one = gpu_predict(g, recs)
    monkeypatch.setenv("PPE_TUNE_PREDICT_SEPARATE", "1")
    sep = gpu_predict(g, recs)
    for r, a3, b3 in zip(recs, one, sep):
        check(g, r, a3, f"one launch {shape} ybc={ybc}")
        for a, b in zip(a3, b3):
            assert np.array_equal(a, b)
