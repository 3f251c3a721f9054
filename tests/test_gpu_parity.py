"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerance: every result within 1e-12 relative to the oracle (the target the
projection step is specified to), measured as
  eps_p  = ||p - p_o|| / ||p_o||              (both zero-mean)
  eps_du = ||(u - u*) - (u_o - u*)|| / ||u_o - u*||   (the correction itself)
  eps_div = ||D u - S_c|| / ||D u* - S_c||     (from the library's own check)
and pointwise: max|p - p_o| <= 1e-12 max|p_o|, and for each velocity
component max|du - du_o| <= 1e-11 max|du_o| (parity_util.check).
The FP64 path is expected near 1e-14; the mixed path must reach 1e-12 after
refinement.  Where the problem's own FP64 conditioning puts 1e-12 out of
reach of any solver (random fields at ny ~ 2048, pressures dominated by a mode
of tiny eigenvalue), the bound is taken from the oracle on the same input --
its change under a one-ulp move of the inputs, or its own divergence figure --
never from the GPU; each such test states which.
"""
import numpy as np
import pytest

import oracle as O
import parity_util as PU
from paper_2103_01874_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = PU.TOL


def _torch():
    import torch
    return torch


def gpu_step(problems, precision=binding.PPE_PREC_FP64, tol=1e-12, max_refine=2, rho0=None, flags=0):
    torch = _torch()
    pr0 = problems[0]
    plan = binding.Plan(pr0.nx, pr0.ny, pr0.nz, pr0.lx, pr0.ly, pr0.lz, precision=precision, tol=tol,
                        max_refine=max_refine, batch=len(problems), ybc=pr0.ybc, flags=flags)
    fields = [binding.to_device(pr) for pr in problems]
    r0 = [pr.rho0 for pr in problems] if rho0 is None else rho0
    outs, info = binding.step(plan, fields, r0, [pr.dt for pr in problems])
    torch.cuda.synchronize()
    res = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    recs = binding.decode_info(info)
    plan.close()
    return res, recs


oracle_step = PU.oracle_step
errors = PU.errors
check = PU.check


TINY = [(6, 4, 6), (12, 5, 9), (8, 3, 4), (4, 2, 3), (9, 7, 12), (1, 4, 8), (8, 4, 1), (32, 16, 24),
        (96, 24, 48), (48, 33, 18)]


@pytest.mark.parametrize("shape", TINY)
def test_fp64_random_fields_tiny(shape):
    pr = synth.random_problem(*shape, seed=sum(shape))
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr))


def test_fp64_dense_oracle_tiny():
    pr = synth.random_problem(6, 5, 6, seed=3)
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr, method="dense"))


def test_fp64_sheet_32():
    pr = synth.sheet_32()
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr))


def test_fp64_rho0_from_min():
    pr = synth.sheet_problem(16, 8, 12, seed=5, rho_g=77.0)
    (got,), (rec,) = gpu_step([pr], rho0=[-1.0])
    ref = oracle_step(pr, rho0=-1.0)
    assert rec["rho0_used"] == float(pr.rho.min())
    check(pr, got, rec, ref)


def test_fp64_sheet_256x128x256_full_oracle():
    pr = synth.sheet_256()
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr, ))


# x and z lengths 512..2048 run the compile-time FFT plans: at 512 a row
# transform fills one wavefront (the real FFTs exchange the mirror half of
# the spectrum with a partner lane across all 64 lanes); above it a transform
# spans several wavefronts and the mirror half goes through LDS or a second
# read.  z lengths above 1024 leave the column kernel fewer kx columns per
# block (4 at 1152..2048), so that a column still fits the LDS of a CU; 1152
# and 1536 run the run-time plan (radix 3); 96, 192 and 384 run compile-time
# plans with a radix-3 stage (12 values per thread).
LARGE_POW2 = [(512, 4, 16), (1024, 2, 16), (2048, 2, 8), (16, 4, 512), (16, 2, 1024), (512, 3, 512),
              (8, 2, 2048), (8, 3, 1536), (16, 2, 1152), (384, 4, 12), (12, 4, 384), (192, 3, 96)]


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
@pytest.mark.parametrize("shape", LARGE_POW2)
def test_large_power_of_two_lengths(shape, precision, ybc):
    pr = synth.random_problem(*shape, seed=7 + sum(shape) + ybc, ybc=ybc)
    # The refinement stops on the divergence residual; the pressure error can
    # exceed it by the conditioning of the solve, which FP32 spectra of long
    # transforms expose (16x2x1152, outflow: one sweep reaches eps_div 6.9e-13
    # and eps_p 1.1e-12).  The mixed runs therefore ask for 1e-13, so that p
    # meets the 1e-12 parity bound too.
    tol = 1e-12 if precision == binding.PPE_PREC_FP64 else 1e-13
    (got,), (rec,) = gpu_step([pr], precision=precision, tol=tol, max_refine=3)
    check(pr, got, rec, oracle_step(pr))


# The row transforms pack rows 2q and 2q + 1 into one complex FFT; an odd
# ny * nz leaves the last pair with one row.  Compile-time plans in one
# wavefront (16..512), across wavefronts (1024) and run-time plans (12, 96),
# with the refinement update of p in both precisions' paths.
ODD_ROWS = [(16, 3, 3), (64, 5, 9), (512, 3, 1), (256, 7, 3), (1024, 3, 3), (96, 5, 3), (12, 5, 9)]


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
@pytest.mark.parametrize("shape", ODD_ROWS)
def test_odd_row_count(shape, precision, ybc):
    pr = synth.random_problem(*shape, seed=11 + sum(shape) + ybc, ybc=ybc)
    tol = 1e-12 if precision == binding.PPE_PREC_FP64 else 1e-13
    (got,), (rec,) = gpu_step([pr], precision=precision, tol=tol, max_refine=3)
    if precision == binding.PPE_PREC_MIXED:
        assert rec["iters"] >= 1  # the update of p ran
    check(pr, got, rec, oracle_step(pr))


LONG_Y = [(8, 2048, 4), (4, 1000, 6), (4, 2047, 4)]


def one_ulp_sensitivity(pr, ref):
    """||p(inputs moved by one ulp, random signs) - p|| / ||p|| of the oracle:
    how far the FP64 rounding of the inputs alone moves the pressure."""
    rng = np.random.default_rng(0)
    moved = [np.nextafter(a, a + rng.choice([-1.0, 1.0], size=a.shape) * np.inf) for a in pr.fields()]
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    p2 = O.ppe_step(g, pr.rho0, pr.dt, *moved)["p"]
    return float(np.linalg.norm((p2 - ref["p"]).ravel()) / np.linalg.norm(ref["p"].ravel()))


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", LONG_Y)
def test_long_y_systems(shape, ybc):
    """ny up to 2048: 128 chunks of 16 rows and a 256-row reduced system per
    (kx, kz) (two systems per block); 1000 = 62 uneven chunks; 2047 uneven.

    The smoothest y mode has eigenvalue 4 sin^2(pi / 2 ny) ~ (pi / ny)^2, so
    random inputs whose rounding reaches that mode determine p only to about
    eps (ny / pi)^2 relative: two correct FP64 solvers differ by that much.  The
    pressure is held to 1e-12 or to twice the oracle's own change under a
    one-ulp move of its inputs, whichever is larger (measured at 4x2047x4 with
    the outflow top: 2.2e-12); the correction and the divergence to 1e-12."""
    pr = synth.random_problem(*shape, seed=3 + sum(shape) + ybc, ybc=ybc)
    (got,), (rec,) = gpu_step([pr])
    ref = oracle_step(pr)
    sens = one_ulp_sensitivity(pr, ref)
    print(f"oracle one-ulp sensitivity of p: {sens:.2e}", flush=True)
    check(pr, got, rec, ref, tol_p=max(TOL, 2.0 * sens))


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(8, 2048, 4), (4, 2047, 4)])
def test_long_y_systems_mixed(shape, ybc):
    """The refined y solve on FP32 spectra: FP32 rounding of the spectra is
    removed by the FP64 refinement sweeps, the elimination's loss on the
    smooth modes by the y refinement inside each solve.  Bounds as for the
    FP64 path; the divergence is asked for 1e-13 so that p meets its bound."""
    pr = synth.random_problem(*shape, seed=3 + sum(shape) + ybc, ybc=ybc)
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, tol=1e-13, max_refine=4)
    ref = oracle_step(pr)
    sens = one_ulp_sensitivity(pr, ref)
    print(f"oracle one-ulp sensitivity of p: {sens:.2e}", flush=True)
    check(pr, got, rec, ref, tol_p=max(TOL, 2.0 * sens))


def y_only_problem(shape, ybc):
    """u* = 0, uniform density, no history, S a function of y alone: the
    pressure is carried by the kx = kz = 0 system alone, mostly by its
    smoothest mode."""
    pr = synth.random_problem(*shape, seed=11, ybc=ybc)
    ny = shape[1]
    yv = (np.arange(ny) + 0.5) / ny
    prof = np.cos(np.pi * yv) + 0.3 * np.sin(5 * np.pi * yv) + 0.05 * np.random.default_rng(1).standard_normal(ny)
    for a in (pr.us, pr.vs, pr.ws, pr.pn, pr.pnm1):
        a[...] = 0.0
    pr.rho[...] = pr.rho.mean()
    pr.S[...] = prof[None, :, None]
    if ybc == 0:
        pr.S[...] -= pr.S.mean()
    return pr


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(8, 2048, 4), (4, 2047, 4)])
def test_long_y_smooth_mode(shape, ybc):
    """The y solve alone on the system the smooth mode dominates: p and the
    correction to 1e-12 (without the difference-form residual sweep the
    elimination loses about 4 eps / (4 sin^2(pi / 2 ny)), ~1e-11 here).  The
    divergence of the corrected field is formed from a p of size ~(ny / pi)^2
    times its source, so its FP64 value carries about eps (ny / pi)^2 in any
    solver; it is held to four times the oracle's figure for its own solution
    (the same FP64 formula, rounded in another order)."""
    pr = y_only_problem(shape, ybc)
    (got,), (rec,) = gpu_step([pr])
    ref = oracle_step(pr)
    own = oracle_divergence(pr, ref)
    print(f"oracle's own eps_div: {own:.2e}", flush=True)
    check(pr, got, rec, ref, tol_div=max(TOL, 4.0 * own))


def oracle_divergence(pr, ref):
    """The oracle's relative divergence error for its own solution: for a
    smooth p of size ~b / lambda_min the FP64 rounding of D G p alone is
    ~4 eps / lambda_min of D u*, whatever solver produced p."""
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    return O.divergence_check(g, pr.us, pr.vs, pr.ws, pr.S, ref["u"], ref["v"], ref["w"])["rel"]


def wide_domain_problem(ybc):
    """A domain 400 long and 1 high, 128 x 64 x 4 cells,
    u* = 0, uniform density, no history, S = cos(2 pi x / lx) g(y) with a
    smooth g: the pressure lives in the kx = 1 systems, whose s = (dy k)^2 is
    about 6e-8."""
    pr = synth.random_problem(128, 64, 4, seed=19, lx=400.0, ly=1.0, ybc=ybc)
    yv = (np.arange(pr.ny) + 0.5) / pr.ny
    xv = (np.arange(pr.nx) + 0.5) * pr.lx / pr.nx
    g = np.cos(np.pi * yv) + 0.3 * np.sin(5 * np.pi * yv) + 0.2
    for a in (pr.us, pr.vs, pr.ws, pr.pn, pr.pnm1):
        a[...] = 0.0
    pr.rho[...] = pr.rho.mean()
    pr.S[...] = g[None, :, None] * np.cos(2 * np.pi * xv / pr.lx)[None, None, :]
    return pr


def gradient_sensitivity(pr, ref):
    """||G p' - G p|| / ||G p|| for p' = the oracle's p moved by one ulp
    (random signs): a p nearly constant in y has a y gradient that is a
    difference of nearly equal values, so even a correctly rounded p carries
    this much relative error into the correction."""
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    p = ref["p"]
    moved = np.nextafter(p, p + np.random.default_rng(0).choice([-1.0, 1.0], size=p.shape) * np.inf)
    a = np.concatenate([x.ravel() for x in O.gradient(g, p)])
    b = np.concatenate([x.ravel() for x in O.gradient(g, moved)])
    return float(np.linalg.norm(a - b) / np.linalg.norm(a))


def gradient_rounding_bound(pr, ref, ulps=16):
    """Pointwise form of the same effect: a pressure in error by `ulps` units
    in the last place of max|p| at each point (the forward error of an FFT
    solve, about log2(nx nz) + a few roundings per value) moves each face
    gradient by up to 2 ulps spacing(max|p|)/h; relative to the component's
    largest gradient, the largest over the components whose oracle gradient
    is not identically zero."""
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    p = ref["p"]
    dp = ulps * np.spacing(np.abs(p).max())
    out = 0.0
    for gc, h in zip(O.gradient(g, p), (g.dx, g.dy, g.dz)):
        m = np.abs(gc).max()
        if m > 0:
            out = max(out, 2.0 * dp / h / m)
    return out


@pytest.mark.parametrize("ybc", [0, 1])
def test_y_refine_flag_on_a_wide_domain(ybc):
    """PPE_FLAG_Y_REFINE at ny = 64: the zero-flux kx = 1 systems have their
    smallest eigenvalue s ~ 6e-8, where the elimination alone leaves ~1e-9
    of p; with the flag p reaches 1e-12.  (The outflow top keeps the smallest
    eigenvalue above 4 sin^2(pi / 256) and needs no refinement.)  The
    divergence is held as in the smooth-mode test above: at s ~ 6e-8 its FP64
    value carries ~1e-9 in any solver.  p is nearly constant in y there, and
    one ulp of p moves the correction by 8e-13 relative: the correction is
    held to twice that figure (at least 1e-12); pointwise, each component to
    what 16 ulps of max|p| at every point put through G (at least 1e-11)."""
    pr = wide_domain_problem(ybc)
    ref = oracle_step(pr)
    (plain,), (rec0,) = gpu_step([pr])
    print(f"without the flag: eps_p={errors(pr, plain, ref)['eps_p']:.2e}", flush=True)
    (got,), (rec,) = gpu_step([pr], flags=binding.PPE_FLAG_Y_REFINE)
    own = oracle_divergence(pr, ref)
    gsens = gradient_sensitivity(pr, ref)
    ginf = gradient_rounding_bound(pr, ref)
    print(f"oracle's own eps_div: {own:.2e}; one-ulp sensitivity of G p: {gsens:.2e}; "
          f"pointwise gradient bound {ginf:.2e}", flush=True)
    check(pr, got, rec, ref, tol_du=max(TOL, 2.0 * gsens), tol_div=max(TOL, 4.0 * own),
          tol_inf_du=max(10 * TOL, ginf))


def test_sheet_512x256x512_full_oracle_fp64_and_mixed():
    """The 512x256x512 sheet (rho 640/60, five interface modes) in the two
    launch configurations the benchmark times for it: the FP64 direct solve,
    and FP32 spectra with one FP64 refinement sweep.  Both against one FP64
    oracle solve, every point."""
    pr = synth.sheet_512()
    ref = oracle_step(pr)
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, ref)
    del got
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, max_refine=1)
    check(pr, got, rec, ref)
    assert rec["iters"] <= 1


@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 32, 48), (96, 64, 96)])
def test_mixed_refined_sheet(shape):
    pr = synth.sheet_problem(*shape, seed=11, rho_l=640.0, rho_g=60.0, nmodes=5)
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, tol=1e-12, max_refine=3)
    check(pr, got, rec, oracle_step(pr))
    assert 1 <= rec["iters"] <= 3


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(6, 5, 6), (8, 4, 8), (12, 5, 9), (16, 8, 16), (32, 16, 24)])
def test_mixed_random_fields_with_incompatible_source(shape, ybc):
    """Random S with a non-zero mean: with zero-flux ends the compatibility
    projection removes a large mean(b) that the refinement residual keeps; the
    residual must reach the FP32 spectra without it."""
    pr = synth.random_problem(*shape, seed=31, ybc=ybc)
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, tol=1e-12, max_refine=4)
    check(pr, got, rec, oracle_step(pr))


def test_mixed_taylor_green():
    pr = synth.sheet_problem(64, 32, 64, seed=12, rho_g=60.0, velocity="taylor_green", nmodes=5)
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, tol=1e-12, max_refine=3)
    check(pr, got, rec, oracle_step(pr))


def test_batched_equals_single_bitwise():
    probs = [synth.mixed_instance(100 + i, shape=(32, 16, 24)) for i in range(3)]
    batched, brecs = gpu_step(probs, precision=binding.PPE_PREC_MIXED, max_refine=2)
    for pr, b, br in zip(probs, batched, brecs):
        (single,), (sr,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, max_refine=2)
        for k in ("p", "u", "v", "w"):
            assert np.array_equal(b[k], single[k]), k
        assert br == sr


@pytest.mark.parametrize("precision", [binding.PPE_PREC_FP64, binding.PPE_PREC_MIXED])
@pytest.mark.parametrize("ybc", [0, 1])
def test_batched_refined_y_solve_equals_single_bitwise(ybc, precision):
    """ny > 256: the refining tridiagonal launch runs one block per listed
    (kx, kz) block and instance; a batch of three equals three single calls."""
    probs = [synth.random_problem(8, 300, 6, seed=60 + i, ybc=ybc) for i in range(3)]
    batched, brecs = gpu_step(probs, precision=precision, tol=1e-13, max_refine=3)
    for pr, b, br in zip(probs, batched, brecs):
        (single,), (sr,) = gpu_step([pr], precision=precision, tol=1e-13, max_refine=3)
        for k in ("p", "u", "v", "w"):
            assert np.array_equal(b[k], single[k]), k
        assert br == sr
    check(probs[1], batched[1], brecs[1], oracle_step(probs[1]))


def test_residual_entry_point():
    torch = _torch()
    pr = synth.sheet_problem(24, 12, 18, seed=9)
    (got,), (rec,) = gpu_step([pr])
    plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = plan.residual([dev(got["u"])], [dev(got["v"])], [dev(got["w"])], [dev(pr.S)])
    out0 = plan.residual([dev(pr.us)], [dev(pr.vs)], [dev(pr.ws)], [dev(pr.S)])
    torch.cuda.synchronize()
    o, o0 = out.cpu().numpy(), out0.cpu().numpy()
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    d0 = O.divergence(g, pr.us, pr.vs, pr.ws) - pr.S
    assert abs(o0[2] - d0.mean()) <= 1e-13 * np.abs(d0).max()
    assert abs(o0[0] - np.linalg.norm(d0 - d0.mean())) <= 1e-12 * np.linalg.norm(d0)
    assert o[0] <= 1e-12 * o0[0]
    plan.close()


# ---------------------------------------------------------------------------
# Symmetry-plane bottom, outflow (p = 0) top: the planar jets' y boundaries
# ---------------------------------------------------------------------------

OUTFLOW_TINY = [(6, 4, 6), (12, 5, 9), (8, 3, 4), (4, 2, 3), (9, 7, 12), (1, 4, 8), (8, 4, 1), (32, 16, 24),
                (48, 33, 18)]


@pytest.mark.parametrize("shape", OUTFLOW_TINY)
def test_outflow_fp64_random_fields_tiny(shape):
    pr = synth.random_problem(*shape, seed=7 * sum(shape), ybc=1)
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr))


def test_outflow_fp64_dense_oracle_tiny():
    pr = synth.random_problem(6, 5, 6, seed=4, ybc=1)
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr, method="dense"))


def test_outflow_fp64_jet_32():
    pr = synth.jet_32()
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr))


def test_outflow_fp64_jet_256x128x256_full_oracle():
    pr = synth.jet_256()
    (got,), (rec,) = gpu_step([pr])
    check(pr, got, rec, oracle_step(pr))


@pytest.mark.parametrize("shape", [(32, 32, 32), (96, 64, 96)])
def test_outflow_mixed_refined_jet(shape):
    pr = synth.jet_problem(*shape, seed=21, rho_l=640.0, rho_g=60.0, nmodes=5)
    (got,), (rec,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, tol=1e-12, max_refine=3)
    check(pr, got, rec, oracle_step(pr))
    assert 1 <= rec["iters"] <= 3


def test_outflow_batched_equals_single_bitwise():
    probs = [synth.jet_problem(24, 16, 32, seed=300 + i, rho_l=100.0 * (3 + i)) for i in range(3)]
    batched, brecs = gpu_step(probs, precision=binding.PPE_PREC_MIXED, max_refine=2)
    for pr, b, br in zip(probs, batched, brecs):
        (single,), (sr,) = gpu_step([pr], precision=binding.PPE_PREC_MIXED, max_refine=2)
        for k in ("p", "u", "v", "w"):
            assert np.array_equal(b[k], single[k]), k
        assert br == sr
