"""Pins of the oracle's whole projection step (assembly, solve, correction:
Sec. 5.4, Eqs. 28-29) to closed-form problems: at uniform density a velocity
u* whose divergence is a discrete eigenfunction times its eigenvalue has that
eigenfunction as its exact pressure (tests/closed_modes.py).  The existing
eigenmode pins check the Laplacian and the spectral solve alone; these go
through the assembly of the right-hand side and Eq. (28) as well, for both y
boundaries, with every mode on its own and all of them summed.  Where a high
mode meets a very smooth one (2048 x 3 x 4), the FP64 rounding of the
right-hand side alone moves any solver's pressure by up to eps times the
ratio of their eigenvalues (closed_modes.rounding_bound); that is the bound
there."""
import numpy as np
import pytest

import closed_modes as CM
import oracle as O

SHAPES = [(8, 4, 8), (12, 6, 9), (6, 5, 12), (9, 7, 10), (32, 16, 24), (16, 1, 8), (1, 8, 4), (4, 8, 1), (2, 2, 2),
          (2048, 3, 4), (24, 3, 1536)]
L = (2.0, 1.5, 3.0)


def _maxrel(a, b, scale):
    return float(np.abs(a - b).max() / scale)


def check(g, fields, ex, tol_p=1e-12, tol_du=1e-11):
    r = O.ppe_step(g, 640.0, 1e-3, *fields)
    e = {"p": _maxrel(r["p"], ex["p"], np.abs(ex["p"]).max())}
    dmax = max(np.abs(ex[c] - f).max() for c, f in zip("uvw", fields[:3]))
    for c, f in zip("uvw", fields[:3]):
        e[c] = _maxrel(r[c] - f, ex[c] - f, dmax)
    assert e["p"] <= tol_p, e
    for c in "uvw":
        assert e[c] <= tol_du, e
    return e


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_each_mode_is_reproduced(shape, ybc):
    nx, ny, nz = shape
    g = O.Grid(nx, ny, nz, *L, ybc=ybc)
    modes = CM.standard_modes(nx, ny, nz, ybc)
    if nx * ny * nz > 1:
        assert modes
    for md in modes:
        fields, ex = CM.mode_problem(nx, ny, nz, *L, ybc, [md])
        check(g, fields, ex, tol_p=max(1e-12, CM.rounding_bound(nx, ny, nz, *L, ybc, [md])))


@pytest.mark.parametrize("ybc", [0, 1])
def test_sum_of_modes(ybc):
    nx, ny, nz = 24, 12, 18
    g = O.Grid(nx, ny, nz, *L, ybc=ybc)
    modes = CM.standard_modes(nx, ny, nz, ybc)
    amps = list(np.random.default_rng(11).uniform(0.5, 2.0, len(modes)))
    fields, ex = CM.mode_problem(nx, ny, nz, *L, ybc, modes, amps=amps)
    check(g, fields, ex)


def test_closed_forms_catch_a_wrong_eigenvalue():
    """The construction is sharp: the same u* with the pressure of a
    neighbouring y mode is far outside the bound (so a mistake in one
    direction's eigenvalue or boundary row cannot pass)."""
    nx, ny, nz = 12, 6, 9
    g = O.Grid(nx, ny, nz, *L)
    fields, ex = CM.mode_problem(nx, ny, nz, *L, 0, [(2, 1, 3)])
    _, other = CM.mode_problem(nx, ny, nz, *L, 0, [(2, 2, 3)])
    r = O.ppe_step(g, 640.0, 1e-3, *fields)
    assert _maxrel(r["p"], other["p"], 1.0) > 0.1
    # the outflow eigenfunctions differ from the wall ones
    _, out = CM.mode_problem(nx, ny, nz, *L, 1, [(2, 1, 3)])
    assert _maxrel(r["p"], out["p"], 1.0) > 0.1
