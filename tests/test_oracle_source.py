"""Pins for the oracle's target divergence S of Eq. (26).

Each expected value comes from outside the oracle's formula:
  * the paper's own reduction: away from the interface S is the compressibility
    of the one phase present (Sec. 5.4, the remark after Eq. 26);
  * the physical meaning of the volume-averaged compressibility: two parcels,
    of volumes (1 - C) V and C V, dilating at their own rates;
  * the velocity-jump condition across the interface (Sec. 2): a planar
    interface crossing one cell carries the normal jump
    (u_g - u_l).n = (1/rho_g - 1/rho_l) m', which the projected velocity must
    reproduce;
  * the treatment of under-resolved interface cells (S = 0 there; appendix on
    under-resolved regions);
  * brute-force loops on a tiny grid.
"""

import math

import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import synth


def random_inputs(shape, seed, garbage=np.nan):
    """Fields of the given shape; the interface-only arrays hold `garbage`
    outside interface cells, and each phase's divergence holds it in the cells
    of the other phase, to show they are never read there."""
    rng = np.random.default_rng(seed)
    C = rng.choice([0.0, 1.0, 0.5], size=shape, p=[0.4, 0.4, 0.2])
    C[C == 0.5] = rng.uniform(0.01, 0.99, size=int((C == 0.5).sum()))
    iface = (C > 0) & (C < 1)
    div_g = rng.standard_normal(shape)
    div_l = rng.standard_normal(shape)
    div_g[C == 1.0] = garbage   # undefined away from the band: never read
    div_l[C == 0.0] = garbage
    arrs = []
    for lo, hi in ((0.1, 1.0), (5.0, 20.0), (50.0, 150.0), (500.0, 800.0)):
        a = np.full(shape, garbage)
        a[iface] = rng.uniform(lo, hi, size=int(iface.sum()))
        arrs.append(a)
    under = (rng.uniform(size=shape) < 0.3).astype(np.uint8)
    return C, div_g, div_l, *arrs, under


def bf_source(C, div_g, div_l, mdot, area, rg, rl, under):
    out = np.empty(C.shape)
    for idx in np.ndindex(C.shape):
        c = C[idx]
        if 0.0 < c < 1.0:
            if under is not None and under[idx]:
                out[idx] = 0.0
            else:
                out[idx] = (1 - c) * div_g[idx] + c * div_l[idx] + mdot[idx] * area[idx] * (1 / rg[idx] - 1 / rl[idx])
        else:
            out[idx] = div_g[idx] if c == 0.0 else div_l[idx]
    return out


def test_brute_force_loops_and_gating():
    f = random_inputs((5, 6, 7), 1)
    S = O.source_term(*f)
    assert np.all(np.isfinite(S))
    assert np.allclose(S, bf_source(*f), rtol=1e-15, atol=0)


def test_single_phase_cells_are_the_phase_compressibility():
    C, dg, dl, m, a, rg, rl, under = random_inputs((4, 8, 6), 2)
    S = O.source_term(C, dg, dl, m, a, rg, rl, under)
    assert np.array_equal(S[C == 0.0], dg[C == 0.0])
    assert np.array_equal(S[C == 1.0], dl[C == 1.0])


@pytest.mark.parametrize("c", [0.1, 0.37, 0.5, 0.93])
def test_volume_averaged_compressibility_of_two_parcels(c):
    """Parcels (1-c)V and cV dilate at rates div_g and div_l; the mixture's
    relative volume rate is S (no phase change)."""
    dg, dl = 0.8, -0.3
    V = 1.0
    h = 1e-7
    Vn = (1 - c) * V * math.exp(dg * h) + c * V * math.exp(dl * h)
    rate = (Vn - V) / (V * h)
    one = np.ones((1, 1, 1))
    S = O.source_term(c * one, dg * one, dl * one, 0 * one, 0 * one, one, one)
    assert abs(S.item() - rate) < 1e-6


@pytest.mark.parametrize("ny,jc", [(16, 5), (24, 11)])
def test_phase_change_reproduces_the_velocity_jump(ny, jc):
    """Incompressible phases, a planar interface crossing cell row jc with
    A/V0 = 1/dy, liquid below at rest on the symmetry plane, outflow top.
    The projected v above the interface is (1/rho_g - 1/rho_l) m' (jump
    condition), and zero below."""
    nx, nz = 4, 3
    g = O.Grid(nx, ny, nz, 1.0, 1.0, 1.0, ybc=1)
    shape = g.shape
    C = np.zeros(shape)
    C[:, :jc, :] = 1.0
    C[:, jc, :] = 0.4
    mdot_area, rg, rl = 0.7, 90.0, 650.0
    f = (C, np.zeros(shape), np.zeros(shape), np.full(shape, mdot_area), np.full(shape, 1.0 / g.dy),
         np.full(shape, rg), np.full(shape, rl))
    S = O.source_term(*f)
    jump = (1 / rg - 1 / rl) * mdot_area
    assert abs(S.sum(axis=1)[0, 0] * g.dy - jump) < 1e-15
    rho = 100.0 + 540.0 * C
    z = np.zeros(shape)
    vs = np.zeros(g.vshape)
    out = O.ppe_step(g, -1.0, 1e-3, z, vs, z, rho, z, z, S)
    v = out["v"][0, :, 0]
    assert np.abs(v[: jc + 1]).max() < 1e-15
    assert np.abs(v[jc + 1:] - jump).max() < 1e-13 * jump
    assert np.abs(out["u"]).max() < 1e-13 and np.abs(out["w"]).max() < 1e-13


def test_under_resolved_interface_cells_are_zero():
    C, dg, dl, m, a, rg, rl, under = random_inputs((6, 5, 4), 3)
    S = O.source_term(C, dg, dl, m, a, rg, rl, under)
    S0 = O.source_term(C, dg, dl, m, a, rg, rl, None)
    iface = (C > 0) & (C < 1)
    masked = iface & (under != 0)
    assert masked.any() and (under[~iface] != 0).any()
    assert np.all(S[masked] == 0.0)
    assert np.array_equal(S[~masked], S0[~masked])
    assert np.all(S0[masked] != 0.0)


def test_generator_shapes_and_band():
    s = synth.sheet_sources(32, 16, 24, seed=5)
    iface = (s.C > 0) & (s.C < 1)
    assert iface.any()
    for a in (s.mdot_area, s.area_density, s.rho_g, s.rho_l):
        assert np.all(a[~iface] == 0.0) and np.all(a[iface] != 0.0)
    assert s.under.dtype == np.uint8 and 0 < s.under.mean() < 0.2
    S = O.source_term(*s.fields())
    assert np.all(np.isfinite(S))
