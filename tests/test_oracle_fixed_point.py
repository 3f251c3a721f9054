"""Pins for the oracle's split fixed point (Sec. 5.4).

The split of Eq. (27) with p_hat fed back as the pressure is a map
F(p_hat) = L^+ [c + D(beta G p_hat)], c = (rho0/dt)(D u* - S_c), whose fixed
point is the pressure of Eq. (25) (the paper notes the split is exact when
grad p_hat equals grad p^{n+1}).  Its linear part M = L^+ D beta G contracts in
the energy norm ||e||_E = ||G e||_W (W = 1 on interior faces, 1/2 on an
outflow face, where D = -G^T W) by at most max beta = 1 - rho0/rho_max.

Independent facts used here: the iteration matrix and the operators built by
brute-force loops and a dense pseudo-inverse; the dense solution of Eq. (25);
the energy norm written as a sum over faces.
"""
import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import synth


def problem(shape, seed, ybc, **kw):
    return synth.random_problem(*shape, seed=seed, ybc=ybc, **kw)


def grid(pr):
    return O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)


def face_gradient_matrix(g):
    """Rows = faces (x faces, interior y faces, [top face], z faces), cols = cells."""
    nz, ny, nx = g.shape
    idx = lambda k, j, i: (k * ny + j) * nx + i
    rows = []
    w = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = np.zeros(g.npts)
                r[idx(k, j, i)] += 1 / g.dx
                r[idx(k, j, (i - 1) % nx)] -= 1 / g.dx
                rows.append(r)
                w.append(1.0)
                r = np.zeros(g.npts)
                r[idx(k, j, i)] += 1 / g.dz
                r[idx((k - 1) % nz, j, i)] -= 1 / g.dz
                rows.append(r)
                w.append(1.0)
                if j >= 1:
                    r = np.zeros(g.npts)
                    r[idx(k, j, i)] += 1 / g.dy
                    r[idx(k, j - 1, i)] -= 1 / g.dy
                    rows.append(r)
                    w.append(1.0)
                if j == ny - 1 and g.ybc == 1:
                    r = np.zeros(g.npts)
                    r[idx(k, j, i)] -= 2 / g.dy
                    rows.append(r)
                    w.append(0.5)
    return np.array(rows), np.array(w)


def face_rho(g, rho):
    """Face densities in the row order of face_gradient_matrix."""
    nz, ny, nx = g.shape
    out = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                out.append(0.5 * (rho[k, j, i] + rho[k, j, (i - 1) % nx]))
                out.append(0.5 * (rho[k, j, i] + rho[(k - 1) % nz, j, i]))
                if j >= 1:
                    out.append(0.5 * (rho[k, j, i] + rho[k, j - 1, i]))
                if j == ny - 1 and g.ybc == 1:
                    out.append(rho[k, j, i])
    return np.array(out)


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(4, 3, 4), (6, 4, 3)])
def test_energy_norm_is_the_weighted_face_sum(shape, ybc):
    pr = problem(shape, 5, ybc)
    g = grid(pr)
    G, w = face_gradient_matrix(g)
    e = np.random.default_rng(6).standard_normal(g.npts)
    want = np.sqrt(np.sum(w * (G @ e) ** 2))
    assert abs(O.energy_norm(g, e.reshape(g.shape)) - want) < 1e-12 * want
    # and L = -G^T W G
    assert np.abs(O.laplacian_matrix(g) + G.T @ (w[:, None] * G)).max() < 1e-10 * np.abs(G).max() ** 2


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(4, 3, 4), (6, 4, 3)])
def test_iteration_matrix_contracts_by_beta_max(shape, ybc):
    pr = problem(shape, 7, ybc)
    g = grid(pr)
    G, w = face_gradient_matrix(g)
    L = -G.T @ (w[:, None] * G)
    beta = 1.0 - pr.rho0 / face_rho(g, pr.rho)
    M = np.linalg.pinv(L) @ (-G.T @ (w[:, None] * (beta[:, None] * G)))
    bmax = 1.0 - pr.rho0 / pr.rho.max()
    rad = np.abs(np.linalg.eigvals(M)).max()
    assert rad <= bmax + 1e-12
    # the oracle's map has this linear part: F(a) - F(b) = M (a - b)
    z = np.zeros(g.shape)
    vz = np.zeros(g.vshape)
    a = np.random.default_rng(8).standard_normal(g.shape)
    Fa = O.split_map(g, pr.rho0, pr.dt, z, vz, z, pr.rho, z, a)
    want = (M @ a.ravel()).reshape(g.shape)
    if ybc == 0:
        want -= want.mean()
    assert np.abs(Fa - want).max() < 1e-10 * np.abs(want).max()
    # and its updates contract in the energy norm at the dense spectral radius
    out = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 60)
    u = out["upd_E"]
    assert all(u[k + 1] <= bmax * u[k] * (1 + 1e-9) for k in range(len(u) - 1))
    assert abs(u[-1] / u[-2] - rad) < 0.02


@pytest.mark.parametrize("ybc", [0, 1])
def test_fixed_point_is_the_variable_coefficient_pressure(ybc):
    pr = problem((6, 4, 6), 11, ybc)
    g = grid(pr)
    q = O.solve_variable_coefficient_dense(g, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.S)
    out = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 500, 1e-13)
    assert out["res"][-1] <= 1e-13
    assert np.linalg.norm(out["p"] - q) <= 1e-11 * np.linalg.norm(q)
    # p_1 is the split solve of the step
    one = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 1)
    step = O.ppe_step(g, pr.rho0, pr.dt, *pr.fields())
    assert np.array_equal(one["p"], step["p"])


@pytest.mark.parametrize("ybc", [0, 1])
def test_a_posteriori_bound_of_the_split(ybc):
    """||p_s - q||_E <= ||F(p_s) - p_s||_E / (1 - beta_max), and not vacuous."""
    pr = problem((6, 5, 6), 13, ybc)
    g = grid(pr)
    q = O.solve_variable_coefficient_dense(g, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.S)
    out = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 2)
    two = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 1)
    ps = two["p"]
    bound = out["upd_E"][1] / (1.0 - (1.0 - pr.rho0 / pr.rho.max()))
    err = O.energy_norm(g, ps - q)
    assert err <= bound * (1 + 1e-9)
    assert bound < 50 * err


def test_constant_density_converges_in_one_map():
    pr = problem((6, 4, 6), 17, 0)
    pr.rho[:] = 3.0
    pr.rho0 = 3.0
    g = grid(pr)
    out = O.split_fixed_point(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, pr.S, 5, 1e-13)
    assert out["iters"] == 1 and out["res"][-1] <= 1e-13
