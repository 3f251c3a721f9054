"""Pins for the CPU oracle, against facts that do not come from the oracle itself.

Each test cites what fixes the expected value: a closed form of the discrete
operators, an independently built matrix, brute-force loops on tiny grids, or
an identity the paper states (Sec. 5.4: the split is exact when grad p_hat
equals grad p^{n+1}; rho0 = min rho; the projected field meets the target
divergence).  A plausible slip in the oracle (a dropped term, a wrong sign or
index, a transposed operand) fails at least one of them.
"""

import numpy as np
import pytest

import oracle as O
from paper_2103_01874_amd import synth

TINY = [(6, 4, 6), (12, 5, 9), (8, 3, 4), (4, 6, 3), (9, 4, 8)]


# ---------------------------------------------------------------------------
# Independent brute-force discretisation (explicit loops, tiny grids only)
# ---------------------------------------------------------------------------

def bf_div(g, u, v, w):
    nz, ny, nx = g.shape
    out = np.zeros(g.shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                out[k, j, i] = ((u[k, j, (i + 1) % nx] - u[k, j, i]) / g.dx
                                + (v[k, j + 1, i] - v[k, j, i]) / g.dy
                                + (w[(k + 1) % nz, j, i] - w[k, j, i]) / g.dz)
    return out


def bf_face_fluxes(g, p, coef_x, coef_y, coef_z):
    """Face fluxes coef(rho_a, rho_b) * (p_b - p_a)/h; wall y-faces carry zero."""
    nz, ny, nx = g.shape
    fx = np.zeros((nz, ny, nx))
    fy = np.zeros((nz, ny + 1, nx))
    fz = np.zeros((nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                im = (i - 1) % nx
                fx[k, j, i] = coef_x(k, j, im, i) * (p[k, j, i] - p[k, j, im]) / g.dx
                km = (k - 1) % nz
                fz[k, j, i] = coef_z(km, j, i, k) * (p[k, j, i] - p[km, j, i]) / g.dz
                if j >= 1:
                    fy[k, j, i] = coef_y(k, j - 1, i, j) * (p[k, j, i] - p[k, j - 1, i]) / g.dy
    return fx, fy, fz


def bf_rhs(g, rho0, dt, us, vs, ws, rho, pn, pnm1, S):
    ph = 2 * pn - pnm1
    cx = lambda k, j, a, b: 1.0 - rho0 / (0.5 * (rho[k, j, a] + rho[k, j, b]))
    cy = lambda k, a, i, b: 1.0 - rho0 / (0.5 * (rho[k, a, i] + rho[k, b, i]))
    cz = lambda a, j, i, b: 1.0 - rho0 / (0.5 * (rho[a, j, i] + rho[b, j, i]))
    fx, fy, fz = bf_face_fluxes(g, ph, cx, cy, cz)
    return (rho0 / dt) * (bf_div(g, us, vs, ws) - S) + bf_div(g, fx, fy, fz)


def bf_correct(g, rho0, dt, us, vs, ws, rho, pn, pnm1, p):
    ph = 2 * pn - pnm1
    one = lambda *a: 1.0
    gx, gy, gz = bf_face_fluxes(g, p, one, one, one)
    hx, hy, hz = bf_face_fluxes(g, ph, one, one, one)
    nz, ny, nx = g.shape
    u, v, w = us.copy(), vs.copy(), ws.copy()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                rxf = 0.5 * (rho[k, j, i] + rho[k, j, (i - 1) % nx])
                u[k, j, i] = us[k, j, i] - dt * (gx[k, j, i] / rho0 + (1 / rxf - 1 / rho0) * hx[k, j, i])
                rzf = 0.5 * (rho[k, j, i] + rho[(k - 1) % nz, j, i])
                w[k, j, i] = ws[k, j, i] - dt * (gz[k, j, i] / rho0 + (1 / rzf - 1 / rho0) * hz[k, j, i])
                if j >= 1:
                    ryf = 0.5 * (rho[k, j, i] + rho[k, j - 1, i])
                    v[k, j, i] = vs[k, j, i] - dt * (gy[k, j, i] / rho0 + (1 / ryf - 1 / rho0) * hy[k, j, i])
    return u, v, w


def kron_laplacian(g):
    """L = Lz (x) I (x) I + I (x) Ly (x) I + I (x) I (x) Lx for C-order [z][y][x]."""
    def periodic(n, h):
        A = -2.0 * np.eye(n)
        for i in range(n):
            A[i, (i + 1) % n] += 1.0
            A[i, (i - 1) % n] += 1.0
        return A / h**2

    def neumann(n, h):
        A = np.zeros((n, n))
        for i in range(n):
            if i > 0:
                A[i, i - 1] += 1.0
                A[i, i] -= 1.0
            if i < n - 1:
                A[i, i + 1] += 1.0
                A[i, i] -= 1.0
        return A / h**2

    Ix, Iy, Iz = np.eye(g.nx), np.eye(g.ny), np.eye(g.nz)
    Lx, Ly, Lz = periodic(g.nx, g.dx), neumann(g.ny, g.dy), periodic(g.nz, g.dz)
    return np.kron(Lz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Ly, Ix)) + np.kron(Iz, np.kron(Iy, Lx))


def problem(shape, seed, **kw):
    nx, ny, nz = shape
    return synth.random_problem(nx, ny, nz, seed=seed, **kw)


def run(pr, **kw):
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    return g, O.ppe_step(g, pr.rho0, pr.dt, *pr.fields(), **kw)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ---------------------------------------------------------------------------
# 1. Closed-form eigenpairs of the staggered Laplacian
# ---------------------------------------------------------------------------

def _mode(g, a, m, c, phx=0.3, phz=1.1):
    i = np.arange(g.nx)
    j = np.arange(g.ny)
    k = np.arange(g.nz)
    fx = np.cos(2 * np.pi * a * i / g.nx + phx)
    fy = np.cos(np.pi * m * (j + 0.5) / g.ny)
    fz = np.cos(2 * np.pi * c * k / g.nz + phz)
    lam = (-(4 / g.dx**2) * np.sin(np.pi * a / g.nx) ** 2
           - (4 / g.dy**2) * np.sin(np.pi * m / (2 * g.ny)) ** 2
           - (4 / g.dz**2) * np.sin(np.pi * c / g.nz) ** 2)
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :], lam


@pytest.mark.parametrize("shape", [(8, 4, 8), (12, 6, 9), (6, 5, 12), (32, 16, 24), (96, 8, 6)])
def test_eigenmodes_closed_form(shape):
    g = O.Grid(*shape, lx=2.0, ly=1.5, lz=3.0)
    modes = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (g.nx // 2, 1, 2), (1, g.ny - 1, g.nz // 2),
             (g.nx // 2, g.ny - 1, g.nz // 2), (2, 2, g.nz - 1)]
    for a, m, c in modes:
        if g.nx % 2 == 0 and a == g.nx // 2:
            phx = 0.0  # the Nyquist cosine is the only real mode there
        else:
            phx = 0.3
        pe, lam = _mode(g, a, m, c, phx=phx)
        # the stencil reproduces the closed-form eigenvalue
        assert rel(O.laplacian(g, pe), lam * pe) < 1e-12
        # the spectral solve inverts it; a non-constant mode has zero mean
        assert rel(O.solve_spectral(g, lam * pe), pe - pe.mean()) < 1e-12


# ---------------------------------------------------------------------------
# 2. Dense direct solve and an independently assembled matrix
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", TINY)
def test_laplacian_matrix_matches_kronecker(shape):
    g = O.Grid(*shape, lx=1.3, ly=0.7, lz=2.1)
    assert np.allclose(O.laplacian_matrix(g), kron_laplacian(g), rtol=0, atol=1e-9 * np.max(np.abs(kron_laplacian(g))))


@pytest.mark.parametrize("shape", TINY)
def test_spectral_equals_dense_and_kronecker(shape):
    g = O.Grid(*shape, lx=1.3, ly=0.7, lz=2.1)
    b = np.random.default_rng(5).standard_normal(g.shape)
    ps = O.solve_spectral(g, b)
    pd = O.solve_dense(g, b)
    assert rel(ps, pd) < 1e-12
    A = kron_laplacian(g)
    # L p = b - mean(b) and mean(p) = 0 with a matrix the oracle never built
    assert rel(A @ ps.ravel(), (b - b.mean()).ravel()) < 1e-11
    assert abs(ps.mean()) < 1e-14 * np.abs(ps).max()
    # and against a plain least-squares solve of the singular system
    pl = np.linalg.lstsq(A, (b - b.mean()).ravel(), rcond=None)[0]
    assert rel(ps.ravel(), pl - pl.mean()) < 1e-10


# ---------------------------------------------------------------------------
# 3. Right-hand side and projection against brute-force loops
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", TINY[:3])
def test_rhs_and_projection_brute_force(shape):
    pr = problem(shape, 11)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    b = O.assemble_rhs(g, pr.rho0, pr.dt, *pr.fields())
    assert rel(b, bf_rhs(g, pr.rho0, pr.dt, *pr.fields())) < 1e-13
    p = np.random.default_rng(3).standard_normal(g.shape)
    got = O.correct(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, p)
    want = bf_correct(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, p)
    for a, c in zip(got, want):
        assert rel(a, c) < 1e-14
    # wall faces of v are left alone
    assert np.array_equal(got[1][:, 0, :], pr.vs[:, 0, :])
    assert np.array_equal(got[1][:, -1, :], pr.vs[:, -1, :])


# ---------------------------------------------------------------------------
# 4. Continuity of the projected field, for variable density
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(6, 4, 6), (12, 5, 9), (16, 8, 16)])
def test_projected_divergence_is_machine_zero(shape):
    pr = problem(shape, 21)
    g, out = run(pr)
    assert out["rel"] < 1e-13
    # recomputed with brute-force loops, independent of the oracle's check
    d = bf_div(g, out["u"], out["v"], out["w"]) - pr.S
    d0 = bf_div(g, pr.us, pr.vs, pr.ws) - pr.S
    Sc_shift = d0.mean()
    assert np.linalg.norm(d - Sc_shift) < 1e-12 * np.linalg.norm(d0 - Sc_shift)


def test_sheet_divergence_and_dense_parity():
    pr = synth.sheet_problem(8, 8, 8, seed=7, rho_l=640.0, rho_g=100.0, h0=0.3, modes=[(0.05, 1, 0.0, 1, 0.0)])
    g, a = run(pr, method="spectral")
    _, b = run(pr, method="dense")
    assert a["rel"] < 1e-13
    assert rel(a["p"], b["p"]) < 1e-12
    assert rel(a["u"] - pr.us, b["u"] - pr.us) < 1e-12


# ---------------------------------------------------------------------------
# 5. Constant density and gauge
# ---------------------------------------------------------------------------

def test_constant_density_ignores_pressure_history():
    pr = problem((8, 6, 8), 31)
    pr.rho[:] = 3.0
    pr.rho0 = 3.0
    g, a = run(pr)
    pr.pn = pr.pn * 5.0 + 1.0
    pr.pnm1 = np.random.default_rng(9).standard_normal(pr.shape)
    _, b = run(pr)
    assert rel(a["p"], b["p"]) < 1e-14
    assert rel(a["u"], b["u"]) < 1e-15


def test_gauge_and_constant_shift():
    pr = problem((10, 6, 8), 41)
    g, a = run(pr)
    assert abs(a["p"].mean()) < 1e-15 * np.abs(a["p"]).max()
    pr.pn = pr.pn + 123.0
    pr.pnm1 = pr.pnm1 - 7.0
    _, b = run(pr)
    assert rel(a["p"], b["p"]) < 1e-13
    assert rel(a["u"], b["u"]) < 1e-14


def test_rho0_default_is_minimum():
    pr = problem((6, 4, 6), 43)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    a = O.ppe_step(g, -1.0, pr.dt, *pr.fields())
    b = O.ppe_step(g, float(pr.rho.min()), pr.dt, *pr.fields())
    assert a["rho0"] == float(pr.rho.min())
    assert rel(a["p"], b["p"]) == 0.0


# ---------------------------------------------------------------------------
# 6. Exactness of the split (Sec. 5.4): p_hat equal to the variable-coefficient
#    pressure makes the split reproduce it.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(6, 4, 6), (8, 5, 6)])
def test_split_exact_when_phat_is_the_true_pressure(shape):
    pr = problem(shape, 51)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    q = O.solve_variable_coefficient_dense(g, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.S)
    # q solves Eq. (25) discretely: check with brute-force loops
    inv = lambda a, b: 1.0 / (0.5 * (a + b))
    rho = pr.rho
    fx, fy, fz = bf_face_fluxes(g, q,
                                lambda k, j, a, b: inv(rho[k, j, a], rho[k, j, b]),
                                lambda k, a, i, b: inv(rho[k, a, i], rho[k, b, i]),
                                lambda a, j, i, b: inv(rho[a, j, i], rho[b, j, i]))
    d0 = bf_div(g, pr.us, pr.vs, pr.ws) - pr.S
    assert rel(bf_div(g, fx, fy, fz), (d0 - d0.mean()) / pr.dt) < 1e-10
    # the split with p^n = p^{n-1} = q returns q, and the projection of Eq. (24)
    out = O.ppe_step(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, q, q, pr.S)
    assert rel(out["p"], q - q.mean()) < 1e-10
    u_exact = pr.us - pr.dt * fx
    assert rel(out["u"] - pr.us, u_exact - pr.us) < 1e-10


# ---------------------------------------------------------------------------
# 7. One-dimensional reduction: v^{n+1} integrates S_c along y
# ---------------------------------------------------------------------------

def test_one_dimensional_closed_form():
    nx, ny, nz = 4, 12, 3
    rng = np.random.default_rng(61)
    prof = lambda n: np.broadcast_to(rng.uniform(1, 5, size=n)[None, :, None], (nz, n, nx)).copy()
    rho = prof(ny)
    vs = prof(ny + 1)
    vs[:, 0, :] = 0.0
    vs[:, ny, :] = 0.0
    S = prof(ny) - 3.0
    pn, pnm1 = prof(ny), prof(ny)
    us = np.zeros((nz, ny, nx))
    ws = np.zeros((nz, ny, nx))
    g = O.Grid(nx, ny, nz, 1.0, 2.0, 1.0)
    out = O.ppe_step(g, -1.0, 1e-2, us, vs, ws, rho, pn, pnm1, S)
    Sc = S[0, :, 0] - S[0, :, 0].mean()
    v = np.concatenate([[0.0], np.cumsum(g.dy * Sc)])
    assert np.allclose(out["v"][0, :, 0], v, rtol=0, atol=1e-13 * np.abs(S).max())
    assert np.abs(out["u"]).max() < 1e-12 and np.abs(out["w"]).max() < 1e-12


# ---------------------------------------------------------------------------
# 8. Manufactured source: choose p, build S so that p solves Eq. (29)
# ---------------------------------------------------------------------------

def test_manufactured_pressure_is_recovered():
    pr = problem((8, 6, 10), 71)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    pe = np.random.default_rng(72).standard_normal(g.shape)
    pe -= pe.mean()
    one = lambda *a: 1.0
    lap_pe = bf_div(g, *bf_face_fluxes(g, pe, one, one, one))
    b_hat_part = bf_rhs(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, np.zeros(g.shape))
    # b = (rho0/dt)(Du* - S) + D(beta G p_hat) = L pe  =>  S = (dt/rho0)(b_hat_part - L pe)
    S = (pr.dt / pr.rho0) * (b_hat_part - lap_pe)
    out = O.ppe_step(g, pr.rho0, pr.dt, pr.us, pr.vs, pr.ws, pr.rho, pr.pn, pr.pnm1, S)
    assert rel(out["p"], pe) < 1e-11


# ---------------------------------------------------------------------------
# 9. Symmetries: linearity, periodic shifts, mirror in y
# ---------------------------------------------------------------------------

def test_linearity_and_shift_and_mirror():
    pr = problem((8, 6, 6), 81)
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    f = lambda us, vs, ws, pn, pnm1, S: O.ppe_step(g, pr.rho0, pr.dt, us, vs, ws, pr.rho, pn, pnm1, S)
    a = f(pr.us, pr.vs, pr.ws, pr.pn, pr.pnm1, pr.S)
    b = f(2 * pr.us, 2 * pr.vs, 2 * pr.ws, 2 * pr.pn, 2 * pr.pnm1, 2 * pr.S)
    assert rel(b["p"], 2 * a["p"]) < 1e-13
    # shift by 3 cells in x and 2 in z: every field moves with the grid
    sh = lambda x: np.roll(np.roll(x, 3, axis=2), 2, axis=0)
    c = O.ppe_step(g, pr.rho0, pr.dt, sh(pr.us), sh(pr.vs), sh(pr.ws), sh(pr.rho), sh(pr.pn), sh(pr.pnm1), sh(pr.S))
    assert rel(c["p"], sh(a["p"])) < 1e-13
    assert rel(c["u"], sh(a["u"])) < 1e-14
    # mirror in y: cell fields flip, v flips and changes sign
    my = lambda x: x[:, ::-1, :].copy()
    d = O.ppe_step(g, pr.rho0, pr.dt, my(pr.us), -my(pr.vs), my(pr.ws), my(pr.rho), my(pr.pn), my(pr.pnm1), my(pr.S))
    assert rel(d["p"], my(a["p"])) < 1e-13
    assert rel(d["v"], -my(a["v"])) < 1e-14


# ---------------------------------------------------------------------------
# 10. Input generators: shapes, walls, sheet density, zero-sum source
# ---------------------------------------------------------------------------

def test_sheet_generator_properties():
    pr = synth.sheet_32()
    assert pr.us.shape == (32, 32, 32) and pr.vs.shape == (32, 33, 32)
    assert np.all(pr.vs[:, 0, :] == 0) and np.all(pr.vs[:, -1, :] == 0)
    assert pr.rho.min() >= 100.0 and pr.rho.max() <= 640.0 and pr.rho0 == 100.0
    assert abs(pr.S.sum()) < 1e-15 * max(1, np.abs(pr.S).sum())
    tg = synth.taylor_green_velocity(np.random.default_rng(0), 16, 8, 12, 2 * np.pi, 2.0, 2 * np.pi, noise=0.0)
    g = O.Grid(16, 8, 12)
    assert np.abs(bf_div(g, *tg)).max() < 1e-12
    again = synth.sheet_32()
    assert np.array_equal(again.pn, pr.pn) and np.array_equal(again.S, pr.S)
