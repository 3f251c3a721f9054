"""Pins for the oracle's predictor u^p, Eq. (23).

Expected values come from outside the oracle's formulas:
  * the SMART characteristic in normalised variables (Gaskell & Lau, cited
    in Sec. 5.4): QUICK in its middle range, bounded, upwind outside [0, 1];
  * exact discrete facts: uniform flow is unchanged; convective and viscous
    fluxes telescope, so x and z momentum are conserved with walls at rest;
    a linear shear has no viscous force away from the walls; a quadratic
    profile's second difference is exact; a dilatation u(x) feels
    (4/3) mu d2u/dx2;
  * symmetry: swapping x and z, and reflecting y between walls, permute the
    result;
  * the balanced CSF force (Sec. 5.4): at constant density and uniform
    sigma*kappa, predictor + projection leave zero velocity and a pressure
    jump of exactly sigma*kappa;
  * a scalar loop implementation of every face on tiny grids.
"""
import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------------------
# SMART in normalised variables
# ---------------------------------------------------------------------------

def test_smart_characteristic():
    U, D = 0.0, 1.0
    for phc in (0.2, 0.5, 0.8):                     # QUICK range
        assert O.smart_face(U, phc, D) == pytest.approx(0.375 * D + 0.75 * phc - 0.125 * U, abs=1e-15)
    assert O.smart_face(U, 0.1, D) == pytest.approx(0.3, abs=1e-15)     # 3 phi_C
    assert O.smart_face(U, 0.9, D) == pytest.approx(1.0, abs=1e-15)     # downwind value
    for phc in (-0.3, 1.4):                          # non-monotone: upwind
        assert O.smart_face(U, phc, D) == phc
    assert O.smart_face(2.0, 2.0, 2.0) == 2.0         # flat
    rng = np.random.default_rng(1)
    a, b, c = rng.standard_normal((3, 10000))
    f = O.smart_face(a, b, c)
    mono = (b - a) * (c - b) > 0
    lo, hi = np.minimum(b, c), np.maximum(b, c)
    assert np.all((f[mono] >= lo[mono] - 1e-15) & (f[mono] <= hi[mono] + 1e-15))
    # invariant under a shift and a scale of the data
    assert np.allclose(O.smart_face(3 * a + 1, 3 * b + 1, 3 * c + 1), 3 * f + 1, atol=1e-12)


def test_interface_faces_follow_the_cell_peclet_number():
    """Sec. 5.4's interface rule in its quotient form: central differences
    where the cell Peclet number Pe = |m| h / mu is below 2, first-order
    upwind otherwise; faces away from the interface take SMART.  Decisions
    within a relative 1e-9 of Pe = 2 are left out (the oracle compares the
    product |m| h against 2 mu, which may round the other way there)."""
    rng = np.random.default_rng(7)
    n = 20000
    m = rng.standard_normal(n) * rng.choice([1.0, 10.0, 100.0], n)
    mu = rng.uniform(0.01, 1.0, n)
    h = rng.uniform(0.01, 0.2, n)
    st = rng.standard_normal((6, n))
    iface = rng.uniform(size=n) < 0.5
    got = O.ppe_oracle._advected(m, *st, iface, mu, h)
    pe = np.abs(m) * h / mu
    keep = np.abs(pe - 2.0) > 1e-9 * 2.0
    up, ce, dn = np.where(m >= 0, st[0], st[3]), np.where(m >= 0, st[1], st[4]), np.where(m >= 0, st[2], st[5])
    want = np.where(pe < 2.0, 0.5 * (ce + dn), ce)
    sel = iface & keep
    assert sel.sum() > 9000 and 0.2 < np.mean(pe[sel] < 2.0) < 0.8
    assert np.array_equal(got[sel], want[sel])
    smart = np.array([_smart1(a, b, c) for a, b, c in zip(up[~iface], ce[~iface], dn[~iface])])
    assert np.allclose(got[~iface], smart, rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def fields(g, seed, interface=True, vwall=0.0):
    rng = np.random.default_rng(seed)
    sh, vs = g.shape, g.vshape
    u = rng.uniform(-1, 1, sh)
    w = rng.uniform(-1, 1, sh)
    v = rng.uniform(-1, 1, vs)
    v[:, 0, :] = vwall
    if g.ybc == 0:
        v[:, -1, :] = vwall
    C = rng.choice([0.0, 1.0], size=sh)
    if interface:
        m = rng.uniform(size=sh) < 0.3
        C[m] = rng.uniform(0.05, 0.95, size=int(m.sum()))
    rho_n = 1.0 + 9.0 * C + 0.1 * rng.uniform(size=sh)
    rho_np1 = rho_n * (1.0 + 0.05 * rng.uniform(-1, 1, sh))
    mu = 0.01 + 0.05 * C + 0.01 * rng.uniform(size=sh)
    ifc = (C > 0) & (C < 1)
    sigma = np.where(ifc, rng.uniform(0.5, 1.5, sh), 0.0)
    kappa = np.where(ifc, rng.uniform(-3, 3, sh), 0.0)
    return dict(u=u, v=v, w=w, rho_n=rho_n, rho_np1=rho_np1, mu=mu, C=C, sigma=sigma, kappa=kappa)


def run(g, f, dt=1e-3, rho_mean=5.0, **kw):
    return O.predictor(g, dt, rho_mean, f["u"], f["v"], f["w"], f["rho_n"], f["rho_np1"], f["mu"], f["C"],
                       f["sigma"], f["kappa"], **kw)


# ---------------------------------------------------------------------------
# exact discrete facts
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ybc", [0, 1])
def test_uniform_flow_is_unchanged(ybc):
    g = O.Grid(8, 6, 4, 1.0, 1.0, 1.0, ybc=ybc)
    sh = g.shape
    u = np.full(sh, 0.7)
    w = np.full(sh, -0.3)
    v = np.zeros(g.vshape)
    rho = np.full(sh, 3.0)
    up, vp, wp = O.predictor(g, 1e-2, 3.0, u, v, w, rho, rho, np.full(sh, 0.1), np.zeros(sh), np.zeros(sh),
                             np.zeros(sh))
    assert np.abs(up - u).max() < 1e-15 and np.abs(wp - w).max() < 1e-15 and np.abs(vp).max() < 1e-15


def test_x_and_z_momentum_conserved_between_walls_at_rest():
    g = O.Grid(8, 6, 6, 1.3, 0.9, 1.1)
    f = fields(g, 2)
    f["sigma"][:] = 0.0
    f["kappa"][:] = 0.0
    up, vp, wp = run(g, f)
    rf = lambda r, ax: 0.5 * (r + np.roll(r, 1, axis=ax))
    for new, old, ax in ((up, f["u"], 2), (wp, f["w"], 0)):
        a = np.sum(rf(f["rho_np1"], ax) * new)
        b = np.sum(rf(f["rho_n"], ax) * old)
        assert abs(a - b) < 1e-13 * np.sum(np.abs(rf(f["rho_n"], ax) * old))


def test_linear_shear_and_quadratic_profile():
    g = O.Grid(6, 8, 4, 1.0, 1.6, 1.0)
    y = (np.arange(g.ny) + 0.5) * g.dy
    sh = g.shape
    zero = np.zeros(sh)
    rho = np.full(sh, 2.0)
    mu = np.full(sh, 0.3)
    dt = 1e-2
    for prof, lap in ((3.0 * y - 1.0, 0.0), (y ** 2, 2.0)):
        u = np.broadcast_to(prof[None, :, None], sh).copy()
        up, vp, wp = O.predictor(g, dt, 2.0, u, np.zeros(g.vshape), zero, rho, rho, mu, zero, zero, zero)
        inner = slice(1, g.ny - 1)
        want = u[:, inner, :] + dt * mu[:, inner, :] * lap / rho[:, inner, :]
        assert np.abs(up[:, inner, :] - want).max() < 1e-12
        assert np.abs(vp).max() < 1e-15 and np.abs(wp).max() < 1e-15


def test_dilatation_feels_four_thirds_mu():
    g = O.Grid(16, 4, 4, 1.0, 1.0, 1.0)
    x = np.arange(g.nx) * g.dx
    sh = g.shape
    base = np.broadcast_to(np.sin(2 * np.pi * x)[None, None, :], sh).copy()
    rho = np.full(sh, 1.5)
    mu = np.full(sh, 0.2)
    zero = np.zeros(sh)
    dt = 1e-3

    def r(eps):
        up, _, _ = O.predictor(g, dt, 1.5, eps * base, np.zeros(g.vshape), zero, rho, rho, mu, zero, zero, zero)
        return (up - eps * base) * rho / dt          # = -eps^2 conv + eps visc
    e1, e2 = 1.0, 2.0
    visc = (e2 ** 2 * r(e1) - e1 ** 2 * r(e2)) / (e1 * e2 ** 2 - e2 * e1 ** 2)
    lap = (np.roll(base, -1, 2) - 2 * base + np.roll(base, 1, 2)) / g.dx ** 2
    assert np.abs(visc - (4.0 / 3.0) * 0.2 * lap).max() < 1e-9 * np.abs(lap).max()


# ---------------------------------------------------------------------------
# symmetries
# ---------------------------------------------------------------------------

def test_swapping_x_and_z():
    g = O.Grid(6, 5, 6, 1.0, 1.0, 1.0)
    f = fields(g, 3)
    up, vp, wp = run(g, f)
    t = lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 2))
    fs = {k: t(a) for k, a in f.items()}
    fs["u"], fs["w"] = t(f["w"]), t(f["u"])
    up2, vp2, wp2 = run(g, fs)
    assert np.abs(up2 - t(wp)).max() < 1e-13
    assert np.abs(wp2 - t(up)).max() < 1e-13
    assert np.abs(vp2 - t(vp)).max() < 1e-13


def test_reflecting_y_between_walls():
    g = O.Grid(6, 7, 4, 1.0, 1.0, 1.0)
    f = fields(g, 4)
    up, vp, wp = run(g, f)
    rc = lambda a: a[:, ::-1, :].copy()
    fr = {k: rc(a) for k, a in f.items() if k != "v"}
    fr["v"] = -f["v"][:, ::-1, :]
    up2, vp2, wp2 = run(g, fr)
    assert np.abs(up2 - rc(up)).max() < 1e-13
    assert np.abs(wp2 - rc(wp)).max() < 1e-13
    assert np.abs(vp2 + vp[:, ::-1, :]).max() < 1e-13


# ---------------------------------------------------------------------------
# balanced surface tension (Sec. 5.4, CSF with density scaling)
# ---------------------------------------------------------------------------

def test_csf_balances_the_projection_pressure_jump():
    g = O.Grid(24, 24, 4, 1.0, 1.0, 1.0)
    x = (np.arange(g.nx) + 0.5) * g.dx
    y = (np.arange(g.ny) + 0.5) * g.dy
    r = np.sqrt((x[None, :] - 0.5) ** 2 + (y[:, None] - 0.5) ** 2)
    C2 = np.clip(0.5 - (r - 0.25) / (3 * g.dx), 0.0, 1.0)     # smooth column, 3-cell band
    C = np.broadcast_to(C2[None], g.shape).copy()
    ifc = (C > 0) & (C < 1)
    sig, kap = 0.07, 4.0
    sigma = np.where(ifc, sig, 0.0)
    kappa = np.where(ifc, kap, 0.0)
    rho = np.full(g.shape, 5.0)
    mu = np.full(g.shape, 0.01)
    zero = np.zeros(g.shape)
    dt = 1e-3
    up, vp, wp = O.predictor(g, dt, 5.0, zero, np.zeros(g.vshape), zero, rho, rho, mu, C, sigma, kappa)
    assert np.abs(up).max() > 0
    out = O.ppe_step(g, 5.0, dt, up, vp, wp, rho, zero, zero, zero)
    assert np.abs(out["u"]).max() < 1e-12 and np.abs(out["v"]).max() < 1e-12
    p = out["p"]
    jump = p[0][C2 == 1.0].mean() - p[0][C2 == 0.0].mean()
    assert abs(jump - sig * kap) < 1e-10


# ---------------------------------------------------------------------------
# scalar loops, every face of tiny grids
# ---------------------------------------------------------------------------

def _smart1(U, Cc, D):
    if D == U:
        return Cc
    ph = (Cc - U) / (D - U)
    if not (0.0 < ph < 1.0):
        return Cc
    if ph < 1.0 / 6.0:
        pf = 3.0 * ph
    elif ph < 5.0 / 6.0:
        pf = 0.75 * ph + 0.375
    else:
        pf = 1.0
    return U + pf * (D - U)


def _adv1(m, up_stencil, dn_stencil, iface, mu_f, h):
    U, Cc, D = up_stencil if m >= 0 else dn_stencil
    if iface:
        return 0.5 * (Cc + D) if abs(m) * h < 2.0 * mu_f else Cc
    return _smart1(U, Cc, D)


def loop_predictor(g, dt, rho_mean, f):
    """Every face written out with explicit indices and ghost rules."""
    nz, ny, nx = g.shape
    dx, dy, dz = g.dx, g.dy, g.dz
    u, v, w = f["u"], f["v"], f["w"]
    R0, R1, MU, C, SG, KP = (f[k] for k in ("rho_n", "rho_np1", "mu", "C", "sigma", "kappa"))
    out_flow = g.ybc == 1

    def jy(j):  # mirrored cell row
        if j < 0:
            return -j - 1
        if j >= ny:
            return 2 * ny - 1 - j
        return j

    cell = lambda a, k, j, i: a[k % nz, jy(j), i % nx]
    U_ = lambda k, j, i: u[k % nz, jy(j), i % nx]
    W_ = lambda k, j, i: w[k % nz, jy(j), i % nx]

    def V_(k, J, i):
        k, i = k % nz, i % nx
        if J < 0:
            return 2 * v[k, 0, i] - v[k, -J, i]
        if J > ny:
            return v[k, ny, i] if out_flow else 2 * v[k, ny, i] - v[k, 2 * ny - J, i]
        return v[k, J, i]

    isif = lambda k, j, i: 0.0 < cell(C, k, j, i) < 1.0

    def div(k, j, i):
        return ((U_(k, j, i + 1) - U_(k, j, i)) / dx + (V_(k, j + 1, i) - V_(k, j, i)) / dy
                + (W_(k + 1, j, i) - W_(k, j, i)) / dz)

    def favg(a, b):
        return b if a == 0.0 else (a if b == 0.0 else 0.5 * (a + b))

    mu4 = lambda cells: 0.25 * sum(cell(MU, *c) for c in cells)
    if4 = lambda cells: any(isif(*c) for c in cells)
    rho_v = lambda k, J, i: 0.5 * (cell(R0, k, J - 1, i) + cell(R0, k, J, i))
    rho_u = lambda k, j, i: 0.5 * (cell(R0, k, j, i - 1) + cell(R0, k, j, i))
    rho_w = lambda k, j, i: 0.5 * (cell(R0, k - 1, j, i) + cell(R0, k, j, i))

    def txy(k, J, i):   # edge: u column i, v face J
        cs = [(k, J - 1, i - 1), (k, J - 1, i), (k, J, i - 1), (k, J, i)]
        return mu4(cs) * ((U_(k, J, i) - U_(k, J - 1, i)) / dy + (V_(k, J, i) - V_(k, J, i - 1)) / dx)

    def txz(k, j, i):   # edge: u column i, w plane k
        cs = [(k - 1, j, i - 1), (k - 1, j, i), (k, j, i - 1), (k, j, i)]
        return mu4(cs) * ((U_(k, j, i) - U_(k - 1, j, i)) / dz + (W_(k, j, i) - W_(k, j, i - 1)) / dx)

    def tyz(k, J, i):   # edge: v face J, w plane k
        cs = [(k - 1, J - 1, i), (k - 1, J, i), (k, J - 1, i), (k, J, i)]
        return mu4(cs) * ((W_(k, J, i) - W_(k, J - 1, i)) / dy + (V_(k, J, i) - V_(k - 1, J, i)) / dz)

    def tdiag(k, j, i, axis):
        d = {0: (U_(k, j, i + 1) - U_(k, j, i)) / dx, 1: (V_(k, j + 1, i) - V_(k, j, i)) / dy,
             2: (W_(k + 1, j, i) - W_(k, j, i)) / dz}[axis]
        return cell(MU, k, j, i) * (2 * d - (2.0 / 3.0) * div(k, j, i))

    up = np.empty_like(u)
    wp = np.empty_like(w)
    vp = v.copy()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                # ---- u face (k, j, i)
                def fx(ic):  # x flux at cell centre ic
                    m = cell(R0, k, j, ic) * 0.5 * (U_(k, j, ic) + U_(k, j, ic + 1))
                    a = _adv1(m, (U_(k, j, ic - 1), U_(k, j, ic), U_(k, j, ic + 1)),
                              (U_(k, j, ic + 2), U_(k, j, ic + 1), U_(k, j, ic)), isif(k, j, ic), cell(MU, k, j, ic), dx)
                    return m * a

                def fy(J):
                    m = 0.5 * (rho_v(k, J, i - 1) * V_(k, J, i - 1) + rho_v(k, J, i) * V_(k, J, i))
                    cs = [(k, J - 1, i - 1), (k, J - 1, i), (k, J, i - 1), (k, J, i)]
                    a = _adv1(m, (U_(k, J - 2, i), U_(k, J - 1, i), U_(k, J, i)),
                              (U_(k, J + 1, i), U_(k, J, i), U_(k, J - 1, i)), if4(cs), mu4(cs), dy)
                    return m * a

                def fz(kk):
                    m = 0.5 * (rho_w(kk, j, i - 1) * W_(kk, j, i - 1) + rho_w(kk, j, i) * W_(kk, j, i))
                    cs = [(kk - 1, j, i - 1), (kk - 1, j, i), (kk, j, i - 1), (kk, j, i)]
                    a = _adv1(m, (U_(kk - 2, j, i), U_(kk - 1, j, i), U_(kk, j, i)),
                              (U_(kk + 1, j, i), U_(kk, j, i), U_(kk - 1, j, i)), if4(cs), mu4(cs), dz)
                    return m * a
                conv = (fx(i) - fx(i - 1)) / dx + (fy(j + 1) - fy(j)) / dy + (fz(k + 1) - fz(k)) / dz
                vis = ((tdiag(k, j, i, 0) - tdiag(k, j, i - 1, 0)) / dx + (txy(k, j + 1, i) - txy(k, j, i)) / dy
                       + (txz(k + 1, j, i) - txz(k, j, i)) / dz)
                st = (favg(cell(SG, k, j, i - 1), cell(SG, k, j, i)) * favg(cell(KP, k, j, i - 1), cell(KP, k, j, i))
                      * (cell(C, k, j, i) - cell(C, k, j, i - 1)) / dx)
                r0 = 0.5 * (cell(R0, k, j, i - 1) + cell(R0, k, j, i))
                r1 = 0.5 * (cell(R1, k, j, i - 1) + cell(R1, k, j, i))
                up[k, j, i] = (r0 * u[k, j, i] + dt * (-conv + vis + r1 / rho_mean * st)) / r1

                # ---- w face (k, j, i)
                def gz(kc):
                    m = cell(R0, kc, j, i) * 0.5 * (W_(kc, j, i) + W_(kc + 1, j, i))
                    a = _adv1(m, (W_(kc - 1, j, i), W_(kc, j, i), W_(kc + 1, j, i)),
                              (W_(kc + 2, j, i), W_(kc + 1, j, i), W_(kc, j, i)), isif(kc, j, i), cell(MU, kc, j, i), dz)
                    return m * a

                def gy(J):
                    m = 0.5 * (rho_v(k - 1, J, i) * V_(k - 1, J, i) + rho_v(k, J, i) * V_(k, J, i))
                    cs = [(k - 1, J - 1, i), (k - 1, J, i), (k, J - 1, i), (k, J, i)]
                    a = _adv1(m, (W_(k, J - 2, i), W_(k, J - 1, i), W_(k, J, i)),
                              (W_(k, J + 1, i), W_(k, J, i), W_(k, J - 1, i)), if4(cs), mu4(cs), dy)
                    return m * a

                def gx(ii):
                    m = 0.5 * (rho_u(k - 1, j, ii) * U_(k - 1, j, ii) + rho_u(k, j, ii) * U_(k, j, ii))
                    cs = [(k - 1, j, ii - 1), (k - 1, j, ii), (k, j, ii - 1), (k, j, ii)]
                    a = _adv1(m, (W_(k, j, ii - 2), W_(k, j, ii - 1), W_(k, j, ii)),
                              (W_(k, j, ii + 1), W_(k, j, ii), W_(k, j, ii - 1)), if4(cs), mu4(cs), dx)
                    return m * a
                conv = (gz(k) - gz(k - 1)) / dz + (gy(j + 1) - gy(j)) / dy + (gx(i + 1) - gx(i)) / dx
                vis = ((tdiag(k, j, i, 2) - tdiag(k - 1, j, i, 2)) / dz + (tyz(k, j + 1, i) - tyz(k, j, i)) / dy
                       + (txz(k, j, i + 1) - txz(k, j, i)) / dx)
                st = (favg(cell(SG, k - 1, j, i), cell(SG, k, j, i)) * favg(cell(KP, k - 1, j, i), cell(KP, k, j, i))
                      * (cell(C, k, j, i) - cell(C, k - 1, j, i)) / dz)
                r0 = 0.5 * (cell(R0, k - 1, j, i) + cell(R0, k, j, i))
                r1 = 0.5 * (cell(R1, k - 1, j, i) + cell(R1, k, j, i))
                wp[k, j, i] = (r0 * w[k, j, i] + dt * (-conv + vis + r1 / rho_mean * st)) / r1

        for J in range(1, ny + 1):
            if J == ny and not out_flow:
                continue
            for i in range(nx):
                def hy(jc):
                    m = cell(R0, k, jc, i) * 0.5 * (V_(k, jc, i) + V_(k, jc + 1, i))
                    a = _adv1(m, (V_(k, jc - 1, i), V_(k, jc, i), V_(k, jc + 1, i)),
                              (V_(k, jc + 2, i), V_(k, jc + 1, i), V_(k, jc, i)), isif(k, jc, i), cell(MU, k, jc, i), dy)
                    return m * a

                def hx(ii):
                    m = 0.5 * (rho_u(k, J - 1, ii) * U_(k, J - 1, ii) + rho_u(k, J, ii) * U_(k, J, ii))
                    cs = [(k, J - 1, ii - 1), (k, J - 1, ii), (k, J, ii - 1), (k, J, ii)]
                    a = _adv1(m, (V_(k, J, ii - 2), V_(k, J, ii - 1), V_(k, J, ii)),
                              (V_(k, J, ii + 1), V_(k, J, ii), V_(k, J, ii - 1)), if4(cs), mu4(cs), dx)
                    return m * a

                def hz(kk):
                    m = 0.5 * (rho_w(kk, J - 1, i) * W_(kk, J - 1, i) + rho_w(kk, J, i) * W_(kk, J, i))
                    cs = [(kk - 1, J - 1, i), (kk - 1, J, i), (kk, J - 1, i), (kk, J, i)]
                    a = _adv1(m, (V_(kk - 2, J, i), V_(kk - 1, J, i), V_(kk, J, i)),
                              (V_(kk + 1, J, i), V_(kk, J, i), V_(kk - 1, J, i)), if4(cs), mu4(cs), dz)
                    return m * a
                conv = (hy(J) - hy(J - 1)) / dy + (hx(i + 1) - hx(i)) / dx + (hz(k + 1) - hz(k)) / dz
                vis = ((tdiag(k, J, i, 1) - tdiag(k, J - 1, i, 1)) / dy + (txy(k, J, i + 1) - txy(k, J, i)) / dx
                       + (tyz(k + 1, J, i) - tyz(k, J, i)) / dz)
                st = (favg(cell(SG, k, J - 1, i), cell(SG, k, J, i)) * favg(cell(KP, k, J - 1, i), cell(KP, k, J, i))
                      * (cell(C, k, J, i) - cell(C, k, J - 1, i)) / dy)
                r0 = 0.5 * (cell(R0, k, J - 1, i) + cell(R0, k, J, i))
                r1 = 0.5 * (cell(R1, k, J - 1, i) + cell(R1, k, J, i))
                vp[k, J, i] = (r0 * v[k, J, i] + dt * (-conv + vis + r1 / rho_mean * st)) / r1
    return up, vp, wp


@pytest.mark.parametrize("ybc", [0, 1])
@pytest.mark.parametrize("shape", [(4, 5, 3), (6, 4, 4), (3, 6, 5)])
def test_scalar_loops_every_face(shape, ybc):
    g = O.Grid(*shape, 1.1, 0.8, 1.3, ybc=ybc)
    f = fields(g, 10 + sum(shape) + ybc, vwall=0.0)
    if ybc == 1:
        f["v"][:, -1, :] = np.random.default_rng(5).uniform(-1, 1, (g.nz, g.nx))
    want = loop_predictor(g, 2e-3, 4.0, f)
    got = run(g, f, dt=2e-3, rho_mean=4.0)
    for a, b in zip(got, want):
        assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(b).max())
