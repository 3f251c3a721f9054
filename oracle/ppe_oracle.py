"""CPU FP64 oracle for the split pressure-gradient projection step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library.

Source: Poblador-Ibanez & Sirignano, "A Volume-of-Fluid method for
variable-density, two-phase flows at supercritical pressure" (arXiv 2103.01874),
Section 5.4 (equation numbers count the paper's numbered displays, a
subequations group counting once):

  * Eq. (27): split of the pressure gradient,
        (1/rho) grad p^{n+1}  ->  (1/rho0) grad p^{n+1} + (1/rho - 1/rho0) grad p_hat,
    with p_hat = 2 p^n - p^{n-1} and rho0 = min(rho).
  * Eq. (28): projection  u^{n+1} = u^p - dt [ grad p/rho0 + (1/rho - 1/rho0) grad p_hat ].
  * Eq. (29): constant-coefficient PPE
        lap p = div[(1 - rho0/rho) grad p_hat] + (rho0/dt)(div u^p - div u^{n+1}).
  * Eq. (25): the variable-coefficient PPE the split replaces (used only by
    ``solve_variable_coefficient_dense`` to pin the split's exactness claim).

Discretisation (Sec. 5 opening: uniform staggered Cartesian mesh, velocities on
face centres, scalars at cell centres; Sec. 5.4: standard finite volumes; the
FFT solver handles periodic or homogeneous-Neumann boundaries):

  Array layout is C order [nz][ny][nx] (x fastest).  x and z are periodic,
  y is bounded by two walls.
    u[k][j][i]  : west face of cell i    (nx faces per row, periodic)
    v[k][j][i]  : south face of cell j   (ny+1 faces; j = 0 and j = ny are walls)
    w[k][j][i]  : back face of cell k    (nz faces, periodic)
  D  = cell divergence of face fluxes, G = face gradient of a cell field
  (zero on wall faces), L = D o G (7-point Laplacian, zero wall flux).

Two y-boundary treatments (Grid.ybc):
  ybc = 0  walls at both ends: zero pressure flux, v on both walls given.
  ybc = 1  symmetry plane at the bottom (zero flux, v given) and an outflow
           top boundary where p = 0 on the face (the paper's planar jets,
           Sec. 6: symmetric jets with outflow at the top).  The top-face
           gradient uses the antisymmetric ghost value, G p = -2 p_{ny-1}/dy,
           the top-face density is that of the last cell, and the top v face is
           corrected like any interior face.  L is then nonsingular: no
           compatibility projection and no gauge.

Readings of points the paper leaves open (each is listed in the design notes):
  * face density rho_f = arithmetic mean of the two adjacent cells, used in both
    the right-hand side and the projection (the same rho_f in both makes the
    projected field's divergence exact);
  * the singular Neumann/periodic problem is made compatible by removing
    mean(b), and p is fixed by mean(p) = 0;
  * rho0 <= 0 requests rho0 = min(rho).

Functions follow the paper's order: the target divergence S (Eq. 26), the
right-hand side (Eq. 29), the Poisson solve, the projection (Eq. 28).  The
spectral solver diagonalises L completely (real FFT in x, complex FFT in z,
DCT-II or DCT-IV in y); the dense solver
factorises the bordered matrix with LAPACK.  Neither is the GPU's algorithm.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

__all__ = [
    "Grid",
    "p_hat",
    "rho0_of",
    "face_density",
    "divergence",
    "gradient",
    "laplacian",
    "assemble_rhs",
    "solve_spectral",
    "solve_dense",
    "laplacian_matrix",
    "correct",
    "divergence_check",
    "solve",
    "ppe_step",
    "solve_variable_coefficient_dense",
    "eigenvalues",
    "source_term",
    "variable_coefficient_operator",
    "energy_norm",
    "split_map",
    "split_fixed_point",
    "smart_face",
    "predictor",
]


class Grid:
    """Uniform staggered grid of nx*ny*nz cells, lengths lx, ly, lz; ybc picks the y boundaries."""

    def __init__(self, nx, ny, nz, lx=2 * np.pi, ly=2.0, lz=2 * np.pi, ybc=0):
        if min(nx, ny, nz) < 1:
            raise ValueError("grid sizes must be positive")
        if ybc not in (0, 1):
            raise ValueError("ybc is 0 (walls) or 1 (symmetry bottom, outflow top)")
        self.ybc = int(ybc)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        self.dx = self.lx / self.nx
        self.dy = self.ly / self.ny
        self.dz = self.lz / self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def vshape(self):
        return (self.nz, self.ny + 1, self.nx)

    @property
    def npts(self):
        return self.nx * self.ny * self.nz


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (27): explicit pressure and reference density
# ---------------------------------------------------------------------------

def p_hat(pn, pnm1):
    """Linear extrapolation in time p_hat = 2 p^n - p^{n-1} (Eq. 27)."""
    return 2.0 * np.asarray(pn, dtype=np.float64) - np.asarray(pnm1, dtype=np.float64)


def rho0_of(rho, rho0):
    """rho0 = min(rho) when the caller passes rho0 <= 0 (Eq. 27), else rho0."""
    return float(np.min(rho)) if rho0 <= 0 else float(rho0)


# ---------------------------------------------------------------------------
# Staggered finite-volume operators (Sec. 5 opening, Sec. 5.4)
# ---------------------------------------------------------------------------

def face_density(rho):
    """Density on the three face families: arithmetic mean of the two cells.

    Returns (rx, ry, rz) shaped like (u, v, w).  The wall entries of ry (j = 0
    and j = ny) carry the adjacent cell's density; they multiply a zero
    gradient and never enter a result.
    """
    rho = np.asarray(rho, dtype=np.float64)
    rx = 0.5 * (rho + np.roll(rho, 1, axis=2))
    rz = 0.5 * (rho + np.roll(rho, 1, axis=0))
    nz, ny, nx = rho.shape
    ry = np.empty((nz, ny + 1, nx))
    ry[:, 1:ny, :] = 0.5 * (rho[:, 1:, :] + rho[:, :-1, :])
    ry[:, 0, :] = rho[:, 0, :]
    ry[:, ny, :] = rho[:, ny - 1, :]
    return rx, ry, rz


def divergence(g: Grid, u, v, w):
    """Cell divergence D of face fluxes (u, v, w)."""
    du = (np.roll(u, -1, axis=2) - u) / g.dx
    dv = (v[:, 1:, :] - v[:, :-1, :]) / g.dy
    dw = (np.roll(w, -1, axis=0) - w) / g.dz
    return du + dv + dw


def gradient(g: Grid, p):
    """Face gradient G of a cell field; zero on wall faces of y, and
    -2 p_{ny-1}/dy on an outflow top face (p = 0 there)."""
    p = np.asarray(p, dtype=np.float64)
    gx = (p - np.roll(p, 1, axis=2)) / g.dx
    gz = (p - np.roll(p, 1, axis=0)) / g.dz
    nz, ny, nx = p.shape
    gy = np.zeros((nz, ny + 1, nx))
    gy[:, 1:ny, :] = (p[:, 1:, :] - p[:, :-1, :]) / g.dy
    if g.ybc == 1:
        gy[:, ny, :] = -2.0 * p[:, ny - 1, :] / g.dy
    return gx, gy, gz


def laplacian(g: Grid, p):
    """L p = D(G p): the 7-point Laplacian with zero flux through the walls."""
    return divergence(g, *gradient(g, p))


def eigenvalues(g: Grid):
    """Closed-form eigenvalues of L on its eigenvectors (modified wavenumbers).

    lam_x(a) = -(4/dx^2) sin^2(pi a / nx)       periodic, a = 0..nx//2
    lam_y(m) = -(4/dy^2) sin^2(pi m / (2 ny))   ybc 0: Neumann both ends, cos(pi m (j+1/2)/ny)
    lam_y(m) = -(4/dy^2) sin^2(pi (2m+1)/(4 ny)) ybc 1: Neumann bottom, p = 0 on the top face,
                                                  cos(pi (m+1/2)(j+1/2)/ny)
    lam_z(c) = -(4/dz^2) sin^2(pi c / nz)       periodic, c = 0..nz-1
    Returned broadcastable as [nz][ny][nx//2+1].
    """
    a = np.arange(g.nx // 2 + 1)
    m = np.arange(g.ny)
    c = np.arange(g.nz)
    lx = -(4.0 / g.dx**2) * np.sin(np.pi * a / g.nx) ** 2
    if g.ybc == 0:
        ly = -(4.0 / g.dy**2) * np.sin(np.pi * m / (2.0 * g.ny)) ** 2
    else:
        ly = -(4.0 / g.dy**2) * np.sin(np.pi * (2 * m + 1) / (4.0 * g.ny)) ** 2
    lz = -(4.0 / g.dz**2) * np.sin(np.pi * c / g.nz) ** 2
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (26): the target divergence S = div u^{n+1}
# ---------------------------------------------------------------------------

def source_term(C, div_g, div_l, mdot_area, area_density, rho_g, rho_l, under=None):
    """S of Eq. (26), cell by cell.

    With the phase-wise velocity divergences div_g = -(1/rho_g) D rho_g/Dt and
    div_l = -(1/rho_l) D rho_l/Dt (the extrapolated compressibilities of
    Sec. 4), Eq. (26) reads
        S = (1 - C) div_g + C div_l + mdot (1/rho_g - 1/rho_l).
    mdot = mdot' delta_Gamma (Sec. 3): mass flux per unit area times the
    interface area density A_Gamma / V0, non-zero only in interface cells
    0 < C < 1, where rho_g, rho_l are the interface densities (Sec. 5.4).
    Each phase's compressibility is extrapolated only into a thin band across
    the interface (Sec. 4), and away from it Eq. (26) reduces to the
    compressibility of the phase present (the remark after Eq. 26): a gas
    cell (C <= 0) takes div_g, a liquid cell (C >= 1) div_l, and neither
    reads the other phase's value; the phase-change arrays are read in
    interface cells only.  Under-resolved interface cells (the appendix on
    under-resolved regions) get S = 0; the mask has no effect on single-phase
    cells.
    """
    C = np.asarray(C, dtype=np.float64)
    div_g = np.asarray(div_g, dtype=np.float64)
    div_l = np.asarray(div_l, dtype=np.float64)
    gas = C <= 0.0
    liq = C >= 1.0
    iface = ~gas & ~liq
    S = np.zeros(C.shape)
    S[gas] = div_g[gas]
    S[liq] = div_l[liq]
    c = C[iface]
    mdot = np.asarray(mdot_area, dtype=np.float64)[iface] * np.asarray(area_density, dtype=np.float64)[iface]
    S[iface] = ((1.0 - c) * div_g[iface] + c * div_l[iface]
                + mdot * (1.0 / np.asarray(rho_g, dtype=np.float64)[iface]
                          - 1.0 / np.asarray(rho_l, dtype=np.float64)[iface]))
    if under is not None:
        S[iface & (np.asarray(under) != 0)] = 0.0
    return S


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (29): right-hand side of the constant-coefficient PPE
# ---------------------------------------------------------------------------

def assemble_rhs(g: Grid, rho0, dt, us, vs, ws, rho, pn, pnm1, S):
    """b = (rho0/dt)(D u* - S) + D(beta_f G p_hat),  beta_f = 1 - rho0/rho_f."""
    ph = p_hat(pn, pnm1)
    rx, ry, rz = face_density(rho)
    gx, gy, gz = gradient(g, ph)
    fx = (1.0 - rho0 / rx) * gx
    fy = (1.0 - rho0 / ry) * gy
    fz = (1.0 - rho0 / rz) * gz
    return (rho0 / dt) * (divergence(g, us, vs, ws) - S) + divergence(g, fx, fy, fz)


# ---------------------------------------------------------------------------
# Poisson solve: L p = b - mean(b), mean(p) = 0
# ---------------------------------------------------------------------------

def solve_spectral(g: Grid, b, workers=None):
    """Full diagonalisation of L: rfft in x, fft in z, DCT-II (walls) or
    DCT-IV (outflow top) in y.

    Walls: the (0,0,0) coefficient carries mean(b); setting it to zero both
    removes the incompatible part of b and imposes mean(p) = 0.  Outflow: L is
    nonsingular and every coefficient is divided.
    """
    b = np.asarray(b, dtype=np.float64)
    ytype = 2 if g.ybc == 0 else 4
    bh = sfft.rfft(b, axis=2, workers=workers)
    bh = sfft.fft(bh, axis=0, workers=workers)
    bh = sfft.dct(bh, type=ytype, axis=1, workers=workers)
    lam = eigenvalues(g)
    if g.ybc == 0:
        lam[0, 0, 0] = 1.0
    ph = bh / lam
    if g.ybc == 0:
        ph[0, 0, 0] = 0.0
    ph = sfft.idct(ph, type=ytype, axis=1, workers=workers)
    ph = sfft.ifft(ph, axis=0, workers=workers)
    return sfft.irfft(ph, n=g.nx, axis=2, workers=workers)


def laplacian_matrix(g: Grid):
    """Dense N x N matrix of L, built by applying L to unit vectors."""
    n = g.npts
    A = np.empty((n, n))
    e = np.zeros(n)
    for col in range(n):
        e[col] = 1.0
        A[:, col] = laplacian(g, e.reshape(g.shape)).ravel()
        e[col] = 0.0
    return A


def solve_dense(g: Grid, b):
    """Bordered dense solve [[L, 1], [1^T, 0]] [p; mu] = [b; 0] (tiny grids).

    Row sums of L vanish, so mu = mean(b) and L p = b - mean(b), sum(p) = 0.
    With an outflow top L is nonsingular and is solved directly.
    """
    n = g.npts
    if n > 4096:
        raise ValueError("dense oracle is for tiny grids only")
    if g.ybc == 1:
        return np.linalg.solve(laplacian_matrix(g), np.asarray(b, dtype=np.float64).ravel()).reshape(g.shape)
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = laplacian_matrix(g)
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[:n] = np.asarray(b, dtype=np.float64).ravel()
    sol = np.linalg.solve(M, rhs)
    return sol[:n].reshape(g.shape)


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (28): projection, and the continuity check it must satisfy
# ---------------------------------------------------------------------------

def correct(g: Grid, rho0, dt, us, vs, ws, rho, pn, pnm1, p):
    """u^{n+1} = u* - dt [ G p / rho0 + gamma_f G p_hat ],  gamma_f = 1/rho_f - 1/rho0.

    Wall faces of v are not corrected: they keep v*.  An outflow top face is
    corrected like an interior face.
    """
    ph = p_hat(pn, pnm1)
    rx, ry, rz = face_density(rho)
    px, py, pz = gradient(g, p)
    hx, hy, hz = gradient(g, ph)
    u = us - dt * (px / rho0 + (1.0 / rx - 1.0 / rho0) * hx)
    w = ws - dt * (pz / rho0 + (1.0 / rz - 1.0 / rho0) * hz)
    v = np.array(vs, dtype=np.float64, copy=True)
    v[:, 1:-1, :] = vs[:, 1:-1, :] - dt * (
        py[:, 1:-1, :] / rho0 + (1.0 / ry[:, 1:-1, :] - 1.0 / rho0) * hy[:, 1:-1, :]
    )
    if g.ybc == 1:
        v[:, -1, :] = vs[:, -1, :] - dt * (py[:, -1, :] / rho0 + (1.0 / ry[:, -1, :] - 1.0 / rho0) * hy[:, -1, :])
    return u, v, w


def divergence_check(g: Grid, us, vs, ws, S, u, v, w):
    """Continuity residual of the projected field (Eq. 25's constraint).

    S_c = S + mean(D u* - S) is the compatible target divergence.  Returns
    dict(div_l2, div_max, div0_l2, rel, compat) with
    rel = ||D u - S_c||_2 / ||D u* - S_c||_2.
    """
    d0 = divergence(g, us, vs, ws) - S
    compat = float(np.mean(d0)) if g.ybc == 0 else 0.0
    d0c = d0 - compat
    d = divergence(g, u, v, w) - S - compat
    l2 = float(np.sqrt(np.sum(d * d)))
    l20 = float(np.sqrt(np.sum(d0c * d0c)))
    return {
        "div_l2": l2,
        "div_max": float(np.max(np.abs(d))),
        "div0_l2": l20,
        "rel": l2 / l20 if l20 > 0 else l2,
        "compat": compat,
    }


def solve(g: Grid, rho0, dt, us, vs, ws, rho, pn, pnm1, S, method="spectral", workers=None):
    """Pressure of the split projection: zero-mean p with L p = b - mean(b)
    (walls), or p with L p = b (outflow top)."""
    r0 = rho0_of(rho, rho0)
    b = assemble_rhs(g, r0, dt, us, vs, ws, rho, pn, pnm1, S)
    if method == "spectral":
        p = solve_spectral(g, b, workers=workers)
    elif method == "dense":
        p = solve_dense(g, b)
    else:
        raise ValueError(method)
    return p, r0, b


def ppe_step(g: Grid, rho0, dt, us, vs, ws, rho, pn, pnm1, S, method="spectral", workers=None):
    """Whole projection step: assemble, solve, project, check continuity."""
    p, r0, b = solve(g, rho0, dt, us, vs, ws, rho, pn, pnm1, S, method=method, workers=workers)
    u, v, w = correct(g, r0, dt, us, vs, ws, rho, pn, pnm1, p)
    chk = divergence_check(g, us, vs, ws, S, u, v, w)
    return {"p": p, "u": u, "v": v, "w": w, "rho0": r0, "b": b,
            "compat_defect": (float(np.mean(b)) * dt / r0) if g.ybc == 0 else 0.0, **chk}


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (25): the variable-coefficient problem the split approximates
# ---------------------------------------------------------------------------

def solve_variable_coefficient_dense(g: Grid, dt, us, vs, ws, rho, S):
    """Zero-mean q with D((1/rho_f) G q) = (1/dt)(D u* - S_c) (tiny grids).

    Sec. 5.4 states the split is exact when grad p_hat equals grad p^{n+1};
    feeding q back as p^n = p^{n-1} = q must therefore return p = q.
    """
    n = g.npts
    if n > 4096:
        raise ValueError("dense oracle is for tiny grids only")
    rx, ry, rz = face_density(rho)
    A = np.empty((n, n))
    e = np.zeros(n)
    for col in range(n):
        e[col] = 1.0
        gx, gy, gz = gradient(g, e.reshape(g.shape))
        A[:, col] = divergence(g, gx / rx, gy / ry, gz / rz).ravel()
        e[col] = 0.0
    d0 = divergence(g, us, vs, ws) - S
    if g.ybc == 1:
        return np.linalg.solve(A, (d0 / dt).ravel()).reshape(g.shape)
    rhs_c = (d0 - np.mean(d0)) / dt
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[:n] = rhs_c.ravel()
    return np.linalg.solve(M, rhs)[:n].reshape(g.shape)


# ---------------------------------------------------------------------------
# Sec. 5.4: the split as a map p_hat -> p, its fixed point (the pressure of
# Eq. 25) and how far one split solve is from it
# ---------------------------------------------------------------------------

def variable_coefficient_operator(g: Grid, rho, p):
    """A p = D((1/rho_f) G p): the operator of Eq. (25)."""
    rx, ry, rz = face_density(rho)
    gx, gy, gz = gradient(g, p)
    return divergence(g, gx / rx, gy / ry, gz / rz)


def energy_norm(g: Grid, e):
    """||e||_E = sqrt(-e . L e), the norm in which the split map contracts."""
    e = np.asarray(e, dtype=np.float64)
    return float(np.sqrt(max(-np.sum(e * laplacian(g, e)), 0.0)))


def split_map(g: Grid, rho0, dt, us, vs, ws, rho, S, ph, workers=None):
    """F(p_hat): the split solve (Eqs. 27-29) with p^n = p^{n-1} = p_hat."""
    p, _, _ = solve(g, rho0, dt, us, vs, ws, rho, ph, ph, S, workers=workers)
    return p


def split_fixed_point(g: Grid, rho0, dt, us, vs, ws, rho, pn, pnm1, S, iters, tol=0.0, workers=None):
    """Iterate p_{k+1} = F(p_k) from p_0 = 2 p^n - p^{n-1}.

    Sec. 5.4 states the split is exact when grad p_hat equals grad p^{n+1}: a
    fixed point of F is the pressure of Eq. (25) (zero mean with zero-flux y
    ends).  p_1 is the ordinary split solve.  For each iterate the relative
    residual of Eq. (25),
        res_k = ||rho0 [(1/dt)(D u* - S_c) - A p_k]||_2 / ||(rho0/dt)(D u* - S_c)||_2,
    is recorded (res_0 belongs to p_0 = p_hat); iteration stops once
    res_k <= tol or after `iters` maps.  Returns dict(p, iters, res, upd_E)
    with upd_E[k] = ||p_{k+1} - p_k||_E.
    """
    r0 = rho0_of(rho, rho0)
    d0 = divergence(g, us, vs, ws) - S
    if g.ybc == 0:
        d0 = d0 - np.mean(d0)
    ref = float(np.linalg.norm((r0 / dt) * d0))
    p = p_hat(pn, pnm1)
    res, upd = [], []

    def residual(q):
        r = r0 * (d0 / dt - variable_coefficient_operator(g, rho, q))
        if g.ybc == 0:
            r = r - np.mean(r)
        return float(np.linalg.norm(r)) / ref if ref > 0 else float(np.linalg.norm(r))

    res.append(residual(p))
    k = 0
    while k < iters and res[-1] > tol:
        q = split_map(g, r0, dt, us, vs, ws, rho, S, p, workers=workers)
        upd.append(energy_norm(g, q - p))
        p = q
        k += 1
        res.append(residual(p))
    return {"p": p, "iters": k, "res": res, "upd_E": upd, "rho0": r0}


# ---------------------------------------------------------------------------
# Sec. 5.4, Eq. (23): the predictor u^p (input of the projection)
# ---------------------------------------------------------------------------
#
# Finite volumes on the staggered mesh (Sec. 5.4: SMART convection, second-
# order central viscous term, CSF surface tension with density scaling):
#   u^p = [ rho^n_f u^n + dt ( -div(rho u u)^n + div(tau)^n
#                              + (rho^{n+1}_f/<rho>)(sigma_f kappa_f grad C + f_s) ) ] / rho^{n+1}_f
# Readings (each listed in the design notes):
#   * rho_f on a face: mean of its two cells (as in the projection); the mass
#     flux through a momentum control-volume face is the mean of the two
#     neighbouring face mass fluxes (rho_f times face velocity), or at a cell
#     centre the cell density times the mean of the two face velocities;
#   * the advected velocity on a control-volume face: SMART in normalised
#     variables; where any cell touching that face is an interface cell
#     (0 < C < 1), central differences if the cell Peclet number
#     |m| h / mu < 2, else first-order upwind;
#   * tau = mu [grad u + grad u^T - (2/3)(div u) I] (Sec. 2) with the velocity
#     of the viscous term given separately (the paper's phase-wise velocities;
#     defaults to u^n); mu at a cell centre, or the mean of the four cells
#     around an edge;
#   * sigma and kappa on a face by Eq. (30); grad C the face difference;
#     f_s the tangential (Marangoni) force on faces, given;
#   * y ends: ghost cells mirror the first two cells (cell fields and the
#     tangential velocities u, w); v beyond a wall or symmetry face is the
#     odd reflection 2 v_b - v, beyond an outflow face it equals v_ny; a
#     ghost cell's stress comes from these ghost velocities; wall faces of v
#     keep v^n, an outflow face is predicted.


def smart_face(U, Cc, D):
    """SMART value on a face from far-upwind U, upwind Cc and downwind D
    (bounded QUICK in the normalised variable phi_C = (Cc - U)/(D - U)):
        0 < phi_C < 1/6    face = U + 3 (Cc - U)
        1/6 <= phi_C < 5/6 face = U + (3/4)(Cc - U) + (3/8)(D - U)
        5/6 <= phi_C < 1   face = D
        otherwise          face = Cc (upwind)
    The ranges are tested as products (a = Cc - U, d = D - U of equal sign,
    6|a| against |d|), without forming the quotient."""
    U, Cc, D = np.broadcast_arrays(np.asarray(U, float), np.asarray(Cc, float), np.asarray(D, float))
    a = Cc - U
    d = D - U
    inside = (a * d > 0) & (np.abs(a) < np.abs(d))
    low = 6.0 * np.abs(a) < np.abs(d)
    mid = 6.0 * np.abs(a) < 5.0 * np.abs(d)
    val = np.where(low, U + 3.0 * a, np.where(mid, U + 0.75 * a + 0.375 * d, D))
    return np.where(inside, val, Cc)


def _advected(m, Um, Cm, Dm, Up, Cp, Dp, iface, mu_face, h):
    """Face value for mass flux m: the m >= 0 stencil is (Um, Cm, Dm), the
    m < 0 one (Up, Cp, Dp); the interface rule uses the cell Peclet number."""
    pos = m >= 0
    U = np.where(pos, Um, Up)
    Cc = np.where(pos, Cm, Cp)
    D = np.where(pos, Dm, Dp)
    s = smart_face(U, Cc, D)
    # cell Peclet number |m| h / mu below 2, tested without the quotient
    hyb = np.where(np.abs(m) * h < 2.0 * mu_face, 0.5 * (Cc + D), Cc)
    return np.where(iface, hyb, s)


def _yext(a, lo, hi):
    """Two ghost layers on each side of axis 1 from callables lo(a), hi(a)."""
    return np.concatenate([lo(a), a, hi(a)], axis=1)


def _mirror(a):
    return _yext(a, lambda x: x[:, 1::-1, :], lambda x: x[:, :-3:-1, :])


def _faceavg(a, b):
    """Eq. (30): one side's value where the other is zero, else the mean."""
    return np.where(a == 0.0, b, np.where(b == 0.0, a, 0.5 * (a + b)))


def predictor(g: Grid, dt, rho_mean, u, v, w, rho_n, rho_np1, mu, C, sigma, kappa,
              uv=None, vv=None, wv=None, fsx=None, fsy=None, fsz=None):
    """u^p, v^p, w^p of Eq. (23).  Needs ny >= 4."""
    if g.ny < 4:
        raise ValueError("the predictor needs ny >= 4")
    f = lambda a: np.asarray(a, dtype=np.float64)
    u, v, w, rho_n, rho_np1, mu, C, sigma, kappa = map(f, (u, v, w, rho_n, rho_np1, mu, C, sigma, kappa))
    uv = u if uv is None else f(uv)
    vv = v if vv is None else f(vv)
    wv = w if wv is None else f(wv)
    nz, ny, nx = g.shape
    dx, dy, dz = g.dx, g.dy, g.dz
    X, Z = 2, 0
    sh = lambda a, s, ax: np.roll(a, s, axis=ax)   # sh(a, 1, X)[i] = a[i-1]

    # y-extended arrays: index J + 2 holds row J
    R = _mirror(rho_n)
    Rn1 = _mirror(rho_np1)
    M = _mirror(mu)
    Ce = _mirror(C)
    Ue, Uve = _mirror(u), _mirror(uv)
    We, Wve = _mirror(w), _mirror(wv)

    def vext(a):
        lo = lambda x: 2.0 * x[:, :1, :] - x[:, 2:0:-1, :]
        if g.ybc == 1:
            hi = lambda x: np.repeat(x[:, -1:, :], 2, axis=1)
        else:
            hi = lambda x: 2.0 * x[:, -1:, :] - x[:, -2:-4:-1, :]
        return _yext(a, lo, hi)
    Ve, Vve = vext(v), vext(vv)        # face J at index J + 2, J = -2 .. ny + 2
    # cell divergence of the viscous-term velocity on real and ghost rows,
    # from the (ghost-extended) velocities: row J at index J + 2
    Dv = ((sh(Uve, -1, X) - Uve) / dx + (Vve[:, 1:, :] - Vve[:, :-1, :])[:, :ny + 4, :] / dy
          + (sh(Wve, -1, Z) - Wve) / dz)
    iface = (Ce > 0.0) & (Ce < 1.0)
    rows = slice(2, 2 + ny)            # the real cell rows in extended arrays


    # face densities on u, w faces (real rows) and v faces (extended)
    rxn, rxn1 = 0.5 * (R + sh(R, 1, X)), 0.5 * (Rn1 + sh(Rn1, 1, X))
    rzn, rzn1 = 0.5 * (R + sh(R, 1, Z)), 0.5 * (Rn1 + sh(Rn1, 1, Z))
    ryn = 0.5 * (R[:, 1:, :] + R[:, :-1, :])      # face J at index J + 1 (J = -1 .. ny + 2)
    ryn1 = 0.5 * (Rn1[:, 1:, :] + Rn1[:, :-1, :])

    def vface(a, J0, J1):
        """Extended v-face array rows J0..J1-1 (J real face index)."""
        return a[:, J0 + 2:J1 + 2, :]

    def yface_rho(J0, J1, n1=False):
        a = ryn1 if n1 else ryn
        return a[:, J0 + 1:J1 + 1, :]

    # ---------------- x momentum on u faces --------------------------------
    # x: control-volume faces at cell centres i (between u_i and u_{i+1})
    m = R * 0.5 * (Ue + sh(Ue, -1, X))
    ut = _advected(m, sh(Ue, 1, X), Ue, sh(Ue, -1, X), sh(Ue, -2, X), sh(Ue, -1, X), Ue, iface, M, dx)
    Fx = m * ut
    conv = (Fx - sh(Fx, 1, X))[:, rows, :] / dx
    # y: edges at v-face rows J = 0..ny, between u rows J-1 and J
    J = np.arange(ny + 1)
    rv = yface_rho(0, ny + 1) * vface(Ve, 0, ny + 1)      # (rho v) on v faces, column i
    mE = 0.5 * (rv + sh(rv, 1, X))                          # columns i-1 and i
    u_m2, u_m1, u_0, u_p1 = (Ue[:, J + 2 + o, :] for o in (-2, -1, 0, 1))
    ie = iface[:, J + 1, :] | iface[:, J + 2, :]
    ie = ie | sh(ie, 1, X)
    me = 0.25 * (M[:, J + 1, :] + M[:, J + 2, :])
    me = me + sh(me, 1, X)
    ut = _advected(mE, u_m2, u_m1, u_0, u_p1, u_0, u_m1, ie, me, dy)
    Fy = mE * ut
    conv = conv + (Fy[:, 1:, :] - Fy[:, :-1, :]) / dy
    # z: edges at back faces k, between u planes k-1 and k
    rw = rzn * We                                            # (rho w) on w faces, extended rows
    mZ = 0.5 * (rw + sh(rw, 1, X))
    iz = iface | sh(iface, 1, Z)
    iz = iz | sh(iz, 1, X)
    mz_mu = 0.25 * (M + sh(M, 1, Z))
    mz_mu = mz_mu + sh(mz_mu, 1, X)
    ut = _advected(mZ, sh(Ue, 2, Z), sh(Ue, 1, Z), Ue, sh(Ue, -1, Z), Ue, sh(Ue, 1, Z), iz, mz_mu, dz)
    Fz = mZ * ut
    conv = conv + (sh(Fz, -1, Z) - Fz)[:, rows, :] / dz
    # viscous
    txx = M * (2.0 * (sh(Uve, -1, X) - Uve) / dx - (2.0 / 3.0) * Dv)
    vis = (txx - sh(txx, 1, X))[:, rows, :] / dx
    txy = me * ((Uve[:, J + 2, :] - Uve[:, J + 1, :]) / dy
                + (vface(Vve, 0, ny + 1) - sh(vface(Vve, 0, ny + 1), 1, X)) / dx)
    vis = vis + (txy[:, 1:, :] - txy[:, :-1, :]) / dy
    txz = mz_mu * ((Uve - sh(Uve, 1, Z)) / dz + (Wve - sh(Wve, 1, X)) / dx)
    vis = vis + (sh(txz, -1, Z) - txz)[:, rows, :] / dz
    # surface tension
    stx = (_faceavg(sh(sigma, 1, X), sigma) * _faceavg(sh(kappa, 1, X), kappa) * (C - sh(C, 1, X)) / dx)
    if fsx is not None:
        stx = stx + f(fsx)
    r0, r1 = rxn[:, rows, :], rxn1[:, rows, :]
    up = (r0 * u + dt * (-conv + vis + (r1 / rho_mean) * stx)) / r1

    # ---------------- z momentum on w faces (x <-> z of the above) ---------
    m = R * 0.5 * (We + sh(We, -1, Z))
    wt = _advected(m, sh(We, 1, Z), We, sh(We, -1, Z), sh(We, -2, Z), sh(We, -1, Z), We, iface, M, dz)
    Fzz = m * wt
    conv = (Fzz - sh(Fzz, 1, Z))[:, rows, :] / dz
    rvz = 0.5 * (rv + sh(rv, 1, Z))
    w_m2, w_m1, w_0, w_p1 = (We[:, J + 2 + o, :] for o in (-2, -1, 0, 1))
    iez = iface[:, J + 1, :] | iface[:, J + 2, :]
    iez = iez | sh(iez, 1, Z)
    mez = 0.25 * (M[:, J + 1, :] + M[:, J + 2, :])
    mez = mez + sh(mez, 1, Z)
    wt = _advected(rvz, w_m2, w_m1, w_0, w_p1, w_0, w_m1, iez, mez, dy)
    Fy = rvz * wt
    conv = conv + (Fy[:, 1:, :] - Fy[:, :-1, :]) / dy
    ru = rxn * Ue                                            # (rho u) on u faces
    mX = 0.5 * (ru + sh(ru, 1, Z))
    wt = _advected(mX, sh(We, 2, X), sh(We, 1, X), We, sh(We, -1, X), We, sh(We, 1, X), iz, mz_mu, dx)
    Fx = mX * wt
    conv = conv + (sh(Fx, -1, X) - Fx)[:, rows, :] / dx
    tzz = M * (2.0 * (sh(Wve, -1, Z) - Wve) / dz - (2.0 / 3.0) * Dv)
    vis = (tzz - sh(tzz, 1, Z))[:, rows, :] / dz
    tyz = mez * ((Wve[:, J + 2, :] - Wve[:, J + 1, :]) / dy
                 + (vface(Vve, 0, ny + 1) - sh(vface(Vve, 0, ny + 1), 1, Z)) / dz)
    vis = vis + (tyz[:, 1:, :] - tyz[:, :-1, :]) / dy
    vis = vis + (sh(txz, -1, X) - txz)[:, rows, :] / dx
    stz = (_faceavg(sh(sigma, 1, Z), sigma) * _faceavg(sh(kappa, 1, Z), kappa) * (C - sh(C, 1, Z)) / dz)
    if fsz is not None:
        stz = stz + f(fsz)
    r0, r1 = rzn[:, rows, :], rzn1[:, rows, :]
    wp = (r0 * w + dt * (-conv + vis + (r1 / rho_mean) * stz)) / r1

    # ---------------- y momentum on v faces J = 1 .. ny (ny only for outflow)
    Jv = np.arange(1, ny + 1)
    # y: control-volume faces at cell centres j = J-1 (below) and J (above)
    jc = np.arange(0, ny + 1)                                # centres 0..ny (ny is a ghost row)
    mc = R[:, jc + 2, :] * 0.5 * (Ve[:, jc + 2, :] + Ve[:, jc + 3, :])
    vt = _advected(mc, Ve[:, jc + 1, :], Ve[:, jc + 2, :], Ve[:, jc + 3, :],
                   Ve[:, jc + 4, :], Ve[:, jc + 3, :], Ve[:, jc + 2, :], iface[:, jc + 2, :], M[:, jc + 2, :], dy)
    Fc = mc * vt                                             # index = centre j
    conv = (Fc[:, Jv, :] - Fc[:, Jv - 1, :]) / dy
    # x: edges at u-face columns i, between v columns i-1 and i, rows J-1 and J
    ru_e = rxn * Ue                                          # extended rows
    mX = 0.5 * (ru_e[:, Jv + 1, :] + ru_e[:, Jv + 2, :])
    Vr = Ve[:, Jv + 2, :]
    iexy = iface[:, Jv + 1, :] | iface[:, Jv + 2, :]
    iexy = iexy | sh(iexy, 1, X)
    mexy = 0.25 * (M[:, Jv + 1, :] + M[:, Jv + 2, :])
    mexy = mexy + sh(mexy, 1, X)
    vt = _advected(mX, sh(Vr, 2, X), sh(Vr, 1, X), Vr, sh(Vr, -1, X), Vr, sh(Vr, 1, X), iexy, mexy, dx)
    Fx = mX * vt
    conv = conv + (sh(Fx, -1, X) - Fx) / dx
    # z: edges at back faces k, rows J-1 and J
    mZ = 0.5 * (rw[:, Jv + 1, :] + rw[:, Jv + 2, :])
    iezy = iface[:, Jv + 1, :] | iface[:, Jv + 2, :]
    iezy = iezy | sh(iezy, 1, Z)
    mezy = 0.25 * (M[:, Jv + 1, :] + M[:, Jv + 2, :])
    mezy = mezy + sh(mezy, 1, Z)
    vt = _advected(mZ, sh(Vr, 2, Z), sh(Vr, 1, Z), Vr, sh(Vr, -1, Z), Vr, sh(Vr, 1, Z), iezy, mezy, dz)
    Fz = mZ * vt
    conv = conv + (sh(Fz, -1, Z) - Fz) / dz
    # viscous
    tyy = M[:, jc + 2, :] * (2.0 * (Vve[:, jc + 3, :] - Vve[:, jc + 2, :]) / dy - (2.0 / 3.0) * Dv[:, jc + 2, :])
    vis = (tyy[:, Jv, :] - tyy[:, Jv - 1, :]) / dy
    vis = vis + (sh(txy[:, Jv, :], -1, X) - txy[:, Jv, :]) / dx
    vis = vis + (sh(tyz[:, Jv, :], -1, Z) - tyz[:, Jv, :]) / dz
    Se, Ke = _mirror(sigma), _mirror(kappa)
    sty = (_faceavg(Se[:, Jv + 1, :], Se[:, Jv + 2, :]) * _faceavg(Ke[:, Jv + 1, :], Ke[:, Jv + 2, :])
           * (Ce[:, Jv + 2, :] - Ce[:, Jv + 1, :]) / dy)
    if fsy is not None:
        sty = sty + f(fsy)[:, Jv, :]
    r0, r1 = yface_rho(1, ny + 1), yface_rho(1, ny + 1, n1=True)
    vpi = (r0 * v[:, 1:, :] + dt * (-conv + vis + (r1 / rho_mean) * sty)) / r1
    vp = v.copy()
    vp[:, 1:ny, :] = vpi[:, :ny - 1, :]
    if g.ybc == 1:
        vp[:, ny, :] = vpi[:, ny - 1, :]
    return up, vp, wp
