"""Seeded synthetic inputs for the projection step: planar liquid sheets.

This module only builds input fields; it holds none of the projection's
arithmetic (no divergence, gradient or Poisson operator of the method).  The
workload imitates the paper's planar-jet configurations (Sec. 6: liquid sheet
in a gas, periodic in the streamwise and spanwise directions): a sheet
|y| < h(x, z) of liquid density rho_l in gas of density rho_g.  Cell density
follows the one-fluid volume average rho = rho_g + (rho_l - rho_g) C of
Sec. 5.4, with C the exact liquid fraction of each cell in y.

Layouts match the library: C order [nz][ny][nx]; u on west faces (nx per row),
v on south faces (ny+1 per column, the two walls included), w on back faces.
All arrays are float64 numpy arrays.

``ybc`` names the y boundaries a request is posed with: 0 = walls at both ends
(v* = 0 on both), 1 = symmetry plane at the bottom (v* = 0 there) and an
outflow top whose v* is free.  The half-jet generator models the paper's
planar jets, which are symmetric about the centre plane and leave the domain
through an outflow boundary at the top (Sec. 6).
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclasses.dataclass
class Problem:
    """One projection request: grid, scalars and the seven input fields."""

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    rho0: float
    dt: float
    us: np.ndarray
    vs: np.ndarray
    ws: np.ndarray
    rho: np.ndarray
    pn: np.ndarray
    pnm1: np.ndarray
    S: np.ndarray
    meta: Dict = dataclasses.field(default_factory=dict)
    ybc: int = 0

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    def fields(self):
        return (self.us, self.vs, self.ws, self.rho, self.pn, self.pnm1, self.S)


def _centres(n: int, length: float, offset: float = 0.0) -> np.ndarray:
    return offset + (np.arange(n) + 0.5) * (length / n)


def liquid_fraction(nx, ny, nz, lx, ly, lz, h0: float, modes: Sequence[Tuple[float, int, float, int, float]]):
    """Exact y-overlap of each cell with the sheet |y| < h0 + eta(x, z).

    modes: (amplitude, kx, phase_x, kz, phase_z) with
    eta = sum a sin(kx * 2pi x/lx + phx) cos(kz * 2pi z/lz + phz), sampled at
    cell centres.  Returns C in [0, 1] with shape [nz][ny][nx].
    """
    x = _centres(nx, lx)
    z = _centres(nz, lz)
    eta = np.zeros((nz, nx))
    for a, kx, phx, kz, phz in modes:
        eta += a * np.cos(kz * TWO_PI * z / lz + phz)[:, None] * np.sin(kx * TWO_PI * x / lx + phx)[None, :]
    h = np.clip(h0 + eta, 0.0, 0.5 * ly)
    dy = ly / ny
    ylo = -0.5 * ly + np.arange(ny) * dy
    yhi = ylo + dy
    lo = np.maximum(ylo[None, :, None], -h[:, None, :])
    hi = np.minimum(yhi[None, :, None], h[:, None, :])
    return np.clip(hi - lo, 0.0, None) / dy


def smooth_pressure(rng, nx, ny, nz, lx, ly, lz, amp=1e3, nterms=8, kmax=3):
    """Sum of separable cosine modes, wall-compatible in y, amplitude amp."""
    x = _centres(nx, lx)
    y = _centres(ny, ly, -0.5 * ly)
    z = _centres(nz, lz)
    p = np.zeros((nz, ny, nx))
    for _ in range(nterms):
        a, m, e = rng.integers(0, kmax + 1, size=3)
        phx, phz = rng.uniform(0, TWO_PI, size=2)
        c = rng.standard_normal()
        fx = np.cos(a * TWO_PI * x / lx + phx)
        fy = np.cos(np.pi * m * (y + 0.5 * ly) / ly)
        fz = np.cos(e * TWO_PI * z / lz + phz)
        p += c * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    return amp * p


def noise_velocity(rng, nx, ny, nz, ybc=0):
    """u*, v*, w* ~ U(-1, 1) on every non-wall face; v* = 0 on the walls
    (both y ends for ybc 0, the bottom only for ybc 1)."""
    us = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    vs = rng.uniform(-1.0, 1.0, size=(nz, ny + 1, nx))
    vs[:, 0, :] = 0.0
    if ybc == 0:
        vs[:, ny, :] = 0.0
    ws = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    return us, vs, ws


def taylor_green_velocity(rng, nx, ny, nz, lx, ly, lz, noise=0.01):
    """Discretely solenoidal field from a stream function plus noise.

    psi = (1/pi) sin(2pi x/lx) cos(2pi z/lz) sin(2pi (y + ly/2)/ly), sampled on
    the (x-face, y-face) edges; u = (psi_{j+1} - psi_j)/dy,
    v = -(psi_{i+1} - psi_i)/dx, w = 0.  psi vanishes on both walls, so v does.
    Then noise * U(-1, 1) is added on every non-wall face.
    """
    dx, dy = lx / nx, ly / ny
    xe = np.arange(nx + 1) * dx
    ye = -0.5 * ly + np.arange(ny + 1) * dy
    zc = _centres(nz, lz)
    psi = (1.0 / np.pi) * (np.cos(TWO_PI * zc / lz)[:, None, None]
                           * np.sin(TWO_PI * (ye + 0.5 * ly) / ly)[None, :, None]
                           * np.sin(TWO_PI * xe / lx)[None, None, :])
    psi[:, 0, :] = 0.0
    psi[:, ny, :] = 0.0
    psi[:, :, nx] = psi[:, :, 0]
    us = (psi[:, 1:, :nx] - psi[:, :-1, :nx]) / dy
    vs = -(psi[:, :, 1:] - psi[:, :, :nx]) / dx
    ws = np.zeros((nz, ny, nx))
    us = us + noise * rng.uniform(-1.0, 1.0, size=us.shape)
    vn = noise * rng.uniform(-1.0, 1.0, size=vs.shape)
    vn[:, 0, :] = 0.0
    vn[:, ny, :] = 0.0
    vs = vs + vn
    ws = ws + noise * rng.uniform(-1.0, 1.0, size=ws.shape)
    return us, vs, ws


def interface_source(rng, C, amp=1e-3):
    """S ~ N(0, amp^2) on cells with 0 < C < 1 minus its mean there, 0 elsewhere."""
    S = np.zeros(C.shape)
    mask = (C > 0.0) & (C < 1.0)
    n = int(mask.sum())
    if n:
        vals = rng.normal(0.0, amp, size=n)
        S[mask] = vals - vals.mean()
    return S


def random_modes(rng, nmodes, amp_lo=0.005, amp_hi=0.02, kmax=4):
    out = []
    for _ in range(nmodes):
        a = rng.uniform(amp_lo, amp_hi)
        kx, kz = rng.integers(1, kmax + 1, size=2)
        phx, phz = rng.uniform(0, TWO_PI, size=2)
        out.append((a, int(kx), phx, int(kz), phz))
    return out


def sheet_problem(nx, ny, nz, *, seed, rho_l=640.0, rho_g=100.0, h0=0.3, modes=None, nmodes=3,
                  velocity="noise", dt=1e-3, lx=TWO_PI, ly=2.0, lz=TWO_PI, s_amp=1e-3,
                  p_amp=1e3) -> Problem:
    """A two-phase sheet request with every field drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    if modes is None:
        modes = random_modes(rng, nmodes)
    C = liquid_fraction(nx, ny, nz, lx, ly, lz, h0, modes)
    rho = rho_g + (rho_l - rho_g) * C
    if velocity == "noise":
        us, vs, ws = noise_velocity(rng, nx, ny, nz)
    elif velocity == "taylor_green":
        us, vs, ws = taylor_green_velocity(rng, nx, ny, nz, lx, ly, lz)
    else:
        raise ValueError(velocity)
    S = interface_source(rng, C, s_amp)
    pn = smooth_pressure(np.random.default_rng(seed + 7919), nx, ny, nz, lx, ly, lz, amp=p_amp)
    pnm1 = 0.9 * smooth_pressure(np.random.default_rng(seed + 104729), nx, ny, nz, lx, ly, lz, amp=p_amp)
    meta = dict(seed=seed, rho_l=rho_l, rho_g=rho_g, h0=h0, modes=modes, velocity=velocity)
    return Problem(nx, ny, nz, lx, ly, lz, rho_g, dt, us, vs, ws, rho, pn, pnm1, S, meta)


def random_problem(nx, ny, nz, *, seed, lx=TWO_PI, ly=2.0, lz=TWO_PI, dt=1e-3, ybc=0) -> Problem:
    """Unstructured test request: random density in [1, 10] and random fields."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1.0, 10.0, size=(nz, ny, nx))
    us, vs, ws = noise_velocity(rng, nx, ny, nz, ybc)
    S = rng.standard_normal((nz, ny, nx))
    pn = rng.standard_normal((nz, ny, nx))
    pnm1 = rng.standard_normal((nz, ny, nx))
    return Problem(nx, ny, nz, lx, ly, lz, float(rho.min()), dt, us, vs, ws, rho, pn, pnm1, S,
                   dict(seed=seed, kind="random"), ybc)


def half_sheet_fraction(nx, ny, nz, lx, ly, lz, h0: float, modes):
    """Exact y-overlap of each cell of [0, ly] with the liquid 0 <= y < h0 + eta(x, z)
    (the upper half of a sheet symmetric about y = 0; eta as in liquid_fraction)."""
    x = _centres(nx, lx)
    z = _centres(nz, lz)
    eta = np.zeros((nz, nx))
    for a, kx, phx, kz, phz in modes:
        eta += a * np.cos(kz * TWO_PI * z / lz + phz)[:, None] * np.sin(kx * TWO_PI * x / lx + phx)[None, :]
    h = np.clip(h0 + eta, 0.0, ly)
    dy = ly / ny
    ylo = np.arange(ny) * dy
    hi = np.minimum(ylo[None, :, None] + dy, h[:, None, :])
    return np.clip(hi - ylo[None, :, None], 0.0, None) / dy


def outflow_pressure(rng, nx, ny, nz, lx, ly, lz, amp=1e3, nterms=8, kmax=3):
    """Sum of separable modes that are even about y = 0 and vanish at y = ly."""
    x = _centres(nx, lx)
    y = _centres(ny, ly)
    z = _centres(nz, lz)
    p = np.zeros((nz, ny, nx))
    for _ in range(nterms):
        a, m, e = rng.integers(0, kmax + 1, size=3)
        phx, phz = rng.uniform(0, TWO_PI, size=2)
        c = rng.standard_normal()
        fx = np.cos(a * TWO_PI * x / lx + phx)
        fy = np.cos(np.pi * (m + 0.5) * y / ly)
        fz = np.cos(e * TWO_PI * z / lz + phz)
        p += c * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    return amp * p


def jet_problem(nx, ny, nz, *, seed, rho_l=640.0, rho_g=100.0, h0=0.3, modes=None, nmodes=3,
                dt=1e-3, lx=TWO_PI, ly=1.0, lz=TWO_PI, s_amp=1e-3, p_amp=1e3,
                outflow_v=0.05) -> Problem:
    """Half of a planar jet: liquid below h(x, z) over a symmetry plane at y = 0,
    gas above, outflow at y = ly (ybc 1).  u*, w* ~ U(-1, 1); v* ~ U(-1, 1) inside,
    0 on the symmetry plane and outflow_v + 0.1 U(-1, 1) on the top face."""
    rng = np.random.default_rng(seed)
    if modes is None:
        modes = random_modes(rng, nmodes)
    C = half_sheet_fraction(nx, ny, nz, lx, ly, lz, h0, modes)
    rho = rho_g + (rho_l - rho_g) * C
    us, vs, ws = noise_velocity(rng, nx, ny, nz, 1)
    vs[:, ny, :] = outflow_v + 0.1 * rng.uniform(-1.0, 1.0, size=(nz, nx))
    S = interface_source(rng, C, s_amp)
    pn = outflow_pressure(np.random.default_rng(seed + 7919), nx, ny, nz, lx, ly, lz, amp=p_amp)
    pnm1 = 0.9 * outflow_pressure(np.random.default_rng(seed + 104729), nx, ny, nz, lx, ly, lz, amp=p_amp)
    meta = dict(seed=seed, rho_l=rho_l, rho_g=rho_g, h0=h0, modes=modes, kind="half_jet")
    return Problem(nx, ny, nz, lx, ly, lz, rho_g, dt, us, vs, ws, rho, pn, pnm1, S, meta, 1)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def sheet_32(seed=1000) -> Problem:
    """32^3 sheet, rho 640/100, eta = 0.02 sin x cos z, noise u*."""
    return sheet_problem(32, 32, 32, seed=seed, rho_l=640.0, rho_g=100.0, h0=0.3,
                         modes=[(0.02, 1, 0.0, 1, 0.0)], velocity="noise")


def sheet_256(seed=2000) -> Problem:
    """256x128x256 sheet, rho 640/100, 3 random interface modes, Taylor-Green u*."""
    return sheet_problem(256, 128, 256, seed=seed, rho_l=640.0, rho_g=100.0, h0=0.3,
                         nmodes=3, velocity="taylor_green")


def sheet_512(seed=3000, velocity="noise") -> Problem:
    """512x256x512 sheet, rho 640/60, 5 random interface modes."""
    return sheet_problem(512, 256, 512, seed=seed, rho_l=640.0, rho_g=60.0, h0=0.3,
                         nmodes=5, velocity=velocity)


def jet_32(seed=5000) -> Problem:
    """32^3 half jet over a symmetry plane with an outflow top, rho 640/100."""
    return jet_problem(32, 32, 32, seed=seed, modes=[(0.02, 1, 0.0, 1, 0.0)])


def jet_256(seed=6000) -> Problem:
    """256x128x256 half jet over a symmetry plane with an outflow top, rho 640/100."""
    return jet_problem(256, 128, 256, seed=seed, nmodes=3)


BATCH_SHAPES = [(64, 64, 64), (96, 64, 96), (128, 64, 128), (192, 96, 192)]
SERVE_SHAPES = [(32, 32, 32), (64, 64, 64), (96, 64, 96), (128, 64, 128), (192, 96, 192), (256, 128, 256)]


def mixed_instance(seed, shapes=BATCH_SHAPES, shape=None) -> Problem:
    """One request of the uneven-size mix: ratio ~ U(3, 12), h0 ~ U(0.15, 0.45)."""
    rng = np.random.default_rng(seed)
    if shape is None:
        shape = shapes[int(rng.integers(0, len(shapes)))]
    ratio = rng.uniform(3.0, 12.0)
    h0 = rng.uniform(0.15, 0.45)
    nx, ny, nz = shape
    return sheet_problem(nx, ny, nz, seed=seed + 17, rho_l=100.0 * ratio, rho_g=100.0, h0=h0,
                         nmodes=3, velocity="noise")


def batch_shapes(count=48, seed=4000, shapes=BATCH_SHAPES) -> List[Tuple[int, int, int]]:
    rng = np.random.default_rng(seed)
    return [shapes[int(i)] for i in rng.integers(0, len(shapes), size=count)]


def batch_48(seed=4000, count=48) -> List[Problem]:
    """48 independent requests of uneven sizes (same-shape ones share launches)."""
    shapes = batch_shapes(count, seed)
    return [mixed_instance(seed + 1 + i, shape=s) for i, s in enumerate(shapes)]


# ---------------------------------------------------------------------------
# Inputs of the target divergence S (Eq. 26): phase-wise compressibilities,
# interface mass flux and area density, interface densities, under-resolved
# mask.  The generator draws them; it does not form S.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Sources:
    C: np.ndarray             # liquid volume fraction
    div_g: np.ndarray         # gas-phase velocity divergence (extrapolated into the liquid band)
    div_l: np.ndarray         # liquid-phase velocity divergence
    mdot_area: np.ndarray     # interface mass flux per unit area (0 outside interface cells)
    area_density: np.ndarray  # interface area per cell volume (0 outside interface cells)
    rho_g: np.ndarray         # interface gas density (0 outside interface cells)
    rho_l: np.ndarray         # interface liquid density (0 outside interface cells)
    under: np.ndarray         # uint8, 1 in the under-resolved block

    def fields(self):
        return (self.C, self.div_g, self.div_l, self.mdot_area, self.area_density, self.rho_g, self.rho_l,
                self.under)


def smooth_field(rng, nx, ny, nz, lx, ly, lz, amp, nterms=6, kmax=3):
    """amp * sum of separable cosine modes with N(0, 1) weights (no y boundary condition)."""
    x = _centres(nx, lx)
    y = _centres(ny, ly)
    z = _centres(nz, lz)
    f = np.zeros((nz, ny, nx))
    for _ in range(nterms):
        a, m, e = rng.integers(0, kmax + 1, size=3)
        phx, phy, phz = rng.uniform(0, TWO_PI, size=3)
        c = rng.standard_normal()
        f += c * (np.cos(e * TWO_PI * z / lz + phz)[:, None, None]
                  * np.cos(m * np.pi * y / ly + phy)[None, :, None]
                  * np.cos(a * TWO_PI * x / lx + phx)[None, None, :])
    return amp * f


def interface_inputs(rng, C, lx, ly, lz, rho_l, rho_g, div_g_amp=1e-2, div_l_amp=1e-3, mdot_mean=0.3,
                     mdot_sd=0.1, under_frac=0.125) -> Sources:
    """Eq. (26) inputs around the interface described by C.

    div_g, div_l: smooth fields of amplitude div_g_amp, div_l_amp everywhere
    (the extrapolated compressibilities cover both phases' bands).  In
    interface cells (0 < C < 1): m' ~ N(mdot_mean, mdot_sd^2) (vaporisation
    positive), A/V0 = U(0.9, 1.3)/dy, rho_g(1 + U(-0.03, 0.03)),
    rho_l(1 + U(-0.01, 0.01)); those four arrays are 0 elsewhere.  The
    under-resolved mask flags the cells of one x-z block covering
    under_frac of the x range and half of the z range, all y."""
    nz, ny, nx = C.shape
    dy = ly / ny
    div_g = smooth_field(rng, nx, ny, nz, lx, ly, lz, div_g_amp)
    div_l = smooth_field(rng, nx, ny, nz, lx, ly, lz, div_l_amp)
    iface = (C > 0.0) & (C < 1.0)
    n = int(iface.sum())
    mdot = np.zeros(C.shape)
    area = np.zeros(C.shape)
    rg = np.zeros(C.shape)
    rl = np.zeros(C.shape)
    mdot[iface] = rng.normal(mdot_mean, mdot_sd, size=n)
    area[iface] = rng.uniform(0.9, 1.3, size=n) / dy
    rg[iface] = rho_g * (1.0 + rng.uniform(-0.03, 0.03, size=n))
    rl[iface] = rho_l * (1.0 + rng.uniform(-0.01, 0.01, size=n))
    under = np.zeros(C.shape, dtype=np.uint8)
    wx = max(1, int(round(under_frac * nx)))
    x0 = int(rng.integers(0, nx))
    z0 = int(rng.integers(0, nz))
    xs = (x0 + np.arange(wx)) % nx
    zs = (z0 + np.arange(max(1, nz // 2))) % nz
    under[np.ix_(zs, np.arange(ny), xs)] = 1
    return Sources(C, div_g, div_l, mdot, area, rg, rl, under)


def sheet_sources(nx, ny, nz, *, seed, rho_l=640.0, rho_g=100.0, h0=0.3, nmodes=3, lx=TWO_PI, ly=2.0,
                  lz=TWO_PI) -> Sources:
    """Eq. (26) inputs for the liquid sheet |y| < h0 + eta(x, z) of sheet_problem."""
    rng = np.random.default_rng(seed)
    modes = random_modes(rng, nmodes)
    C = liquid_fraction(nx, ny, nz, lx, ly, lz, h0, modes)
    return interface_inputs(rng, C, lx, ly, lz, rho_l, rho_g)


def sources_256(seed=7000) -> Sources:
    """256x128x256 sheet, rho 640/100: inputs of S."""
    return sheet_sources(256, 128, 256, seed=seed)


# ---------------------------------------------------------------------------
# Inputs of the predictor (Eq. 23) around a request's interface: viscosity,
# volume fraction, surface tension and curvature.  Drawn, not computed.
# ---------------------------------------------------------------------------

def predictor_inputs(pr: Problem, seed: int, mu_l=2e-3, mu_g=2e-5, sigma=0.02, drho=0.02) -> Dict:
    """Predictor inputs for request `pr`: u^n = its u*, v*, w*; rho^n = its rho;
    rho^{n+1} = rho (1 + drho U(-1, 1)); C from rho (the generator's own
    rho = rho_g + (rho_l - rho_g) C); mu = mu_g + (mu_l - mu_g) C; in interface
    cells sigma = sigma (1 + 0.1 U(-1, 1)) and kappa = N(0, 1) / h0, zero
    elsewhere; <rho> = (rho_g + rho_l)/2."""
    rng = np.random.default_rng(seed)
    rl, rg = pr.meta["rho_l"], pr.meta["rho_g"]
    C = (pr.rho - rg) / (rl - rg)
    iface = (C > 0.0) & (C < 1.0)
    n = int(iface.sum())
    sg = np.zeros(C.shape)
    kp = np.zeros(C.shape)
    sg[iface] = sigma * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, size=n))
    kp[iface] = rng.standard_normal(n) / pr.meta.get("h0", 0.3)
    return {"u": pr.us, "v": pr.vs, "w": pr.ws, "rho_n": pr.rho,
            "rho_np1": pr.rho * (1.0 + drho * rng.uniform(-1.0, 1.0, size=C.shape)),
            "mu": mu_g + (mu_l - mu_g) * C, "C": C, "sigma": sg, "kappa": kp,
            "rho_mean": 0.5 * (rg + rl), "dt": pr.dt}
