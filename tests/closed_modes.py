"""Projection problems whose exact discrete solution is a closed form
(Sec. 5.4, Eqs. 28-29 at uniform density).

With rho = rho0 everywhere, p_hat = 0 and S = 0, Eq. (29) reduces to
L p = (rho0/dt) D u* and Eq. (28) to u = u* - (dt/rho0) G p.  Let e be a
discrete eigenfunction of the staggered Laplacian L with eigenvalue lam.  A
velocity u* whose discrete divergence is (dt/rho0) lam e then has the
pressure p = e exactly, and the corrected velocity u* - (dt/rho0) G e.  A
non-constant eigenfunction has zero mean, so the wall gauge (zero-mean p)
leaves it as it is; the outflow top has no gauge.  Sums of modes solve the
sum.  The eigenfunctions are products of
    x:  cos(2 pi a i / nx + phx)                  periodic, cell centres i
    y:  cos(pi m (j + 1/2) / ny)                  walls (Neumann at both ends)
        cos(pi (m + 1/2) (j + 1/2) / ny)          outflow top (p = 0 on the top face)
    z:  cos(2 pi c k / nz + phz)                  periodic
and lam is the sum over the three directions of -(4/h^2) sin^2(t/2), with t
the phase step of that direction.  u* is put on one face family: on u faces
when a != 0 (a sine shifted by half a cell, whose forward difference is the
cosine), else on w faces when c != 0, else on v faces (a sine vanishing on the
bottom face, and on the top face at walls).

Nothing here calls the library or the oracle: these are the values the
method must reach, from the mathematics alone.
"""
import numpy as np


def _steps(nx, ny, nz, ybc, a, m, c):
    tx = 2.0 * np.pi * a / nx
    ty = np.pi * (m + 0.5 * ybc) / ny
    tz = 2.0 * np.pi * c / nz
    return tx, ty, tz


def eigenvalue(nx, ny, nz, lx, ly, lz, ybc, a, m, c):
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    tx, ty, tz = _steps(nx, ny, nz, ybc, a, m, c)
    return -(4 / dx**2) * np.sin(tx / 2) ** 2 - (4 / dy**2) * np.sin(ty / 2) ** 2 - (4 / dz**2) * np.sin(tz / 2) ** 2


def smallest_eigenvalue(nx, ny, nz, lx, ly, lz, ybc):
    """|lam| of the smoothest non-constant mode: the lowest mode of one
    direction (walls), or the (0, 0, 0) mode of the outflow y operator."""
    if ybc == 1:
        return abs(eigenvalue(nx, ny, nz, lx, ly, lz, 1, 0, 0, 0))
    cand = [abs(eigenvalue(nx, ny, nz, lx, ly, lz, 0, *md)) for md, n in
            (((1, 0, 0), nx), ((0, 1, 0), ny), ((0, 0, 1), nz)) if n > 1]
    return min(cand)


def rounding_bound(nx, ny, nz, lx, ly, lz, ybc, modes, amps=None):
    """Relative pressure error that the FP64 rounding of the right-hand side
    alone may cause in any solver: eps times the ratio of the modes' |lam| to
    the smallest |lam| of the operator (a rounding of b reaches the smooth
    modes, which L^-1 amplifies by that ratio).  It exceeds 1e-12 only where
    a high mode meets a domain with a very smooth one (2048 x 3 x 4)."""
    amps = [1.0] * len(modes) if amps is None else amps
    top = sum(abs(a) * abs(eigenvalue(nx, ny, nz, lx, ly, lz, ybc, *md)) for md, a in zip(modes, amps))
    return np.finfo(np.float64).eps * top / (min(abs(a) for a in amps) *
                                             smallest_eigenvalue(nx, ny, nz, lx, ly, lz, ybc))


def _phases(nx, nz, a, c):
    # the Nyquist cosine is the only real mode of its frequency
    phx = 0.0 if (2 * a == nx) else 0.3
    phz = 0.0 if (2 * c == nz) else 1.1
    return phx, phz


def _angle(q, period):
    """2 pi q / period for integer q, reduced exactly to [0, 2 pi) first: a
    product t * i at i ~ 2000 would carry a phase rounding of ~1e-12."""
    return 2.0 * np.pi * (np.asarray(q, dtype=np.int64) % period) / period


def mode_problem(nx, ny, nz, lx, ly, lz, ybc, modes, rho0=640.0, dt=1e-3, amps=None):
    """Fields (us, vs, ws, rho, pn, pnm1, S) and the exact (p, u, v, w) for
    the sum of the given (a, m, c) modes; a constant mode is not allowed."""
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    us = np.zeros((nz, ny, nx))
    vs = np.zeros((nz, ny + 1, nx))
    ws = np.zeros((nz, ny, nx))
    p = np.zeros((nz, ny, nx))
    amps = [1.0] * len(modes) if amps is None else amps
    s = dt / rho0
    for (a, m, c), amp in zip(modes, amps):
        if a == 0 and c == 0 and m == 0 and ybc == 0:
            raise ValueError("the constant mode has no source")
        tx, ty, tz = _steps(nx, ny, nz, ybc, a, m, c)
        phx, phz = _phases(nx, nz, a, c)
        lam = eigenvalue(nx, ny, nz, lx, ly, lz, ybc, a, m, c)
        ii = np.arange(nx, dtype=np.int64)
        jj = np.arange(ny, dtype=np.int64)
        JJ = np.arange(ny + 1, dtype=np.int64)
        kk = np.arange(nz, dtype=np.int64)
        qy = 2 * m + ybc  # y phase step t_y = 2 pi qy / (4 ny)
        fx = np.cos(_angle(a * ii, nx) + phx)
        fy = np.cos(_angle(qy * (2 * jj + 1), 8 * ny))
        fz = np.cos(_angle(c * kk, nz) + phz)
        p += amp * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        if a != 0:
            g = np.sin(_angle(a * (2 * ii - 1), 2 * nx) + phx)  # forward difference 2 sin(tx/2) fx
            us += (amp * s * lam * dx / (2 * np.sin(tx / 2))) * fz[:, None, None] * fy[None, :, None] * g[None, None, :]
        elif c != 0:
            g = np.sin(_angle(c * (2 * kk - 1), 2 * nz) + phz)
            ws += (amp * s * lam * dz / (2 * np.sin(tz / 2))) * g[:, None, None] * fy[None, :, None] * fx[None, None, :]
        else:
            g = np.sin(_angle(qy * 2 * JJ, 8 * ny))  # zero on the bottom face; on the top face too at walls
            if ybc == 0:
                g[-1] = 0.0
            vs += (amp * s * lam * dy / (2 * np.sin(ty / 2))) * fz[:, None, None] * g[None, :, None] * fx[None, None, :]
    # Eq. (28) with the exact pressure: periodic x and z, v fixed on the
    # bottom face (and the top at walls), ghost p = -p beyond an outflow top
    u = us - s * (p - np.roll(p, 1, axis=2)) / dx
    w = ws - s * (p - np.roll(p, 1, axis=0)) / dz
    v = vs.copy()
    v[:, 1:ny, :] -= s * (p[:, 1:, :] - p[:, :-1, :]) / dy
    if ybc == 1:
        v[:, ny, :] -= s * (-2.0 * p[:, ny - 1, :]) / dy
    rho = np.full((nz, ny, nx), rho0)
    zero = np.zeros((nz, ny, nx))
    fields = (us, vs, ws, rho, zero, zero.copy(), zero.copy())
    return fields, {"p": p, "u": u, "v": v, "w": w}


def standard_modes(nx, ny, nz, ybc):
    """The lowest mode of each direction, all three Nyquist frequencies at
    once, and mixed high and low frequencies (every one on a different
    driving face family)."""
    top = ny - 1
    modes = [(1, 0, 0), (0, 1, 0), (0, 0, 1),
             (nx // 2, top, nz // 2),
             (3 % nx, 2 % ny, nz - 1),
             (max(nx // 2 - 1, 1), ny // 2, 5 % nz),
             (0, top, nz // 2), (nx - 1, 1, 0)]
    out = []
    for a, m, c in modes:
        a, m, c = a % nx, m % ny, c % nz
        if a == 0 and m == 0 and c == 0 and ybc == 0:
            continue
        if (a, m, c) not in out:
            out.append((a, m, c))
    return out
