"""Shared GPU-vs-oracle comparison for the projection step (Sec. 5.4).

Two norms per result, both relative to the oracle:
  l2   eps_p  = ||p - p_o||_2 / ||p_o||_2                     (both zero-mean)
       eps_du = ||(u - u*) - (u_o - u*)||_2 / ||u_o - u*||_2  (u, v, w together)
  linf inf_p  = max|p - p_o| / max|p_o|
       inf_du[c] = max|du_c - du_o,c| / max|du_o,c|, c = u, v, w separately
The l2 norms alone could hide an error confined to one y row, one kx column
or the Nyquist plane of a grid of millions of points; the per-point bounds
catch those.  A pointwise error spread evenly over many points is a few times
its rms, so the linf bounds are set at the l2 bound (p) and ten times it
(each velocity component, whose smallest entries carry the largest relative
rounding); a test that widens an l2 bound from the oracle's own conditioning
widens the matching linf bound by the same factor.
"""
import numpy as np

import oracle as O

TOL = 1e-12


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_step(pr, rho0=None, method="spectral"):
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, ybc=pr.ybc)
    return O.ppe_step(g, pr.rho0 if rho0 is None else rho0, pr.dt, *pr.fields(), method=method)


def errors(pr, got, ref):
    comps = (("u", "us"), ("v", "vs"), ("w", "ws"))
    du = {k: got[k] - getattr(pr, s) for k, s in comps}
    duo = {k: ref[k] - getattr(pr, s) for k, s in comps}
    cat = lambda d: np.concatenate([d[k].ravel() for k, _ in comps])
    out = {"eps_p": rel(got["p"], ref["p"]), "eps_du": rel(cat(du), cat(duo)),
           "inf_p": rel_inf(got["p"], ref["p"])}
    for k, _ in comps:
        out["inf_d" + k] = rel_inf(du[k], duo[k])
    return out


def check(pr, got, rec, ref, tol=TOL, tol_p=None, tol_du=None, tol_div=None, tol_inf_du=None, label=""):
    """Every bound of the projection step against the oracle's result `ref`.
    tol_inf_du overrides the pointwise velocity bound (10 x the l2 one)."""
    e = errors(pr, got, ref)
    tp = tol if tol_p is None else tol_p
    tu = tol if tol_du is None else tol_du
    tiu = 10.0 * tu if tol_inf_du is None else tol_inf_du
    print(f"[{label}{pr.nx}x{pr.ny}x{pr.nz}] eps_p={e['eps_p']:.2e} eps_du={e['eps_du']:.2e} "
          f"inf_p={e['inf_p']:.2e} inf_du=({e['inf_du']:.2e},{e['inf_dv']:.2e},{e['inf_dw']:.2e}) "
          f"eps_div={rec['res_rel']:.2e} iters={rec['iters']} status={rec['status']}", flush=True)
    assert rec["status"] == 0, rec
    assert e["eps_p"] <= tp, e
    assert e["eps_du"] <= tu, e
    assert e["inf_p"] <= tp, e
    for k in ("inf_du", "inf_dv", "inf_dw"):
        assert e[k] <= tiu, (k, e)
    assert rec["res_rel"] <= (tol if tol_div is None else tol_div), rec
    assert abs(rec["rho0_used"] - ref["rho0"]) <= 1e-15 * ref["rho0"]
    # v on the bottom face (wall or symmetry plane) is copied, never corrected
    assert np.array_equal(got["v"][:, 0, :], pr.vs[:, 0, :])
    if pr.ybc == 0:
        assert abs(rec["p_mean"]) <= 1e-13 * np.abs(ref["p"]).max()
        assert np.array_equal(got["v"][:, -1, :], pr.vs[:, -1, :])
        scale = abs(ref["compat"]) + ref["div0_l2"] / np.sqrt(pr.npts)
        assert abs(rec["compat_defect"] - ref["compat"]) <= 1e-13 * scale
    else:
        # outflow top: nothing removed, no gauge, top face corrected
        assert rec["compat_defect"] == 0.0
        assert abs(rec["p_mean"] - ref["p"].mean()) <= 1e-12 * np.abs(ref["p"]).max()
        assert not np.array_equal(got["v"][:, -1, :], pr.vs[:, -1, :])
    return e
