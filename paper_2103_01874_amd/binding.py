"""Thin ctypes binding of libppe.so (include/ppe.h): argument marshalling only.

Every step of the projection runs in the HIP library.  This module checks
shapes, dtypes and devices of torch tensors, passes their device pointers
and the current HIP stream, and decodes the per-instance ``ppe_info_t``
records.  It fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppe.so")

PPE_PREC_FP64 = 0
PPE_PREC_MIXED = 1
PPE_YBC_WALLS = 0
PPE_YBC_OUTFLOW = 1
PPE_FLAG_VARCOEF = 1
PPE_FLAG_Y_REFINE = 2
PPE_OK = 0
PPE_ERR_ARG = -1
PPE_ERR_NOMEM = -2
PPE_ERR_NOT_CONVERGED = -4
PPE_ERR_UNSUPPORTED = -6
MAX_BATCH = 64

STATUS = {0: "ok", -1: "bad argument", -2: "out of memory", -3: "device error", -4: "not converged",
          -5: "non-finite", -6: "unsupported"}


class PPEError(RuntimeError):
    pass


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("precision", ctypes.c_int32), ("ybc", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_refine", ctypes.c_int32), ("batch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


assert ctypes.sizeof(Desc) == 72


INFO_DTYPE = np.dtype([("status", "<i4"), ("iters", "<i4"), ("rho0_used", "<f8"), ("compat_defect", "<f8"),
                       ("res_rel", "<f8"), ("div_l2", "<f8"), ("div_max", "<f8"), ("div0_l2", "<f8"),
                       ("p_mean", "<f8")])
assert INFO_DTYPE.itemsize == 64

EXPORTS = ["ppe_plan_workspace_bytes", "ppe_plan", "ppe_plan_destroy", "ppe_plan_set_stream", "ppe_solve",
           "ppe_rhs", "ppe_correct", "ppe_residual", "ppe_source", "ppe_predict", "ppe_solve_varcoef", "ppe_ring_create",
           "ppe_ring_step",
           "ppe_ring_pressure", "ppe_ring_read", "ppe_ring_steps", "ppe_ring_destroy", "ppe_plan_profile",
           "ppe_plan_profile_read", "ppe_version", "ppe_solve_noalloc"]

SOURCE_FIELDS = ("C", "div_g", "div_l", "mdot", "area", "rho_g", "rho_l")


PREDICT_FIELDS = ("u", "v", "w", "uv", "vv", "wv", "rho_n", "rho_np1", "mu", "C", "sigma", "kappa", "fsx", "fsy",
                  "fsz")
PREDICT_OPTIONAL = ("uv", "vv", "wv", "fsx", "fsy", "fsz")
PREDICT_VFACE = ("v", "vv", "fsy")


class PredictIn(ctypes.Structure):
    """ppe_predict_t: device pointers of the Eq. (23) inputs of one instance."""
    _fields_ = [(k, ctypes.c_void_p) for k in PREDICT_FIELDS] + [("rho_mean", ctypes.c_double),
                                                                  ("dt", ctypes.c_double)]


class Source(ctypes.Structure):
    """ppe_source_t: device pointers of the Eq. (26) inputs of one instance."""
    _fields_ = [(k, ctypes.c_void_p) for k in SOURCE_FIELDS] + [("under", ctypes.c_void_p)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]

_lib = None


def load(path: str = LIB_PATH):
    """Load libppe.so once; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PPEError(f"{path} is not built; run `python -m paper_2103_01874_amd.build`")
    # torch first: its bundled HIP runtime (same soname) must be the one the
    # library binds to, or torch and the library would run on two runtimes
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    D = ctypes.POINTER(ctypes.c_double)
    lib.ppe_plan_workspace_bytes.argtypes = [ctypes.POINTER(Desc)]
    lib.ppe_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.ppe_plan.argtypes = [ctypes.POINTER(Desc), P, ctypes.POINTER(P)]
    lib.ppe_plan.restype = ctypes.c_int
    lib.ppe_plan_destroy.argtypes = [P]
    lib.ppe_plan_destroy.restype = ctypes.c_int
    lib.ppe_plan_set_stream.argtypes = [P, P]
    lib.ppe_plan_set_stream.restype = ctypes.c_int
    lib.ppe_solve.argtypes = [P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, P]
    lib.ppe_solve.restype = ctypes.c_int
    lib.ppe_rhs.argtypes = [P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, P]
    lib.ppe_rhs.restype = ctypes.c_int
    lib.ppe_solve_noalloc.argtypes = [ctypes.POINTER(Desc), P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, PP, PP, PP, P]
    lib.ppe_solve_noalloc.restype = ctypes.c_int
    lib.ppe_correct.argtypes = [P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, PP, PP, PP, P]
    lib.ppe_correct.restype = ctypes.c_int
    lib.ppe_residual.argtypes = [P, PP, PP, PP, PP, P]
    lib.ppe_residual.restype = ctypes.c_int
    lib.ppe_source.argtypes = [P, ctypes.POINTER(Source), PP]
    lib.ppe_source.restype = ctypes.c_int
    lib.ppe_predict.argtypes = [P, ctypes.POINTER(PredictIn), PP, PP, PP]
    lib.ppe_predict.restype = ctypes.c_int
    lib.ppe_solve_varcoef.argtypes = [P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, P, ctypes.c_int32, ctypes.c_double,
                                      P]
    lib.ppe_solve_varcoef.restype = ctypes.c_int
    lib.ppe_ring_create.argtypes = [P, PP, PP, ctypes.POINTER(P)]
    lib.ppe_ring_create.restype = ctypes.c_int
    lib.ppe_ring_step.argtypes = [P, D, D, PP, PP, PP, PP, PP, PP, PP, PP, P, P]
    lib.ppe_ring_step.restype = ctypes.c_int
    lib.ppe_ring_pressure.argtypes = [P, ctypes.c_int32, PP]
    lib.ppe_ring_pressure.restype = ctypes.c_int
    lib.ppe_ring_read.argtypes = [P, ctypes.c_int32, PP]
    lib.ppe_ring_read.restype = ctypes.c_int
    lib.ppe_ring_steps.argtypes = [P]
    lib.ppe_ring_steps.restype = ctypes.c_int64
    lib.ppe_ring_destroy.argtypes = [P]
    lib.ppe_ring_destroy.restype = ctypes.c_int
    lib.ppe_plan_profile.argtypes = [P, ctypes.c_int32]
    lib.ppe_plan_profile.restype = ctypes.c_int
    lib.ppe_plan_profile_read.argtypes = [P, ctypes.POINTER(KernelTime), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.ppe_plan_profile_read.restype = ctypes.c_int
    lib.ppe_version.argtypes = []
    lib.ppe_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_desc(nx, ny, nz, lx=2 * np.pi, ly=2.0, lz=2 * np.pi, precision=PPE_PREC_FP64, tol=1e-12,
              max_refine=1, batch=1, ybc=PPE_YBC_WALLS, flags=0) -> Desc:
    return Desc(int(nx), int(ny), int(nz), float(lx), float(ly), float(lz), int(precision), int(ybc),
                float(tol), int(max_refine), int(batch), int(flags), 0)


def workspace_bytes(desc: Desc) -> int:
    return int(load().ppe_plan_workspace_bytes(ctypes.byref(desc)))


def _check(st: int, what: str):
    if st != 0:
        raise PPEError(f"{what} failed: {STATUS.get(st, st)}")


def _ptrs(tensors) -> ctypes.Array:
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


def _dbl(vals) -> ctypes.Array:
    arr = (ctypes.c_double * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = float(v)
    return arr


def decode_info(info_tensor) -> List[Dict]:
    """Copy ppe_info_t records (device tensor of float64, 8 per record) to dicts."""
    raw = info_tensor.detach().cpu().numpy().tobytes()
    recs = np.frombuffer(raw, dtype=INFO_DTYPE)
    return [{k: (int(r[k]) if k in ("status", "iters") else float(r[k])) for k in INFO_DTYPE.names} for r in recs]


class Plan:
    """A plan for `batch` same-shape instances, bound to a torch CUDA stream."""

    def __init__(self, nx, ny, nz, lx=2 * np.pi, ly=2.0, lz=2 * np.pi, precision=PPE_PREC_FP64, tol=1e-12,
                 max_refine=1, batch=1, stream=None, device=None, ybc=PPE_YBC_WALLS, flags=0):
        import torch

        self._torch = torch
        self.lib = load()
        self.desc = make_desc(nx, ny, nz, lx, ly, lz, precision, tol, max_refine, batch, ybc, flags)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.ppe_plan(ctypes.byref(self.desc), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(self._h)), "ppe_plan")
        self.nx, self.ny, self.nz, self.batch = int(nx), int(ny), int(nz), int(batch)
        # what every field tensor must match (checked on each call, cheaply)
        self._shape_c = torch.Size((self.nz, self.ny, self.nx))
        self._shape_v = torch.Size((self.nz, self.ny + 1, self.nx))
        self._dev_index = self.device.index

    @property
    def workspace_bytes(self) -> int:
        return workspace_bytes(self.desc)

    def set_stream(self, stream):
        self.stream = stream
        _check(self.lib.ppe_plan_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "ppe_plan_set_stream")

    def profile(self, enable: bool):
        """Turn per-kernel HIP-event timing on (clearing totals) or off."""
        _check(self.lib.ppe_plan_profile(self._h, 1 if enable else 0), "ppe_plan_profile")

    def profile_read(self) -> Dict[str, Dict]:
        """{kernel family: {"launches": n, "total_ms": t, "avg_us": t/n*1e3}} (waits for the stream)."""
        cap = 64
        buf = (KernelTime * cap)()
        n = ctypes.c_int32(0)
        _check(self.lib.ppe_plan_profile_read(self._h, buf, cap, ctypes.byref(n)), "ppe_plan_profile_read")
        out = {}
        for i in range(min(n.value, cap)):
            k = buf[i]
            out[k.name.decode()] = {"launches": int(k.launches), "total_ms": float(k.total_ms),
                                    "avg_us": 1e3 * float(k.total_ms) / max(1, int(k.launches))}
        return out

    def close(self):
        if self._h is not None and self._h.value:
            self.lib.ppe_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- validation ---------------------------------------------------------
    def _field(self, t, shape, name, i):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.shape != shape \
                or not t.is_cuda or t.get_device() != self._dev_index or not t.is_contiguous():
            raise PPEError(f"{name}[{i}]: expected contiguous float64 {tuple(shape)} on {self.device}")
        return t

    def _cell(self, t, name):
        return self._field(t, self._shape_c, name, 0)

    def _vface(self, t, name):
        return self._field(t, self._shape_v, name, 0)

    def _batch(self, seq, name, v=False):
        if len(seq) != self.batch:
            raise PPEError(f"{name}: expected {self.batch} tensors, got {len(seq)}")
        shape = self._shape_v if v else self._shape_c
        return [self._field(t, shape, name, i) for i, t in enumerate(seq)]

    def new_info(self):
        """Zeroed info records, allocated and cleared on the plan's stream (the
        library writes them on that stream, so the fill is ordered before)."""
        torch = self._torch
        with torch.cuda.stream(self.stream):
            return torch.zeros(self.batch * 8, dtype=torch.float64, device=self.device)

    # -- entry points -------------------------------------------------------
    def solve(self, rho0: Sequence[float], dt: Sequence[float], us, vs, ws, rho, pn, pnm1, S, p, info=None):
        """ppe_solve: writes p (list of tensors) and the info records (returned)."""
        if info is None:
            info = self.new_info()
        B = self.batch
        if len(rho0) != B or len(dt) != B:
            raise PPEError("rho0 and dt need one value per instance")
        args = [self._batch(us, "us"), self._batch(vs, "vs", v=True), self._batch(ws, "ws"),
                self._batch(rho, "rho"), self._batch(pn, "pn"), self._batch(pnm1, "pnm1"), self._batch(S, "S"),
                self._batch(p, "p")]
        st = self.lib.ppe_solve(self._h, _dbl(rho0), _dbl(dt), *[_ptrs(a) for a in args],
                                ctypes.c_void_p(info.data_ptr()))
        _check(st, "ppe_solve")
        return info

    def rhs(self, rho0: Sequence[float], dt: Sequence[float], us, vs, ws, rho, pn, pnm1, S, b, info=None):
        """ppe_rhs: the right-hand side of Eq. (29) into the tensors b; returns info."""
        if info is None:
            info = self.new_info()
        B = self.batch
        if len(rho0) != B or len(dt) != B:
            raise PPEError("rho0 and dt need one value per instance")
        args = [self._batch(us, "us"), self._batch(vs, "vs", v=True), self._batch(ws, "ws"),
                self._batch(rho, "rho"), self._batch(pn, "pn"), self._batch(pnm1, "pnm1"), self._batch(S, "S"),
                self._batch(b, "b")]
        st = self.lib.ppe_rhs(self._h, _dbl(rho0), _dbl(dt), *[_ptrs(a) for a in args],
                              ctypes.c_void_p(info.data_ptr()))
        _check(st, "ppe_rhs")
        return info

    def solve_varcoef(self, rho0: Sequence[float], dt: Sequence[float], us, vs, ws, rho, pn, pnm1, S, p,
                      max_iters: int, tol: float, info=None, hist=None):
        """ppe_solve_varcoef: pressure of Eq. (25) by the split fixed point.
        Returns (info, hist); hist is a float64 tensor [batch][max_iters + 1]
        of relative residuals (-1 after convergence) when requested with
        hist=True or given as a tensor."""
        torch = self._torch
        if info is None:
            info = self.new_info()
        if hist is True:
            hist = torch.empty(self.batch * (max_iters + 1), dtype=torch.float64, device=self.device)
        B = self.batch
        if len(rho0) != B or len(dt) != B:
            raise PPEError("rho0 and dt need one value per instance")
        args = [self._batch(us, "us"), self._batch(vs, "vs", v=True), self._batch(ws, "ws"),
                self._batch(rho, "rho"), self._batch(pn, "pn"), self._batch(pnm1, "pnm1"), self._batch(S, "S"),
                self._batch(p, "p")]
        hp = ctypes.c_void_p(hist.data_ptr()) if hist is not None else None
        st = self.lib.ppe_solve_varcoef(self._h, _dbl(rho0), _dbl(dt), *[_ptrs(a) for a in args],
                                        ctypes.c_void_p(info.data_ptr()), int(max_iters), float(tol), hp)
        _check(st, "ppe_solve_varcoef")
        return info, hist

    def correct(self, dt: Sequence[float], us, vs, ws, rho, pn, pnm1, p, S, u, v, w, info=None, rho0=None):
        """ppe_correct: writes u, v, w and the continuity fields of `info`.

        rho0=None projects with the rho0 and compatibility defect that
        ppe_solve left in `info`; a sequence of per-instance values (<= 0:
        min(rho)) projects a pressure from anywhere, and `info` is then
        initialised by the call (allocated here when None)."""
        if info is None:
            if rho0 is None:
                raise PPEError("correct: without rho0 the info records of the solve are needed")
            info = self.new_info()
        if rho0 is not None and len(rho0) != self.batch:
            raise PPEError("rho0 needs one value per instance")
        if len(dt) != self.batch:
            raise PPEError("dt needs one value per instance")
        args = [self._batch(us, "us"), self._batch(vs, "vs", v=True), self._batch(ws, "ws"),
                self._batch(rho, "rho"), self._batch(pn, "pn"), self._batch(pnm1, "pnm1"), self._batch(p, "p"),
                self._batch(S, "S"), self._batch(u, "u"), self._batch(v, "v", v=True), self._batch(w, "w")]
        st = self.lib.ppe_correct(self._h, _dbl(rho0) if rho0 is not None else None, _dbl(dt),
                                  *[_ptrs(a) for a in args], ctypes.c_void_p(info.data_ptr()))
        _check(st, "ppe_correct")
        return info

    def source(self, srcs: Sequence[Dict], S):
        """ppe_source: S[i] from the Eq. (26) inputs srcs[i] (dicts of float64
        cell tensors named as SOURCE_FIELDS, plus an optional uint8 'under')."""
        torch = self._torch
        if len(srcs) != self.batch:
            raise PPEError(f"sources: expected {self.batch} records, got {len(srcs)}")
        recs = (Source * self.batch)()
        for i, d in enumerate(srcs):
            for k in SOURCE_FIELDS:
                if d.get(k) is None:
                    raise PPEError(f"sources[{i}]: missing {k}")
                setattr(recs[i], k, self._field(d[k], self._shape_c, k, i).data_ptr())
            m = d.get("under")
            if m is not None:
                if not isinstance(m, torch.Tensor) or m.dtype != torch.uint8 or m.device != self.device \
                        or tuple(m.shape) != (self.nz, self.ny, self.nx) or not m.is_contiguous():
                    raise PPEError(f"under[{i}]: expected contiguous uint8 cell tensor on {self.device}")
                recs[i].under = m.data_ptr()
            else:
                recs[i].under = None
        outs = self._batch(S, "S")
        _check(self.lib.ppe_source(self._h, recs, _ptrs(outs)), "ppe_source")
        return S

    def predict(self, ins: Sequence[Dict], up, vp, wp):
        """ppe_predict: u^p, v^p, w^p of Eq. (23) from the records `ins` (dicts
        of float64 tensors named as PREDICT_FIELDS, optional ones may be absent,
        plus 'rho_mean' and 'dt' floats)."""
        if len(ins) != self.batch:
            raise PPEError(f"predict: expected {self.batch} records, got {len(ins)}")
        recs = (PredictIn * self.batch)()
        for i, d in enumerate(ins):
            for k in PREDICT_FIELDS:
                t = d.get(k)
                if t is None:
                    if k in PREDICT_OPTIONAL:
                        setattr(recs[i], k, None)
                        continue
                    raise PPEError(f"predict[{i}]: missing {k}")
                chk = self._vface if k in PREDICT_VFACE else self._cell
                setattr(recs[i], k, chk(t, f"{k}[{i}]").data_ptr())
            recs[i].rho_mean = float(d["rho_mean"])
            recs[i].dt = float(d["dt"])
        st = self.lib.ppe_predict(self._h, recs, _ptrs(self._batch(up, "up")), _ptrs(self._batch(vp, "vp", v=True)),
                                  _ptrs(self._batch(wp, "wp")))
        _check(st, "ppe_predict")
        return up, vp, wp

    def residual(self, u, v, w, S, out=None):
        """ppe_residual: per instance (||d - mean d||_2, max|d - mean d|, mean d), d = D u - S."""
        torch = self._torch
        if out is None:
            out = torch.zeros(self.batch * 3, dtype=torch.float64, device=self.device)
        args = [self._batch(u, "u"), self._batch(v, "v", v=True), self._batch(w, "w"), self._batch(S, "S")]
        st = self.lib.ppe_residual(self._h, *[_ptrs(a) for a in args], ctypes.c_void_p(out.data_ptr()))
        _check(st, "ppe_residual")
        return out


def to_device(problem, device="cuda"):
    """Copy a synth.Problem's fields to the device (float64, contiguous)."""
    import torch

    return {k: torch.from_numpy(np.ascontiguousarray(getattr(problem, k))).to(device)
            for k in ("us", "vs", "ws", "rho", "pn", "pnm1", "S")}


class Ring:
    """Device-resident pressure history for a time loop (ppe_ring_*)."""

    def __init__(self, plan: Plan, pn, pnm1=None):
        self.plan = plan
        self.lib = plan.lib
        self._h = ctypes.c_void_p()
        a = _ptrs(plan._batch(pn, "pn"))
        b = _ptrs(plan._batch(pnm1, "pnm1")) if pnm1 is not None else None
        _check(self.lib.ppe_ring_create(plan._h, a, b, ctypes.byref(self._h)), "ppe_ring_create")

    def step(self, rho0, dt, us, vs, ws, rho, S, u, v, w, info=None, defect=False):
        """One projection step with the ring's history; returns (info, defect)
        where defect is a [batch][2] tensor of Eq. (25) residuals when asked."""
        plan = self.plan
        torch = plan._torch
        if info is None:
            info = plan.new_info()
        d = None
        if defect is True:
            d = torch.empty(plan.batch * 2, dtype=torch.float64, device=plan.device)
        elif defect is not False and defect is not None:
            d = defect
        B = plan.batch
        if len(rho0) != B or len(dt) != B:
            raise PPEError("rho0 and dt need one value per instance")
        args = [plan._batch(us, "us"), plan._batch(vs, "vs", v=True), plan._batch(ws, "ws"),
                plan._batch(rho, "rho"), plan._batch(S, "S"), plan._batch(u, "u"), plan._batch(v, "v", v=True),
                plan._batch(w, "w")]
        st = self.lib.ppe_ring_step(self._h, _dbl(rho0), _dbl(dt), *[_ptrs(x) for x in args],
                                    ctypes.c_void_p(info.data_ptr()),
                                    ctypes.c_void_p(d.data_ptr()) if d is not None else None)
        _check(st, "ppe_ring_step")
        return info, d

    def read(self, lag, out):
        """Copy p^n (lag 0) or p^{n-1} (lag 1) into the tensors `out`."""
        _check(self.lib.ppe_ring_read(self._h, int(lag), _ptrs(self.plan._batch(out, "out"))), "ppe_ring_read")
        return out

    @property
    def steps(self) -> int:
        return int(self.lib.ppe_ring_steps(self._h))

    def close(self):
        if self._h:
            self.lib.ppe_ring_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sources_to_device(src, device="cuda") -> Dict:
    """Copy a synth.Sources' fields to the device under the binding's names."""
    import torch

    names = {"C": "C", "div_g": "div_g", "div_l": "div_l", "mdot": "mdot_area", "area": "area_density",
             "rho_g": "rho_g", "rho_l": "rho_l", "under": "under"}
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(src, v))).to(device) for k, v in names.items()}


def step(plan: Plan, fields: List[Dict], rho0, dt, outputs: Optional[List[Dict]] = None, info=None):
    """solve + correct for a batch of field dicts; returns (outputs, info tensor)."""
    torch = plan._torch
    if outputs is None:
        # allocated on the plan's stream, which writes them
        with torch.cuda.stream(plan.stream):
            outputs = [{"p": torch.empty_like(f["rho"]), "u": torch.empty_like(f["us"]),
                        "v": torch.empty_like(f["vs"]), "w": torch.empty_like(f["ws"])} for f in fields]
    g = lambda k: [f[k] for f in fields]
    o = lambda k: [x[k] for x in outputs]
    info = plan.solve(rho0, dt, g("us"), g("vs"), g("ws"), g("rho"), g("pn"), g("pnm1"), g("S"), o("p"), info)
    plan.correct(dt, g("us"), g("vs"), g("ws"), g("rho"), g("pn"), g("pnm1"), o("p"), g("S"), o("u"), o("v"),
                 o("w"), info)
    return outputs, info


def solve_noalloc(nx, ny, nz, fields: List[Dict], rho0, dt, outputs: List[Dict], info, lx=2 * np.pi, ly=2.0,
                  lz=2 * np.pi, precision=PPE_PREC_FP64, tol=1e-12, max_refine=1, ybc=PPE_YBC_WALLS, stream=None,
                  project=True):
    """ppe_solve_noalloc: a whole batch solved (and projected, with `project`)
    in the library's static device workspace, with no plan; `outputs` holds
    preallocated p (and u, v, w) tensors, `info` a preallocated record tensor.
    Returns the ppe_status_t code (PPE_ERR_NOMEM when the grid exceeds the
    static workspace) rather than raising, so callers can fall back."""
    import torch

    desc = make_desc(nx, ny, nz, lx, ly, lz, precision, tol, max_refine, len(fields), ybc, 0)
    dev = outputs[0]["p"].device
    shape_c, shape_v = (nz, ny, nx), (nz, ny + 1, nx)

    def chk(t, shape, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or tuple(t.shape) != shape \
                or t.device != dev or not t.is_contiguous():
            raise PPEError(f"{name}: expected contiguous float64 {shape} on {dev}")
        return t

    g = lambda k, shape: _ptrs([chk(f[k], shape, k) for f in fields])
    o = lambda k, shape: _ptrs([chk(x[k], shape, k) for x in outputs])
    if len(rho0) != len(fields) or len(dt) != len(fields) or len(outputs) != len(fields):
        raise PPEError("one rho0, dt and output record per instance")
    if info.numel() < 8 * len(fields) or info.dtype != torch.float64 or info.device != dev:
        raise PPEError("info: expected float64 records on the fields' device")
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    uvw = (o("u", shape_c), o("v", shape_v), o("w", shape_c)) if project else (None, None, None)
    lib = load()
    return int(lib.ppe_solve_noalloc(ctypes.byref(desc), ctypes.c_void_p(s.cuda_stream), _dbl(rho0), _dbl(dt),
                                     g("us", shape_c), g("vs", shape_v), g("ws", shape_c), g("rho", shape_c),
                                     g("pn", shape_c), g("pnm1", shape_c), g("S", shape_c), o("p", shape_c), *uvw,
                                     ctypes.c_void_p(info.data_ptr())))
