"""Benchmark of the split pressure-gradient projection step on one MI355X.

A step is one pass of the whole hot path -- ppe_solve + ppe_correct: right-hand
side (Eq. 29), real FFT in x, FFT in z, tridiagonal sweeps in y, inverse FFTs,
refinement sweeps when the precision is mixed, projection (Eq. 28) and its
continuity check -- over one synthetic two-phase sheet whose fields are
resident in HBM before the timed region starts.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

The roofline entry is measured live: a second pass over the same steps runs
with the library's per-kernel HIP-event timing (events on the plan's stream)
and the kernel with the largest total time is reported against the MI355X HBM
peak, with its algorithmic bytes per launch.  `traffic` is taken from the
committed rocprofv3 counter summary when it was collected from the current
kernel sources, else null.  The CPU baseline times the FP64 oracle (numpy /
scipy) on the same workload on the host.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# name -> (synth builder, precision, max_refine, description)
WORKLOADS = {
    "sheet_256x128x256_fp64": ("sheet_256", 0, 0,
                               "FP64 direct solve, 256x128x256 liquid sheet rho 640/100, Taylor-Green u* + 1% noise"),
    "sheet_512x256x512_mixed": ("sheet_512", 1, 1,
                                "FP32 spectra + FP64 refinement to 1e-12, 512x256x512 sheet rho 640/60"),
    "sheet_512x256x512_fp64": ("sheet_512", 0, 0, "FP64 direct solve, 512x256x512 sheet rho 640/60"),
    "sheet_32_fp64": ("sheet_32", 0, 0, "FP64 direct solve, 32^3 sheet rho 640/100"),
}

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, vendor figure


def source_hash() -> str:
    """Hash of the kernel sources (counter summaries are valid for one hash)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2103_01874_amd", "csrc", "*"))):
        if f.endswith((".hip", ".hpp", ".inc", ".cpp")):
            h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, nx: int, ny: int, nz: int, precision: int, mode_update: bool = False) -> float:
    """Bytes one launch must move for one instance (the compulsory traffic).

    N cells, Nv = nx (ny+1) nz v-faces, Ns = (nx/2+1) ny nz spectral values of
    cs bytes (16 FP64, 8 FP32)."""
    N = nx * ny * nz
    Nv = nx * (ny + 1) * nz
    Ns = (nx // 2 + 1) * ny * nz
    cs = 16 if precision == 0 else 8
    table = {
        "k_rhs": 8 * (6 * N + Nv) + 8 * N,           # u*, v*, w*, rho, p^n, p^{n-1}, S -> b
        "k_r2c": 8 * N + cs * Ns,                      # b (or r) -> half spectrum
        "k_fft_z_fwd": 2 * cs * Ns,
        "k_fft_z_inv": 2 * cs * Ns,
        "k_tri": 2 * cs * Ns,
        "k_c2r": cs * Ns + 8 * N + (8 * N if mode_update else 0),
        "k_resid": 3 * 8 * N,                          # b, p -> r
        "k_correct": 8 * (7 * N + Nv) + 8 * (2 * N + Nv),  # u*,v*,w*,rho,p^n,p^{n-1},p,S -> u,v,w
    }
    return float(table.get(kernel, 0.0))


def cpu_baseline(pr, budget_s: float = 12.0):
    """The FP64 oracle on the same workload, timed on the host."""
    import oracle as O

    workers = max(1, min(16, os.cpu_count() or 1))
    g = O.Grid(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz)
    steps = 0
    t0 = time.perf_counter()
    while True:
        O.ppe_step(g, pr.rho0, pr.dt, *pr.fields(), workers=workers)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 20:
            break
    return {"value": pr.npts * steps / el, "unit": "points/s", "cores": workers, "kind": "oracle",
            "sample": f"{steps} full step(s) of the same workload ({pr.nx}x{pr.ny}x{pr.nz}) in {el:.1f} s; "
                      f"scipy.fft with {workers} workers, numpy elementwise work on one thread"}


def counter_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from profiles/counters_<workload>.json,
    if those counters were taken from the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sheet_256x128x256_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed roofline pass")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run a plain device copy of this many bytes 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: a projection step of one grid runs on one MI355X here; "
                                   "sharding across GPUs is described in the design notes, not built",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2103_01874_amd import binding, synth

    builder, precision, max_refine, desc = WORKLOADS[args.workload]
    pr = getattr(synth, builder)()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        plan = binding.Plan(pr.nx, pr.ny, pr.nz, pr.lx, pr.ly, pr.lz, precision=precision, tol=1e-12,
                            max_refine=max_refine, stream=stream)
        fields = binding.to_device(pr, dev)
        outs = {"p": torch.empty_like(fields["rho"]), "u": torch.empty_like(fields["us"]),
                "v": torch.empty_like(fields["vs"]), "w": torch.empty_like(fields["ws"])}
        info = plan.new_info()
    torch.cuda.synchronize()
    g = lambda k: [fields[k]]
    o = lambda k: [outs[k]]

    def one_step():
        plan.solve([pr.rho0], [pr.dt], g("us"), g("vs"), g("ws"), g("rho"), g("pn"), g("pnm1"), g("S"), o("p"),
                   info)
        plan.correct([pr.dt], g("us"), g("vs"), g("ws"), g("rho"), g("pn"), g("pnm1"), o("p"), g("S"), o("u"),
                     o("v"), o("w"), info)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        one_step()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps
    rec = binding.decode_info(info)[0]
    npts = pr.npts
    print(f"# timed {args.steps} steps: {ms:.4f} ms/step, eps_div={rec['res_rel']:.3e} iters={rec['iters']}",
          file=sys.stderr, flush=True)

    roofline = None
    kernels = None
    if not args.no_profile:
        plan.profile(True)
        for _ in range(args.steps):
            one_step()
        kernels = plan.profile_read()
        plan.profile(False)
        dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
        kname, kv = dom
        per_launch = algorithmic_bytes(kname, pr.nx, pr.ny, pr.nz, precision,
                                       mode_update=(kname == "k_c2r" and max_refine > 0))
        if kname == "k_c2r" and max_refine > 0:
            # half of the launches update p (read + write), half write it: average
            per_launch = 0.5 * (algorithmic_bytes(kname, pr.nx, pr.ny, pr.nz, precision, False)
                                + algorithmic_bytes(kname, pr.nx, pr.ny, pr.nz, precision, True))
        achieved = per_launch / (kv["avg_us"] * 1e-6) / 1e9
        traffic = counter_traffic(args.workload, kname)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": kname,
                    "avg_launch_us": kv["avg_us"], "bytes_per_launch": per_launch}
        kernels = {k: round(v["avg_us"], 2) for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ms"])}

    if args.copy_bytes > 0:
        n = args.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr)

    out = {
        "metric": "PPE grid points/s (projection step: solve + correction) at 1e-12 relative divergence residual",
        "value": npts / (ms * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "grid": [pr.nx, pr.ny, pr.nz],
                   "points": npts, "precision": "fp64" if precision == 0 else "mixed",
                   "max_refine": max_refine, "parallelism": "single GPU"},
        "result": {"eps_div": rec["res_rel"], "iters": rec["iters"], "status": rec["status"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_avg_us": kernels,
        "wall_s": wall,
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
