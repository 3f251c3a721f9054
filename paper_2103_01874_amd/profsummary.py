"""Summaries of rocprofv3 databases (rocpd SQLite) for the profiles/ folder.

  python -m paper_2103_01874_amd.profsummary trace  DB  --cmd "..."  > profiles/<name>.txt
  python -m paper_2103_01874_amd.profsummary pmc DB... --title T --cmd "..." > profiles/<name>.txt
  python -m paper_2103_01874_amd.profsummary counters --fetch DB1 --write DB2 --workload W \
         --copy-bytes B --cmd-fetch "..." --cmd-write "..." --out profiles/counters_W.json

`trace` prints per-kernel launch counts and average durations from a
--kernel-trace run.  `pmc` prints the mean per dispatch of every counter of
one or more --pmc runs, per kernel family.  `counters` turns FETCH_SIZE and WRITE_SIZE (KiB per
dispatch, from two separate --pmc runs) into HBM bytes per launch, each scaled
by what the same counter reads for the plain device copy of known size that
the benchmark runs with --copy-bytes (a 1 GiB read + 1 GiB write elementwise
kernel).
"""

from __future__ import annotations

import argparse
import collections
import json
import os
import re
import sqlite3
import sys


def _short(name: str) -> str:
    n = re.sub(r"\(.*", "", name).replace("void ", "").replace("ppe::", "")
    return n.strip()


def family(name: str) -> str:
    """Kernel family as the library's event timing names it."""
    n = _short(name)
    if n.startswith("k_fft_z"):
        # k_fft_z<TS, E, DIR[, plan]>: DIR = -1 forward, 1 inverse
        return "k_fft_z_fwd" if re.match(r"k_fft_z<[^,]+, *\d+, *-1\b", n) else "k_fft_z_inv"
    if n.startswith("k_predict_march_uvw"):
        return "k_predict"  # the three components in one launch
    m = re.match(r"k_predict(?:_tile|_march)?<(\d)", n)
    if m:
        # k_predict*<COMP, ...>: COMP 0 and 3 u, 1 v, 2 w
        return "k_predict_" + "uvwu"[int(m.group(1))]
    return re.sub(r"<.*", "", n)


def trace_stats(db_path: str):
    db = sqlite3.connect(db_path)
    agg = collections.OrderedDict()
    for name, start, end in db.execute("select name, start, end from kernels"):
        a = agg.setdefault(_short(name), [0, 0.0])
        a[0] += 1
        a[1] += (end - start) * 1e-3
    return agg


def cmd_trace(args):
    agg = trace_stats(args.db)
    tot = sum(v[1] for v in agg.values())
    print(f"# rocprofv3 kernel trace: {os.path.basename(os.path.dirname(os.path.abspath(args.db)))}")
    print(f"# command: {args.cmd}")
    print(f"# {'kernel':<48} {'launches':>8} {'avg_us':>10} {'total_us':>11} {'share':>6}")
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"  {k[:48]:<48} {n:8d} {t / n:10.2f} {t:11.1f} {100 * t / tot:5.1f}%")


def _counter(db_path: str, counter: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                      "where counter_name = ? order by dispatch_id", (counter,)).fetchall()
    return rows


def cmd_counters(args):
    out = {"workload": args.workload, "source_hash": args.source_hash, "copy_bytes": args.copy_bytes,
           "commands": {"fetch": args.cmd_fetch, "write": args.cmd_write}, "kernels": {}}
    per = {}
    factors = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        rows = _counter(path, counter)
        # calibration: the elementwise copy kernel over copy_bytes (largest grid of that family)
        cal = [v for _, name, gs, v in rows if "elementwise" in name and gs * 32 >= args.copy_bytes // 8]
        cal = cal[-3:]
        if not cal:
            raise SystemExit(f"no calibration copy found in {path}")
        kib = sum(cal) / len(cal)
        factors[counter] = args.copy_bytes / (kib * 1024.0)
        for _, name, gs, v in rows:
            fam = family(name)
            if not fam.startswith("k_"):
                continue
            per.setdefault(fam, {}).setdefault(counter, []).append(v)
    out["factor"] = factors
    for fam, d in sorted(per.items()):
        rec = {}
        tot = 0.0
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = d.get(counter, [])
            if not vals:
                continue
            kib = sum(vals) / len(vals)
            b = kib * 1024.0 * factors[counter]
            rec[counter.lower() + "_kib_per_dispatch"] = kib
            rec[counter.split("_")[0].lower() + "_bytes_per_launch"] = b
            tot += b
        rec["hbm_bytes_per_launch"] = tot
        out["kernels"][fam] = rec
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def cmd_pmc(args):
    """Mean value per dispatch of every counter in the given --pmc databases,
    per kernel family, with per-wave figures where SQ_WAVES was collected
    and byte figures for the TCC request counters (every request of a
    TCC_EA0_RDREQ_128B count is 128 bytes, TCC_EA0_WRREQ_64B 64 bytes)."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in args.db:
        db = sqlite3.connect(path)
        for name, cn, v in db.execute("select kernel_name, counter_name, value from counters_collection"):
            fam = family(name)
            if fam.startswith("k_"):
                acc[fam][cn].append(v)
    print(f"# rocprofv3 counters, mean per dispatch: {args.title}")
    for cmd in args.cmd:
        print(f"# command: {cmd}")
    for fam in sorted(acc):
        d = {cn: sum(v) / len(v) for cn, v in acc[fam].items()}
        waves = d.get("SQ_WAVES")
        parts = []
        for cn in sorted(d):
            x = d[cn]
            if waves and cn.startswith("SQ_INSTS"):
                parts.append(f"{cn}/wave={x / waves:.1f}")
            elif cn == "TCC_EA0_RDREQ_128B":
                parts.append(f"read_bytes={x * 128 / 1e6:.1f}MB")
            elif cn == "TCC_EA0_WRREQ_64B":
                parts.append(f"write_bytes={x * 64 / 1e6:.1f}MB")
            else:
                parts.append(f"{cn}={x:.6g}")
        if waves and "SQ_WAIT_INST_ANY" in d and "SQ_WAVE_CYCLES" in d:
            parts.append(f"wait_inst_frac={d['SQ_WAIT_INST_ANY'] / d['SQ_WAVE_CYCLES']:.3f}")
        print(f"  {fam}: " + " ".join(parts))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--source-hash", required=True)
    c.add_argument("--cmd-fetch", required=True)
    c.add_argument("--cmd-write", required=True)
    c.add_argument("--out", required=True)
    m = sub.add_parser("pmc")
    m.add_argument("db", nargs="+")
    m.add_argument("--title", required=True)
    m.add_argument("--cmd", action="append", default=[])
    args = ap.parse_args(argv)
    if args.cmd_name == "trace":
        cmd_trace(args)
    elif args.cmd_name == "pmc":
        cmd_pmc(args)
    else:
        cmd_counters(args)


if __name__ == "__main__":
    main(sys.argv[1:])
