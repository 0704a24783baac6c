"""Turn rocprofv3 CSV output into the short summaries kept under ``profiles/``.

    python -m paper_2404_02950_amd.rocprof_summary stats  KERNEL_STATS_CSV  OUT_MD  --cmd "..."
    python -m paper_2404_02950_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV OUT_JSON OUT_MD \\
        --kernel SUBSTRING --n 512 --prec f64 --alg-bytes 64 --cmd-fetch "..." --cmd-write "..."

``stats`` tabulates a ``--kernel-trace --stats`` run (calls, mean duration, share).

``traffic`` takes one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of the same
program.  Both counters report KiB per dispatch.  Each is scaled by the factor that makes
the library's plain copy kernel ``k_xfer`` read back its known size (it reads a dense FP64
state, 4 components x cells x 8 B, and writes it into the boxes, 4 x cells x element
size, nothing else), so the figures are HBM bytes per launch; the factors are stored
with the result.  The JSON also
records the SHA-256 of the kernel sources, so a consumer can tell whether the figure
still describes the kernels it runs.
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics
import sys
from collections import defaultdict


def _per_kernel(path: str, counter: str):
    vals = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def _pick(vals, sub: str):
    names = [k for k in vals if sub in k]
    if len(names) != 1:
        raise SystemExit(f"expected one kernel matching {sub!r}, found {names}")
    return names[0], vals[names[0]]


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    lines = ["# rocprofv3 kernel statistics", "", f"Command: `{args.cmd}`", "",
             "| Kernel | Calls | Mean (us) | Min (us) | Max (us) | Share (%) |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"] if len(r["Name"]) < 110 else r["Name"][:107] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def traffic(args):
    from paper_2404_02950_amd.build_lib import KERNEL_SOURCES, kernel_family, kernel_source_sha
    fetch = _per_kernel(args.fetch, "FETCH_SIZE")
    write = _per_kernel(args.write, "WRITE_SIZE")
    esize = 8 if args.prec == "f64" else 4
    ref_read = 4 * args.n ** 3 * 8            # k_xfer: the dense FP64 state in ...
    ref_write = 4 * args.n ** 3 * esize       # ... and the boxed state out
    _, xf = _pick(fetch, "k_xfer")
    _, xw = _pick(write, "k_xfer")
    f_fac = ref_read / (statistics.mean(xf) * 1024)
    w_fac = ref_write / (statistics.mean(xw) * 1024)
    kname, kf = _pick(fetch, args.kernel)
    _, kw = _pick(write, args.kernel)
    fb = statistics.mean(kf) * 1024 * f_fac
    wb = statistics.mean(kw) * 1024 * w_fac
    alg = args.alg_bytes * args.n ** 3
    rec = {
        "kernel": kname,
        "workload": f"single-level periodic {args.n}^3, {args.prec}",
        "dispatches": len(kf),
        "fetch_kib_per_dispatch_raw": statistics.mean(kf),
        "write_kib_per_dispatch_raw": statistics.mean(kw),
        "calibration": {"reference_kernel": "k_xfer", "reference_read_bytes": ref_read,
                        "reference_write_bytes": ref_write,
                        "fetch_kib_raw": statistics.mean(xf), "write_kib_raw": statistics.mean(xw),
                        "fetch_factor": f_fac, "write_factor": w_fac},
        "hbm_read_bytes_per_launch": fb,
        "hbm_write_bytes_per_launch": wb,
        "hbm_bytes_per_launch": fb + wb,
        "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": (fb + wb) / alg,
        "kernel_source_sha256": kernel_source_sha(kernel_family(kname)),
        "kernel_sources": list(KERNEL_SOURCES[kernel_family(kname)]),
        "command_fetch": args.cmd_fetch,
        "command_write": args.cmd_write,
    }
    json.dump(rec, open(args.out_json, "w"), indent=1)
    md = [f"# HBM traffic of `{kname}`", "",
          f"Workload: {rec['workload']}; {len(kf)} dispatches.", "",
          f"FETCH_SIZE run: `{args.cmd_fetch}`", "", f"WRITE_SIZE run: `{args.cmd_write}`", "",
          "| | raw KiB/dispatch | factor | bytes/launch |", "|---|---|---|---|",
          f"| read | {statistics.mean(kf):.0f} | {f_fac:.3f} | {fb:.4g} |",
          f"| write | {statistics.mean(kw):.0f} | {w_fac:.3f} | {wb:.4g} |",
          f"| total | | | {fb + wb:.4g} |", "",
          f"Algorithmic bytes per launch: {alg:.4g} ({args.alg_bytes} B per cell); traffic / algorithmic = "
          f"{(fb + wb) / alg:.3f}.", "",
          f"Calibration: `k_xfer` reads {ref_read} B and writes {ref_write} B; the counters read back "
          f"{statistics.mean(xf):.0f} KiB (FETCH_SIZE) and {statistics.mean(xw):.0f} KiB (WRITE_SIZE) per "
          "dispatch.", ""]
    open(args.out_md, "w").write("\n".join(md))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("out_json")
    t.add_argument("out_md")
    t.add_argument("--kernel", required=True)
    t.add_argument("--n", type=int, required=True)
    t.add_argument("--prec", choices=("f64", "f32"), required=True)
    t.add_argument("--alg-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    args = ap.parse_args(argv)
    stats(args) if args.mode == "stats" else traffic(args)


if __name__ == "__main__":
    sys.exit(main())
