"""Turn rocprofv3 CSV output into the short summaries kept under ``profiles/``.

    python -m paper_2404_02950_amd.rocprof_summary stats  KERNEL_STATS_CSV  OUT_MD  --cmd "..."
    python -m paper_2404_02950_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV OUT_JSON OUT_MD \\
        --kernel SUBSTRING --n 512 --prec f64 --alg-bytes 64 --cmd-fetch "..." --cmd-write "..."

``stats`` tabulates a ``--kernel-trace --stats`` run (calls, mean duration, share).

``amr-traffic`` sums FETCH_SIZE / WRITE_SIZE runs of an AMR workload by kernel class and
sets the per-stage kernels against their algorithmic bytes.

``counters`` tabulates one ``--pmc`` run of SQ counters for one kernel (mean per dispatch,
wait and activity ratios):

    python -m paper_2404_02950_amd.rocprof_summary counters COUNTER_CSV OUT_MD \\
        --kernel SUBSTRING --workload "..." --cmd "..."

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
    if args.trace:
        # the launches a timed region covers are the last ones: their mean, for comparison
        # with the figure the program measured itself
        durs = [(int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
                for r in csv.DictReader(open(args.trace)) if args.timed_kernel in r["Kernel_Name"]]
        durs = [d for _, d in sorted(durs)][-args.timed_last:]
        lines += ["", f"Mean over the last {len(durs)} launches of `{args.timed_kernel}` (the timed steps; "
                      f"kernel trace): {statistics.mean(durs):.1f} us (min {min(durs):.1f}, max {max(durs):.1f})."]
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


def counters(args):
    """Mean per dispatch of every counter of one --pmc run for the kernel matching
    ``--kernel``, with the wait and activity ratios the SQ counters give."""
    rows = list(csv.DictReader(open(args.csv)))
    names = sorted({r["Kernel_Name"] for r in rows if args.kernel in r["Kernel_Name"]})
    if len(names) != 1:
        raise SystemExit(f"expected one kernel matching {args.kernel!r}, found {names}")
    kname = names[0]
    per = defaultdict(lambda: defaultdict(float))
    for r in rows:
        if r["Kernel_Name"] == kname:
            per[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    mean = {c: statistics.mean(v.values()) for c, v in per.items()}
    nd = len(next(iter(per.values())))
    lines = [f"# SQ counters of `{kname}`", "", f"Workload: {args.workload}; {nd} dispatches (mean per dispatch).",
             "", f"Command: `{args.cmd}`", "", "| Counter | Mean per dispatch |", "|---|---|"]
    lines += [f"| {c} | {v:.4g} |" for c, v in sorted(mean.items())]
    ratios = []
    cyc = mean.get("SQ_WAVE_CYCLES")
    if cyc:
        for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS"):
            if c in mean:
                ratios.append(f"{c} / SQ_WAVE_CYCLES = {mean[c] / cyc:.2f}")
    if "SQ_INSTS_VALU" in mean and mean.get("SQ_WAVES"):
        ratios.append(f"VALU instructions per wave = {mean['SQ_INSTS_VALU'] / mean['SQ_WAVES']:.0f}")
    if ratios:
        lines += ["", "Ratios: " + "; ".join(ratios) + "."]
    open(args.out, "w").write("\n".join(lines) + "\n")


def amr_traffic(args):
    """HBM bytes per kernel class of an AMR run (one FETCH_SIZE and one WRITE_SIZE run,
    summed over all dispatches, scaled by the k_xfer calibration as in ``traffic``), with
    the algorithmic bytes of the per-stage RK4 kernels: the refined levels' cells per
    stage class are (cell-stage updates - 4 x level-0 cells x coarse steps) / 4, at 96 /
    160 / 160 / 96 B per cell (FP64) for stages 1-4."""
    def load(path, counter):
        tot, n = defaultdict(float), defaultdict(int)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                tot[r["Kernel_Name"]] += float(r["Counter_Value"])
                n[r["Kernel_Name"]] += 1
        return tot, n
    fetch, nf = load(args.fetch, "FETCH_SIZE")
    write, nw = load(args.write, "WRITE_SIZE")
    xk = [k for k in fetch if "k_xfer" in k]
    if len(xk) != 1:
        raise SystemExit("expected one k_xfer dispatch kernel for the calibration")
    ref = 4 * args.n0 ** 3 * 8
    ff = ref / (fetch[xk[0]] / nf[xk[0]] * 1024)
    fw = ref / (write[xk[0]] / nw[xk[0]] * 1024)
    ref_cells = (args.cell_stage_updates - 4 * args.n0 ** 3 * args.coarse_steps) / 4
    alg = (96, 160, 160, 96)

    def bytes_of(sel):
        rb = sum(fetch[k] for k in fetch if sel(k)) * 1024 * ff
        wb = sum(write[k] for k in write if sel(k)) * 1024 * fw
        return rb, wb
    lines = ["# HBM traffic of an AMR run by kernel class", "", f"Workload: {args.workload}.", "",
             f"FETCH_SIZE run: `{args.cmd_fetch}`", "", f"WRITE_SIZE run: `{args.cmd_write}`", "",
             f"Calibration (k_xfer, {ref} B read and written): factors {ff:.3f} (read), {fw:.3f} (write). "
             f"Refined-level cells per stage class: {ref_cells:.4g}.", "",
             "| Kernels | Dispatches | HBM read GB | HBM write GB | Algorithmic GB | Traffic / algorithmic |",
             "|---|---|---|---|---|---|"]
    for s in range(4):
        sel = (lambda k, s=s: k.startswith((f"void k_stage<double, {s}, ", f"void k_stage_lds<double, {s}, ")))
        rb, wb = bytes_of(sel)
        nd = sum(nf[k] for k in fetch if sel(k))
        a = ref_cells * alg[s]
        lines.append(f"| RK4 stage {s + 1} (`k_stage`, `k_stage_lds`) | {nd} | {rb / 1e9:.1f} | {wb / 1e9:.1f} | "
                     f"{a / 1e9:.1f} | {(rb + wb) / a:.2f} |")
    for label, sub in (("coarse/fine interpolation", "k_ghost_interp"), ("same-level copy", "k_ghost_copy"),
                       ("average down", "k_avgdown"), ("fused level-0 step", "k_fused_step"), ("tagging", "k_tag")):
        rb, wb = bytes_of(lambda k, sub=sub: sub in k)
        nd = sum(nf[k] for k in fetch if sub in k)
        lines.append(f"| {label} (`{sub}`) | {nd} | {rb / 1e9:.1f} | {wb / 1e9:.1f} | | |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--trace", help="kernel trace CSV of the same run")
    s.add_argument("--timed-kernel", default="k_fused_step")
    s.add_argument("--timed-last", type=int, default=20)
    q = sub.add_parser("counters")
    q.add_argument("csv")
    q.add_argument("out")
    q.add_argument("--kernel", required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--cmd", required=True)
    a = sub.add_parser("amr-traffic")
    a.add_argument("fetch")
    a.add_argument("write")
    a.add_argument("out")
    a.add_argument("--n0", type=int, required=True)
    a.add_argument("--coarse-steps", type=int, required=True)
    a.add_argument("--cell-stage-updates", type=float, required=True)
    a.add_argument("--workload", required=True)
    a.add_argument("--cmd-fetch", required=True)
    a.add_argument("--cmd-write", required=True)
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
    {"stats": stats, "counters": counters, "traffic": traffic, "amr-traffic": amr_traffic}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
