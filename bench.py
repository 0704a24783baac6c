#!/usr/bin/env python3
"""Throughput of the per-level time step on one MI355X.

Workload (default): one periodic level of 512^3 cells (L = 512, dx = 1), the axion-string
EOM with lambda = 1, alpha = 2, beta = 2, classic RK4 with dt = dx/4 from eta = 0.1, the
seeded Gaussian-random-field initial state; FP64 (``--prec f64``) or FP32 storage with
FP64 accumulation (``--prec f32``).  A step is one sh_advance_level: by default one kernel
that computes all four RK stages of the step, then one refill of the level's 4-deep
periodic ghost shell (with ``SHAMR_TUNE=fuse=0``: four stage kernels with a ghost copy
between them).  ``--integrator 10`` (or 3) runs SSPRK3 instead: by default one kernel for
its three stages (with ``fuse=0``: three stage kernels with a ghost copy between them).

Prints one JSON line: cell-updates/s per RK stage (whole job), the roofline of the
dominant kernel from HIP events recorded around each of its launches inside the timed
region (on the level's stream), and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
# algorithmic bytes per cell of the fused stage kernel, stages 1-4 (each array element
# moved once: 12/20/20/12 values; FP32-mixed keeps the accumulator in FP64)
STAGE_BYTES = {"f64": (96, 160, 160, 96), "f32": (64, 112, 112, 64)}
# the fused four-stage step reads U_n and writes U_{n+1}: 8 values per cell
FUSED_BYTES = {"f64": 64, "f32": 32}
# SSPRK3 stages 1-3: X in, Y out (8 values); X and U_n in, Y out (12 values) twice
SSP_STAGE_BYTES = {"f64": (64, 96, 96), "f32": (32, 48, 48)}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_from_profiles(prec: str, n: int, kname: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"{kname}_{n}cubed_{prec}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    from paper_2404_02950_amd.build_lib import kernel_family, kernel_source_sha
    if rec.get("kernel_source_sha256") != kernel_source_sha(kernel_family(kname)):
        return None
    return rec.get("hbm_bytes_per_launch")


# the whole lattice the slab workers step: set before the pool forks, read by the workers
_SLAB_STATE = {}


def _slab_step(task):
    """One oracle step of z-planes [z0, z1) of the lattice in _SLAB_STATE: the slab is cut
    out with `halo` planes on either side (periodically) and stepped by the oracle as a
    periodic lattice of its own; the wrap corrupts at most `halo` planes at each end, so
    the planes in between are the whole-lattice step's.  Returns (z0, interior or its
    sum, seconds)."""
    z0, z1, halo, kw, keep = task
    import numpy as np
    from oracle.level import rk4_step, ssprk3_step
    U = _SLAB_STATE["U"]
    n = U.shape[1]
    t0 = time.perf_counter()
    X = U[:, np.arange(z0 - halo, z1 + halo) % n]
    step = rk4_step if kw["integrator"] == 4 else ssprk3_step
    Y = step(X, kw["eta"], kw["dt"], kw["inv_dx2"], kw["alpha"], kw["lam"], kw["beta"], order=kw["order"],
             ko=kw["ko"])[:, halo:halo + (z1 - z0)]
    dt = time.perf_counter() - t0
    return z0, (Y.copy() if keep else float(Y.sum())), dt


def oracle_step_slabs(U, nslabs: int, workers: int, integrator: int = 4, order: int = 1, ko_order: int = 0,
                      ko_eps: float = 0.0, keep: bool = False, first_only: bool = False):
    """One oracle step (eta 0.1, dt 0.25, dx 1, alpha 2, lambda 1, beta 2) of the periodic
    lattice U split into nslabs z-slabs run by `workers` forked processes (1: in this
    process).  The oracle code is unchanged: each slab carries enough extra planes
    (stages x stencil reach) that its own periodic wrap never reaches the planes it
    keeps.  first_only runs the first slab alone.  Returns (seconds, the stepped state if
    keep else the per-slab sums)."""
    import numpy as np
    from oracle.level import ko_coef
    n = U.shape[1]
    nst = 4 if integrator == 4 else 3
    halo = nst * max(order, ko_order)
    if n % nslabs:
        raise ValueError("the lattice must split into whole slabs")
    kw = {"integrator": integrator, "eta": 0.1, "dt": 0.25, "inv_dx2": 1.0, "alpha": 2.0, "lam": 1.0, "beta": 2,
          "order": order, "ko": (ko_order, ko_coef(ko_order, ko_eps, 1.0)) if ko_order else None}
    w = n // nslabs
    tasks = [(i * w, (i + 1) * w, halo, kw, keep) for i in range(1 if first_only else nslabs)]
    _SLAB_STATE["U"] = U
    try:
        if workers <= 1:
            t0 = time.perf_counter()
            res = [_slab_step(t) for t in tasks]
            dt = time.perf_counter() - t0
        else:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                pool.map(len, [()] * workers)  # workers up before the clock starts
                t0 = time.perf_counter()
                res = pool.map(_slab_step, tasks, chunksize=1)
                dt = time.perf_counter() - t0
    finally:
        _SLAB_STATE.clear()
    res.sort(key=lambda r: r[0])
    if keep:
        return dt, np.concatenate([r[1] for r in res], axis=1)
    return dt, [r[1] for r in res]


def host_cpu():
    """(cores this process may run on, capped at the 16 a one-GPU share holds; CPU model)."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return ncpu, min(ncpu, 16), model


def cpu_baseline(U0, n: int, integrator: int = 4, order: int = 1, ko_order: int = 0, ko_eps: float = 0.0):
    """The oracle on this host's cores (run before the GPU is touched, so the forked
    workers hold no device state): one full step of the n^3 lattice as z-slabs over all
    usable cores, and the first of 8 such slabs alone on one core."""
    nproc, workers, model = host_cpu()
    nst, name = (4, "RK4") if integrator == 4 else (3, "SSPRK3")
    nslabs = workers
    while n % nslabs:
        nslabs += 1
    t_all, _ = oracle_step_slabs(U0, nslabs, workers, integrator, order, ko_order, ko_eps)
    t_one, _ = oracle_step_slabs(U0, 8, 1, integrator, order, ko_order, ko_eps, first_only=True)
    return {"value": nst * n ** 3 / t_all, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "nproc": nproc, "cpu_model": model,
            "value_1core": nst * (n // 8) * n * n / t_one,
            "sample": f"one {name} step ({nst} stages) of the {n}^3 FP64 lattice: numpy oracle on {nslabs} z-slabs "
                      f"in {workers} processes, {t_all:.1f} s wall; one core: one slab of {n // 8} planes, "
                      f"{t_one:.1f} s"}


def stream_bandwidth(stream, nbytes: int = 2 ** 32, reps: int = 10):
    """GB/s of the library's streaming probes over nbytes buffers (well beyond the 256 MB
    last-level cache), events on stream: {read, write, copy (read + write counted)}."""
    import torch
    from paper_2404_02950_amd import shamr
    out = {}
    with torch.cuda.stream(stream):
        a = torch.zeros(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for kind, name, moved in ((1, "write", nbytes), (0, "read", nbytes), (2, "copy", 2 * nbytes)):
            for _ in range(3):
                shamr.stream_probe(kind, a, b, nbytes, stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                shamr.stream_probe(kind, a, b, nbytes, stream)
            e1.record(stream)
            e1.synchronize()
            out[name] = moved * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    return out


DIVERGED_PSI = 10.0  # |psi| of the FP64 run beyond which the field counts as diverged


def fp32_error_series(U0, n: int, steps: int, stream, args, beta: int = 2):
    """FP32 storage against FP64 from the same initial state, after every step: the
    largest |psi_32 - psi_64| and |Pi_32 - Pi_64| over all cells, with max |psi_64| for
    scale.  The FP64 run is the library's FP64 path, which equals the FP64 oracle bit for
    bit (the sampled full-size parity tests); values are compared on the device.  With
    the paper's beta = 2 at dt = dx/4 the radial mode goes unstable within the run; the
    divergence onset is the first step at which max |psi_64| exceeds DIVERGED_PSI (the
    field is of order 1 before it) or turns non-finite."""
    import math
    import torch
    from paper_2404_02950_amd import shamr
    hs = {}
    for prec in (shamr.SH_F64, shamr.SH_F32):
        h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=0, prec=prec, stream=stream,
                            integrator=args.integrator, lap_order=args.lap_order, ko_order=args.ko_order,
                            ko_eps=args.ko_eps)
        h.set_layout(0, [(0, 0, 0, n - 1, n - 1, n - 1)])
        h.write_dense(0, U0)
        h.fill_ghosts(0)
        hs[prec] = h
    cells = n ** 3
    e_psi, e_pi, m_psi, first_bad = [], [], [], None
    log(f"FP32 vs FP64 error series over {steps} steps (beta {beta})")
    for k in range(steps):
        for h in hs.values():
            h.advance(0)
        with torch.cuda.stream(stream):
            a = hs[shamr.SH_F32].read_device(0).view(4, cells)
            b = hs[shamr.SH_F64].read_device(0).view(4, cells)
            if first_bad is None and not bool(torch.isfinite(b).all()):
                first_bad = k + 1
            d = (a - b).abs_()
            vals = torch.stack([d[:2].max(), d[2:].max(), b[:2].abs().max()]).cpu().tolist()
        del a, b, d
        for lst, v in zip((e_psi, e_pi, m_psi), vals):
            lst.append(float(f"{v:.4g}") if math.isfinite(v) else None)
    for h in hs.values():
        h.close()
    torch.cuda.empty_cache()
    onset = next((k + 1 for k, m in enumerate(m_psi) if m is None or m > DIVERGED_PSI), None)
    before = [k for k in range(steps) if onset is None or k + 1 < onset]
    return {"reference": "FP64 run of the same lattice on the GPU (equal to the FP64 oracle bit for bit)",
            "beta": beta, "steps": steps, "max_abs_err_psi": e_psi, "max_abs_err_pi": e_pi,
            "max_abs_psi_fp64": m_psi, "first_nonfinite_step_fp64": first_bad,
            "divergence_onset_step": onset, "divergence_rule": f"max |psi_64| > {DIVERGED_PSI} or non-finite",
            "max_abs_err_psi_before_onset": max((e_psi[k] for k in before if e_psi[k] is not None), default=None),
            "max_abs_err_pi_before_onset": max((e_pi[k] for k in before if e_pi[k] is not None), default=None)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--prec", choices=("f64", "f32"), default="f64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-steps", type=int, default=200,
                    help="--prec f32: steps of the FP32-vs-FP64 error series (0: none)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (calibrates rocprofv3 byte counters)")
    ap.add_argument("--workload", choices=("single", "amr256", "amr512", "serve"), default="single",
                    help="single: the 512^3 level step (default); amr256: 256^3 + 3 levels, 8 string loops, "
                         "50 coarse steps; amr512: 512^3 + 2 levels, 16 loops, FP64 vs FP32, 20 coarse steps; "
                         "serve: 256 Poisson-arriving ensemble jobs")
    ap.add_argument("--integrator", type=int, default=4, choices=(3, 4, 10),
                    help="4: classic RK4 (default); 3 or 10: SSPRK3")
    ap.add_argument("--lap-order", type=int, default=1, choices=(1, 2, 3),
                    help="Laplacian order: 1 = 7-point (default), 2 = 13-point, 3 = 19-point (per-stage kernels)")
    ap.add_argument("--ko-order", type=int, default=0, choices=(0, 2, 3),
                    help="Kreiss-Oliger dissipation order (0 = off; per-stage wave-row kernels)")
    ap.add_argument("--ko-eps", type=float, default=0.01, help="Kreiss-Oliger dissipation strength")
    ap.add_argument("--regrid", choices=("global", "local"), default="global",
                    help="AMR workloads: global regrids, or local regrids with a global one when due")
    ap.add_argument("--interp", type=int, default=1, choices=(1, 4),
                    help="AMR workloads: ghost/new-cell interpolation, 1 = linear, 4 = quartic conservative")
    ap.add_argument("--beta", type=int, default=2, help="potential exponent (2: the paper's EOM; 0: stable companion)")
    ap.add_argument("--coarse-steps", type=int, default=None)
    ap.add_argument("--tag-mode", type=int, default=1, choices=(1, 2, 3),
                    help="amr256: refine by plaquette winding (1), truncation error estimate (2) or either (3)")
    ap.add_argument("--te-crit", type=float, default=1e-2, help="amr256: truncation error threshold")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="single workload: record this many level steps as one HIP graph and time its "
                         "replays (per-kernel timing and the roofline are then not collected)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding a level over several GPUs "
              "is described but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_02950_amd import shamr
    from synth import random_state

    n, K, W = args.n, args.steps, args.warmup
    cpu = None
    if args.workload == "single":
        log(f"initial state {n}^3 (seed {args.seed})")
        U0 = random_state(n, float(n), args.seed)
        if not args.no_cpu_baseline and args.prec == "f64":
            # before anything touches the GPU: the slab workers are forked from this process
            log("cpu baseline (oracle over the host cores)")
            cpu = cpu_baseline(U0, n, args.integrator, args.lap_order, args.ko_order, args.ko_eps)
            log(f"cpu baseline {cpu['sample']}")
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload in ("amr256", "amr512"):
        return bench_amr(args)
    if args.workload == "serve":
        from paper_2404_02950_amd.serve import bench_serving
        print(json.dumps(bench_serving(log=log)), flush=True)
        return
    prec = shamr.SH_F64 if args.prec == "f64" else shamr.SH_F32
    stream = torch.cuda.Stream()
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 2, max_level=0, prec=prec, stream=stream,
                        integrator=args.integrator, lap_order=args.lap_order, ko_order=args.ko_order,
                        ko_eps=args.ko_eps)
    nst = 4 if args.integrator == 4 else 3
    h.set_layout(0, [(0, 0, 0, n - 1, n - 1, n - 1)])
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    h.sync()
    log(f"warmup {W} steps")
    for _ in range(W):
        h.advance(0)
    h.sync()
    torch.cuda.synchronize()
    graph = None
    G = args.graph_steps
    if G > 1:
        if K % G:
            print("--steps must be a multiple of --graph-steps", file=sys.stderr)
            sys.exit(2)
        with h.capture() as c:
            for _ in range(G):
                h.advance(0)
        graph = c.graph
    log(f"timing {K} steps" + (f" as {K // G} replays of a {G}-step graph" if graph else ""))
    h.profile(graph is None)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(h.stream)
    if graph is not None:
        for _ in range(K // G):
            graph.launch()
    else:
        for _ in range(K):
            h.advance(0)
    e1.record(h.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    prof = h.profile_read()
    h.profile(False)
    e, bad = h.energy()
    cells = n ** 3
    value = cells * nst * K / (ms / 1e3)
    sb = STAGE_BYTES[args.prec] if nst == 4 else SSP_STAGE_BYTES[args.prec]
    roofline = None
    if prof["fused_step"][1]:
        kname = "fused_rk4_step" if nst == 4 else "fused_ssprk3_step"
        k_ms, k_n = prof["fused_step"]
        k_bytes = FUSED_BYTES[args.prec] * cells * k_n
    else:
        kname = (("rk4_stage" if nst == 4 else "ssprk3_stage") + ("" if args.lap_order == 1 else f"_lap{args.lap_order}")
                 + ("" if args.ko_order == 0 else f"_ko{args.ko_order}"))
        k_ms = sum(prof[f"stage{s + 1}"][0] for s in range(nst))
        k_n = sum(prof[f"stage{s + 1}"][1] for s in range(nst))
        k_bytes = sum(sb[s] * cells * prof[f"stage{s + 1}"][1] for s in range(nst))
    if k_n:  # (not collected for graph replays)
        achieved = k_bytes / (k_ms / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(args.prec, n, kname)}
        log(f"{kname} kernel {k_ms / k_n:.3f} ms/launch, {achieved:.0f} GB/s algorithmic")
    log(f"{ms / K:.3f} ms/step (event), wall {wall / K * 1e3:.3f} ms/step; energy {e[3]:.6g}, "
        f"nonfinite cells {bad}")
    out = {
        "metric": "cell-updates/s per RK stage",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"single-level periodic {n}^3, {'RK4' if nst == 4 else 'SSPRK3'} + "
                               f"{ {1: 7, 2: 13, 3: 19}[args.lap_order]}-point Laplacian, "
                               + (f"Kreiss-Oliger order {args.ko_order} (eps {args.ko_eps}), " if args.ko_order else "")
                               + ('FP64' if args.prec == 'f64' else 'FP32 storage / FP64 accumulation'),
                   "lattice": n, "dx": 1.0, "dt": 0.25, "eta0": 0.1, "lambda": 1.0, "seed": args.seed,
                   "integrator": args.integrator, "lap_order": args.lap_order, "ko_order": args.ko_order,
                   "graph_steps": G if graph is not None else None},
        "roofline": roofline,
        # a rate ratio, not a roofline: this cell-update rate over the most that a kernel
        # running one RK stage per pass could reach at the HBM peak (it must move the
        # mean per-stage bytes below for every cell-stage)
        "vs_per_stage_peak_rate": {"bytes_per_cell_stage": sum(sb) / nst,
                                   "per_stage_peak_rate": HBM_PEAK_GBS * 1e9 / (sum(sb) / nst),
                                   "ratio": value / (HBM_PEAK_GBS * 1e9 / (sum(sb) / nst))},
        "cell_steps_per_s": value / nst,
        "kernel_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items() if v[1]},
        "wall_ms_per_step": wall / K * 1e3,
        "nonfinite_cells_at_end": bad,
    }
    out["cpu_baseline"] = cpu
    if graph is not None:
        graph.close()
    h.close()
    if out["roofline"] is not None:
        # achievable HBM bandwidth on this machine: the library's read, write and copy probes
        # over 4 GiB buffers, timed the same way (events on the same stream), beside the
        # nominal peak; the ceiling is the best of the three
        bw = stream_bandwidth(stream)
        ceil = max(bw.values())
        out["roofline"]["stream_GBs"] = bw
        out["roofline"]["ceiling_GBs"] = ceil
        out["roofline"]["frac_of_ceiling"] = out["roofline"]["achieved"] / ceil
        log("streaming probes " + ", ".join(f"{k} {v:.0f} GB/s" for k, v in bw.items()))
    if args.prec == "f32" and args.error_steps > 0:
        out["fp32_error_vs_fp64"] = fp32_error_series(U0, n, args.error_steps, stream, args)
        # the stable companion: the same run with beta = 0 (no growing radial mode)
        out["fp32_error_vs_fp64_beta0"] = fp32_error_series(U0, n, args.error_steps, stream, args, beta=0)
    if args.calib_copy:
        a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        s = a.sum()
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * a.numel() * 8
        out["calib_sum_read_bytes"] = a.numel() * 8
        del s
        del a, b
    print(json.dumps(out), flush=True)


def bench_amr(args):
    """AMR hierarchies seeded with string loops (coarse dx = 1, dt_0 = 1/4, eta0 = 0.1)."""
    from paper_2404_02950_amd import shamr, workloads
    from synth import string_loop_state
    if args.workload == "amr256":
        n0, levels, loops, steps = 256, 3, 8, 50
    else:
        n0, levels, loops, steps = 512, 2, 16, 20
    if args.coarse_steps is not None:
        steps = args.coarse_steps
    log(f"initial state {n0}^3 with {loops} string loops (seed {args.seed})")
    U0 = string_loop_state(n0, float(n0), args.seed, loops)
    out = {"metric": "cell-updates/s per RK stage (AMR, all levels)", "unit": "cell-updates/s",
           "n_gpus": 1, "data": "synthetic", "higher_is_better": True,
           "config": {"workload": f"AMR {n0}^3 + {levels} levels, {loops} string loops R in [20, 60], "
                                  f"blocking factor 8, max box 64, tag buffer 2, regrid every 2 coarse steps, "
                                  f"{steps} coarse steps, beta = {args.beta}"
                                  + (f", tag mode {args.tag_mode}, te_crit {args.te_crit}" if args.tag_mode != 1 else "")
                                  + (", SSPRK3" if args.integrator != 4 else "")
                                  + (f", Laplacian order {args.lap_order}" if args.lap_order != 1 else "")
                                  + (", quartic interpolation" if args.interp == 4 else "")
                                  + (", local regrids" if args.regrid == "local" else "")
                                  + (f", Kreiss-Oliger order {args.ko_order} eps {args.ko_eps}" if args.ko_order else ""),
                      "seed": args.seed}}
    if args.workload == "amr256":
        prec = shamr.SH_F64 if args.prec == "f64" else shamr.SH_F32
        h, rep = workloads.run_amr(U0, levels, steps, prec=prec, beta=args.beta, log=log, tag_mode=args.tag_mode,
                                   te_crit=args.te_crit, integrator=args.integrator, lap_order=args.lap_order,
                                   interp=args.interp, ko_order=args.ko_order, ko_eps=args.ko_eps,
                                   regrid_mode=args.regrid)
        h.close()
        out.update({"value": rep["cell_updates_per_s_end_to_end"], "dtype": args.prec, "report": rep})
    else:
        res = workloads.fp32_vs_fp64(U0, levels, steps, beta=args.beta, log=log, regrid_mode=args.regrid)
        out.update({"value": res["f64"]["cell_updates_per_s_end_to_end"], "dtype": "f64 and f32",
                    "value_f32": res["f32"]["cell_updates_per_s_end_to_end"], "report": res})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
