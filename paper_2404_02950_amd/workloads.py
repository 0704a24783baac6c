"""Measured workloads beyond the single-level step: AMR hierarchies with string loops.

``run_amr`` builds a hierarchy from seeded string loops (coarse level n0^3, dx = 1), tags
and clusters it into refinement levels (Berger-Rigoutsos, blocking factor 8, boxes up to
64^3, tag buffer 2), then advances it with Berger-Oliger subcycling, regridding every
``regrid_every`` coarse steps, and reports per-level sizes, throughput and energies.
"""
from __future__ import annotations

import time

import numpy as np

from . import driver, shamr


def build_hierarchy(U0: np.ndarray, max_level: int, prec: int, beta: int = 2, max_box: int = 64,
                    blocking_factor: int = 8, n_error_buf: int = 2, efficiency: float = 0.7, integrator: int = 4,
                    lap_order: int = 1, interp: int = 1, ko_order: int = 0, ko_eps: float = 0.0):
    n0 = U0.shape[-1]
    h = shamr.Hierarchy(n0, float(n0), 0.25, 0.1, 1.0, 2.0, beta, max_level=max_level,
                        blocking_factor=blocking_factor, max_box=max_box, n_error_buf=n_error_buf, prec=prec,
                        integrator=integrator, lap_order=lap_order, interp=interp, ko_order=ko_order,
                        ko_eps=ko_eps)
    h.set_layout(0, [(0, 0, 0, n0 - 1, n0 - 1, n0 - 1)])
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    driver.regrid(h, max_level, efficiency=efficiency)
    return h


def level_summary(h):
    out = []
    for lev in range(h.num_levels()):
        info = h.level_info(lev)
        out.append({"level": lev, "boxes": info["nboxes"], "cells": info["ncells"], "k": info["k"]})
    return out


def run_amr(U0: np.ndarray, max_level: int, coarse_steps: int, prec: int = shamr.SH_F64, beta: int = 2,
            regrid_every: int = 2, log=print, efficiency: float = 0.7, max_level_bytes: int | None = None,
            tag_mode: int = 1, te_crit: float = 1e-2, integrator: int = 4, lap_order: int = 1, interp: int = 1,
            ko_order: int = 0, ko_eps: float = 0.0, regrid_mode: str = "global"):
    """Advance an AMR hierarchy; returns (hierarchy, report dict).

    ``max_level_bytes`` (default: a quarter of the device memory free at the start) caps
    any one level's arena at regrid; see ``driver.regrid``.  ``tag_mode``: 1 = plaquette
    winding, 2 = truncation error estimate above ``te_crit``, 3 = either.  With estimates
    the shadow level is started two coarse steps before each regrid, takes its one step,
    and gives level 0 its estimate at the regrid (the finer levels get theirs at every
    synchronisation); the initial layout uses the plaquettes, no estimate existing yet.
    ``integrator``: 4 = classic RK4, 3 or 10 = SSPRK3; ``lap_order``: 1, 2, 3 = 7-, 13-,
    19-point Laplacian; ``interp``: 1 linear, 4 quartic conservative; ``ko_order``/``ko_eps``:
    Kreiss-Oliger dissipation; ``regrid_mode``: "global" (cluster all tags every time) or
    "local" (local regrids, with a global one when driver.RegridPolicy asks for it)."""
    import torch
    if max_level_bytes is None:
        max_level_bytes = torch.cuda.mem_get_info()[0] // 4
    use_tee = bool(tag_mode & 2)
    if use_tee and regrid_every < 2:
        raise ValueError("estimates need at least two coarse steps between regrids (the shadow step)")
    t0 = time.perf_counter()
    h = build_hierarchy(U0, max_level, prec, beta=beta, efficiency=efficiency, integrator=integrator,
                        lap_order=lap_order, interp=interp, ko_order=ko_order, ko_eps=ko_eps)
    nst = 3 if integrator in (3, 10) else 4
    if use_tee:
        h.set_tee(True, te_crit, tag_mode)
    h.sync()
    t_build = time.perf_counter() - t0
    e0, bad0 = h.energy()
    levels0 = level_summary(h)
    log(f"built hierarchy in {t_build:.1f} s: {levels0}")
    cell_stages = 0
    t_regrid = 0.0
    regrid_parts = {}
    capped = []
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    shadow = False
    policy = driver.RegridPolicy()
    policy.after_global([lv["cells"] for lv in levels0])
    kinds = {"global": 0, "local": 0}
    for step in range(coarse_steps):
        if step > 0 and step % regrid_every == 0:
            if shadow:
                h.shadow_end()
                shadow = False
            h.sync()  # the queued level steps are not regrid time
            tr = time.perf_counter()
            nlev = h.num_levels()
            kind, start = policy.decide() if regrid_mode == "local" else ("global", 1)
            if kind == "local":
                policy.after_local(driver.local_regrid(h, max_level, log=None, timing=regrid_parts))
            else:
                driver.regrid(h, max_level, efficiency=efficiency, max_level_bytes=max_level_bytes, log=log,
                              timing=regrid_parts, start=start)
                policy.after_global([h.level_info(lev)["ncells"] for lev in range(h.num_levels())])
            kinds[kind] += 1
            h.sync()
            if h.num_levels() < nlev:
                capped.append({"coarse_step": step, "levels": h.num_levels()})
            t_regrid += time.perf_counter() - tr
        if use_tee and step % regrid_every == regrid_every - 2 and step + 2 <= coarse_steps:
            h.shadow_begin()
            h.shadow_advance()
            shadow = True
        # cell updates of this coarse step: level l takes 2^l steps of nst stages
        for lev in range(h.num_levels()):
            cell_stages += h.level_info(lev)["ncells"] * nst * (1 << lev)
        driver.coarse_step(h)
        if (step + 1) % 10 == 0:
            h.sync()
            log(f"coarse step {step + 1}: {level_summary(h)}")
    if shadow:
        h.shadow_end()
    h.sync()
    wall = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile(False)
    e1, bad1 = h.energy()
    kernel_ms = sum(v[0] for v in prof.values())
    report = {
        "coarse_steps": coarse_steps,
        "levels_start": levels0,
        "levels_end": level_summary(h),
        "wall_s": wall,
        "regrid_s": t_regrid,
        "regrid_parts_s": regrid_parts,
        "refinement_capped": capped,
        "build_s": t_build,
        "cell_stage_updates": cell_stages,
        "cell_updates_per_s_end_to_end": cell_stages / wall,
        "cell_updates_per_s_kernels": cell_stages / (kernel_ms / 1e3) if kernel_ms else None,
        "kernel_ms": {k: v[0] for k, v in prof.items() if v[1]},
        "launches": {k: v[1] for k, v in prof.items() if v[1]},
        "energy_start": e0,
        "energy_end": e1,
        "nonfinite_end": bad1,
        "tag_mode": tag_mode,
        "integrator": integrator,
        "regrid_mode": regrid_mode,
        "regrids": kinds,
        "lap_order": lap_order,
        "interp": interp,
        "ko_order": ko_order,
        "cell_steps_per_s_end_to_end": cell_stages / nst / wall,
        "te_crit": te_crit if use_tee else None,
    }
    return h, report


def fp32_vs_fp64(U0: np.ndarray, max_level: int, coarse_steps: int, beta: int = 2, log=print,
                 regrid_mode: str = "global"):
    """The same AMR run in FP64 and FP32-storage mode: energies, tag-mask differences
    on the coarse level and the largest coarse-level field difference at the end.

    The reference is this library's FP64 run, not the oracle: at these sizes the oracle
    cannot run, and the FP64 GPU path equals it bit for bit wherever both run (the AMR
    parity suite, and the sampled 512^3 single-level parity).  Each run regrids from its
    own tags, so the refined levels may differ in layout; only level 0 is compared."""
    res = {}
    fields = {}
    masks = {}
    for name, prec in (("f64", shamr.SH_F64), ("f32", shamr.SH_F32)):
        h, rep = run_amr(U0, max_level, coarse_steps, prec=prec, beta=beta, log=log, regrid_mode=regrid_mode)
        res[name] = rep
        fields[name] = h.read_dense(0)
        masks[name] = h.tag_mask_dense(0)
        h.close()
    d = np.abs(fields["f32"] - fields["f64"])
    finite = np.isfinite(fields["f64"])
    res["coarse_max_abs_diff"] = float(np.max(d[finite])) if finite.any() else None
    res["coarse_max_rel_diff"] = (float(np.max(d[finite]) / np.max(np.abs(fields["f64"][finite])))
                                  if finite.any() else None)
    res["coarse_tag_mask_differences"] = int(np.count_nonzero(masks["f32"] != masks["f64"]))
    res["reference"] = ("the library's FP64 run (bit-identical to the FP64 oracle wherever both run); "
                        "level 0 only, each precision regridding from its own tags")
    e64, e32 = res["f64"]["energy_end"][3], res["f32"]["energy_end"][3]
    res["energy_total_rel_diff"] = abs(e32 - e64) / abs(e64) if e64 else None
    return res
