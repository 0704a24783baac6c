"""Launch-shape autotuner for the level step.

``tune(h)`` times the candidate launch shapes of level 0 on a twin of the hierarchy
(same parameters, layout and state, its own stream), so the simulation itself does not
move, and applies the fastest to ``h`` with ``sh_set_tuning``.  Every candidate gives the
same bits (the shapes change only the data movement), so the choice is purely a matter of
time.  Candidates: the fused four-stage step over footprints x kernel variants (those the
level's boxes admit), and the per-stage kernels as a fallback.
"""
from __future__ import annotations

import time

from . import shamr

# (fused_shape, fused_variant); footprints (x, y) of the shapes
FUSED_SHAPES = {0: (32, 8), 1: (64, 4), 2: (32, 16), 3: (16, 8)}
FUSED_VARIANTS = (0, 3, 4, 5, 6, 7, 8)


def candidates(boxes, params=None):
    """Launch shapes that apply to a level with these boxes:
    (kind, nontemporal, tile_z, fuse, fused_shape, fused_tile_z, fused_variant).  With the
    hierarchy's params, fused shapes are offered only where the fused step applies (the
    7-point stencil without dissipation, not RKN4), and SSPRK3 skips the accumulator
    variants."""
    out = [(8, 1, 0, 0, 0, 0, 0), (0, 1, 0, 0, 0, 0, 0)]
    if params is not None and (params.lap_order > 1 or params.ko_order or params.integrator == 21):
        return out
    variants = FUSED_VARIANTS
    if params is not None and params.integrator in (3, 10):
        variants = tuple(v for v in FUSED_VARIANTS if v not in (3, 6))   # they run as 4 and 5
    for shape, (tx, ty) in FUSED_SHAPES.items():
        if all(shamr.box_shape(b)[2] % tx == 0 and shamr.box_shape(b)[1] % ty == 0 for b in boxes):
            out += [(8, 1, 0, 4, shape, 0, v) for v in variants]
    return out


def _twin(h, stream):
    p = h.params
    t = shamr.Hierarchy(p.n0, p.L, p.cfl, p.eta0, p.lam, p.alpha_fric, p.beta_pot, max_level=0,
                        blocking_factor=p.blocking_factor, max_box=p.max_box, n_error_buf=p.n_error_buf,
                        prec=p.prec, stream=stream, integrator=p.integrator, lap_order=p.lap_order,
                        interp=p.interp, ko_order=p.ko_order, ko_eps=p.ko_eps)
    t.set_layout(0, h.boxes[0])
    t.write_dense(0, h.read_dense(0))
    t.fill_ghosts(0)
    return t


def tune(h, steps: int = 5, cands=None, log=None):
    """Time each candidate for ``steps`` level-0 steps (after one untimed step) on a twin
    of ``h``; apply the fastest to ``h``.  Returns {candidate: ms per step}, fastest first."""
    import torch
    stream = torch.cuda.Stream()
    twin = _twin(h, stream)
    cands = cands if cands is not None else candidates(h.boxes[0], h.params)
    times = {}
    try:
        for c in cands:
            twin.set_tuning(*c)
            twin.advance(0)
            twin.sync()
            t0 = time.perf_counter()
            for _ in range(steps):
                twin.advance(0)
            twin.sync()
            times[c] = (time.perf_counter() - t0) / steps * 1e3
            if log is not None:
                log(f"autotune {c}: {times[c]:.3f} ms/step")
    finally:
        twin.close()
    best = min(times, key=times.get)
    h.set_tuning(*best)
    return dict(sorted(times.items(), key=lambda kv: kv[1]))
