"""Berger-Oliger subcycling and regridding on top of the C-ABI (host orchestration).

Order (section II.A, Fig. 2): a level takes one step of dt_l; if a finer level exists it
then takes two steps of dt_l/2 (the first and second sub-step), after which the two
levels are synchronised (fine averaged onto coarse, fine ghosts refilled).  Each level
step itself (stages, ghost fills between stages, the fill at its end) is issued by
sh_advance_level.  Regrid (section II, "regridding"): tag a level, cluster the tags into
boxes of the next level, set that layout; repeated from the coarsest level upwards so
each new level is nested in the level below it as it now is.
"""
from __future__ import annotations

import time


def _advance(h, lev: int, sub: int, finest: int):
    h.advance(lev, sub)
    if lev < finest:
        _advance(h, lev + 1, 0, finest)
        _advance(h, lev + 1, 1, finest)
        h.average_down(lev + 1)


def coarse_step(h):
    """One step of the coarse level with every finer level subcycled under it."""
    _advance(h, 0, 0, h.num_levels() - 1)


def regrid(h, max_level: int, layout_for=None, efficiency: float = 0.7, max_level_bytes: int | None = None,
           log=None, timing: dict | None = None):
    """Rebuild levels 1..max_level from tags.

    ``layout_for(lev, ntag, idx)`` may return the boxes of level lev+1; by default the
    tags are clustered by the library (Berger-Rigoutsos).  ``max_level_bytes`` caps the
    device arena of any one new level: a layout above it is not built, and that level
    and every finer one are removed instead (a field that has blown up tags nearly every
    plaquette, and refining all of it would not fit in memory).  ``timing``, if given,
    accumulates host seconds spent in tagging, clustering and layout changes.  Returns
    the tag counts.
    """
    counts = []
    for lev in range(max_level):
        if lev >= h.num_levels():
            break
        t0 = time.perf_counter()
        ntag, idx = h.tag(lev)
        t1 = time.perf_counter()
        counts.append(ntag)
        boxes = layout_for(lev, ntag, idx) if layout_for is not None else h.cluster(lev, idx, efficiency)
        t2 = time.perf_counter()
        if boxes and max_level_bytes is not None:
            need = h.arena_bytes(lev + 1, boxes)
            if need > max_level_bytes:
                if log is not None:
                    log(f"regrid: level {lev + 1} would need {need / 2**30:.1f} GiB "
                        f"(cap {max_level_bytes / 2**30:.1f} GiB, {ntag} tags on level {lev}); "
                        f"levels >= {lev + 1} removed")
                boxes = []
        h.set_layout(lev + 1, boxes)
        if timing is not None:
            t3 = time.perf_counter()
            for k, v in (("tag", t1 - t0), ("cluster", t2 - t1), ("layout", t3 - t2)):
                timing[k] = timing.get(k, 0.0) + v
        if not boxes:
            break
    return counts
