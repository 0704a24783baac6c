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


def _advance(h, lev: int, sub: int, finest: int):
    h.advance(lev, sub)
    if lev < finest:
        _advance(h, lev + 1, 0, finest)
        _advance(h, lev + 1, 1, finest)
        h.average_down(lev + 1)


def coarse_step(h):
    """One step of the coarse level with every finer level subcycled under it."""
    _advance(h, 0, 0, h.num_levels() - 1)


def regrid(h, max_level: int, layout_for=None, efficiency: float = 0.7):
    """Rebuild levels 1..max_level from tags.

    ``layout_for(lev, ntag, idx)`` may return the boxes of level lev+1; by default the
    tags are clustered by the library (Berger-Rigoutsos).  Returns the tag counts.
    """
    counts = []
    for lev in range(max_level):
        if lev >= h.num_levels():
            break
        ntag, idx = h.tag(lev)
        counts.append(ntag)
        boxes = layout_for(lev, ntag, idx) if layout_for is not None else h.cluster(lev, idx, efficiency)
        h.set_layout(lev + 1, boxes)
        if not boxes:
            break
    return counts
