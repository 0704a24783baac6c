"""Local regrid (oracle; test infrastructure only).

Section II, "Local versus global regrid": instead of clustering all tagged cells anew, a
local regrid keeps every existing box of the finer level and only expands that level
around tagged cells that lie closer than ``n_error_buf`` cells to its boundary (or outside
it); the refined volume only grows.  Coarser levels are expanded as well where that is
needed to keep the finer level properly nested.  Restated here on the block grid of each
level (blocks of ``bf`` cells, the blocking factor, which every box of a refined level is
made of):

* a tagged cell X of level l needs the level-(l+1) blocks that meet the refinement of the
  cube [X - n_error_buf, X + n_error_buf] (periodic); needed blocks not yet in level l+1
  are added;
* a level-(k+1) block B needs the level-k blocks that meet its coarsening grown by bf/2
  level-k cells (the nesting gap); missing ones are added to level k (k >= 1; level 0
  covers the domain), and in turn need their own support on level k-1;
* added blocks become boxes in three merges, each at most ``max_box`` cells long and
  without wrapping: runs of consecutive blocks along x in each (y, z) block row (from the
  lowest x); then runs with the same x extent in consecutive y rows of a z plane (from
  the lowest y); then rectangles with the same x and y extents in consecutive z planes
  (from the lowest z).  Boxes are listed by (z, y, x) of their lowest corner.
"""
from __future__ import annotations

import numpy as np


def _blocks_of(boxes, bf: int, M: int) -> np.ndarray:
    """Block occupancy (NB^3 bool, [z, y, x]) of a level's boxes; every box must consist of
    whole blocks."""
    nb = M // bf
    occ = np.zeros((nb, nb, nb), dtype=bool)
    for b in boxes:
        lo = np.array(b[:3])
        hi = np.array(b[3:]) + 1
        if np.any(lo % bf) or np.any(hi % bf):
            raise ValueError(f"box {b} is not made of whole {bf}-blocks")
        occ[lo[2] // bf:hi[2] // bf, lo[1] // bf:hi[1] // bf, lo[0] // bf:hi[0] // bf] = True
    return occ


def _mark_range(need: np.ndarray, lo, hi):
    """Mark blocks lo..hi (inclusive, per axis [x, y, z], may wrap periodically)."""
    nb = need.shape[0]
    zs = [z % nb for z in range(lo[2], hi[2] + 1)]
    ys = [y % nb for y in range(lo[1], hi[1] + 1)]
    xs = [x % nb for x in range(lo[0], hi[0] + 1)]
    need[np.ix_(zs, ys, xs)] = True


def _merge_runs(items, key, pos, run_max):
    """Greedy merge of items whose ``key`` agrees and whose ``pos`` are consecutive: items
    sorted by (key, pos), a run grows from its lowest pos while the next item continues it
    and the run is shorter than run_max.  Items are (key..., lo, hi) with lo/hi = pos
    extent; returns merged (key, lo, hi)."""
    out = []
    items = sorted(items, key=lambda t: (key(t), pos(t)[0]))
    i = 0
    while i < len(items):
        k, (lo, hi) = key(items[i]), pos(items[i])
        j = i + 1
        while (j < len(items) and key(items[j]) == k and pos(items[j])[0] == hi + 1
               and pos(items[j])[1] - lo + 1 <= run_max):
            hi = pos(items[j])[1]
            j += 1
        out.append((k, lo, hi))
        i = j
    return out


def blocks_to_boxes(new: np.ndarray, bf: int, max_box: int):
    """Boxes (fine index, inclusive) from a block mask by the three merges above."""
    nb = new.shape[0]
    run_max = max(1, max_box // bf)
    runs = []                                            # (z, y, x0, x1)
    for bz in range(nb):
        for by in range(nb):
            bx = 0
            while bx < nb:
                if not new[bz, by, bx]:
                    bx += 1
                    continue
                start = bx
                while bx < nb and new[bz, by, bx] and bx - start < run_max:
                    bx += 1
                runs.append((bz, by, start, bx - 1))
    # y: same (z, x0, x1), consecutive y
    rects = [(k[0], lo, hi, k[1], k[2]) for k, lo, hi in
             _merge_runs(runs, key=lambda r: (r[0], r[2], r[3]), pos=lambda r: (r[1], r[1]), run_max=run_max)]
    # z: same (y0, y1, x0, x1), consecutive z; rects are (z, y0, y1, x0, x1)
    boxes = [(lo, k[0], k[1], k[2], k[3], hi) for k, lo, hi in
             _merge_runs(rects, key=lambda r: (r[1], r[2], r[3], r[4]), pos=lambda r: (r[0], r[0]), run_max=run_max)]
    # (z0, y0, y1, x0, x1, z1) -> fine boxes, ordered by lowest corner (z, y, x)
    boxes.sort(key=lambda b: (b[0], b[1], b[3]))
    return [(x0 * bf, y0 * bf, z0 * bf, (x1 + 1) * bf - 1, (y1 + 1) * bf - 1, (z1 + 1) * bf - 1)
            for z0, y0, y1, x0, x1, z1 in boxes]


def tag_blocks(tag_idx, M_coarse: int, bf: int, n_error_buf: int) -> np.ndarray:
    """Level-(l+1) blocks needed by the tagged level-l cells (tag_idx: (n, 3) x, y, z)."""
    nb = 2 * M_coarse // bf
    need = np.zeros((nb, nb, nb), dtype=bool)
    for x, y, z in np.asarray(tag_idx).reshape(-1, 3):
        lo = [2 * (c - n_error_buf) for c in (x, y, z)]
        hi = [2 * (c + n_error_buf) + 1 for c in (x, y, z)]
        _mark_range(need, [v // bf for v in lo], [v // bf for v in hi])
    return need


def nest_blocks(fine_new: np.ndarray, bf: int) -> np.ndarray:
    """Level-k blocks needed by the level-(k+1) blocks in fine_new (coarsening grown by
    bf/2 level-k cells)."""
    nbf = fine_new.shape[0]
    need = np.zeros((nbf // 2,) * 3, dtype=bool)
    h = bf // 2
    for bz, by, bx in np.argwhere(fine_new):
        lo = [B * h - h for B in (bx, by, bz)]           # level-k cells, coarsened block grown
        hi = [B * h + h - 1 + h for B in (bx, by, bz)]
        _mark_range(need, [v // bf for v in lo], [v // bf for v in hi])
    return need


def local_regrid(level_boxes, n0: int, lev: int, tag_idx, bf: int, n_error_buf: int, max_box: int):
    """Added boxes per level for a local regrid driven by the tags of level ``lev``.

    level_boxes: boxes of levels 0..finest (level_boxes[k] in level-k index space); level
    lev+1 may be absent (a new level).  Returns {k: [added boxes]} for k = 1..lev+1, empty
    lists omitted.
    """
    M = lambda k: n0 << k  # noqa: E731
    fine = lev + 1
    have = _blocks_of(level_boxes[fine], bf, M(fine)) if fine < len(level_boxes) else \
        np.zeros((M(fine) // bf,) * 3, dtype=bool)
    new = tag_blocks(tag_idx, M(lev), bf, n_error_buf) & ~have
    out = {}
    if new.any():
        out[fine] = blocks_to_boxes(new, bf, max_box)
    k = lev
    while new.any() and k >= 1:
        need = nest_blocks(new, bf)
        have = _blocks_of(level_boxes[k], bf, M(k))
        new = need & ~have
        if new.any():
            out[k] = blocks_to_boxes(new, bf, max_box)
        k -= 1
    return out
