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

import numpy as np

from . import shamr


def _advance(h, lev: int, sub: int, finest: int):
    h.advance(lev, sub)
    if lev < finest:
        _advance(h, lev + 1, 0, finest)
        _advance(h, lev + 1, 1, finest)
        h.average_down(lev + 1)


def coarse_step(h):
    """One step of the coarse level with every finer level subcycled under it."""
    _advance(h, 0, 0, h.num_levels() - 1)


def normalised_tee_scales(h):
    """Modifier scales s_c = 1 / max |U_c| over the whole hierarchy (appendix D's
    normalisation of the truncation error estimates of each field, section IV.C), 1 for a
    component whose maximum is 0; for sh_set_tee_fields before a regrid."""
    m = h.field_absmax()
    return [1.0 / v if v > 0.0 else 1.0 for v in m]


def carried_tags(idx_fine, M_coarse: int, grow: int = 1, n_error_buf: int = 2, blocking_factor: int = 8):
    """Tags of level l+1 carried down to level l, as a (n, 3) int32 list of level-l cells
    (x, y, z).  Clustering grows every tag by ``n_error_buf`` cells and tags the blocks of
    bf/2 cells it meets, so what a carried set must reproduce is the set of blocks met by
    the coarse parents of the fine tags grown by ``grow + n_error_buf`` cells (periodic,
    M_coarse cells per axis).  That set is built on a dense mask of blocks and returned
    as one cell per pair of adjacent blocks (a cell n_error_buf cells into the lower
    block meets exactly the two once grown), so its size follows the number of tagged
    blocks, not the number of fine tags.  With n_error_buf = 2 and one cell of growth the
    rebuilt level l+1 extends at least 6 fine cells beyond every fine tag: the tag's own
    buffer of 2 and the nesting gap of half a blocking factor (4) that the level-l+2 box
    refining it needs."""
    b = blocking_factor // 2
    n = n_error_buf
    r = grow + n
    idx = np.asarray(idx_fine).reshape(-1, 3)
    if idx.size == 0:
        return np.zeros((0, 3), np.int32)
    # a cell n into block a meets blocks a and a+1 once grown; p +- r meets two or three
    if not (b <= 2 * n < 2 * b) or M_coarse % b or not (b < 2 * r + 1 and r < b):
        return _carried_cells(idx, M_coarse, grow)
    nb = M_coarse // b
    # per axis: blocks A..B (two or three) met by parent +- r, i.e. block pairs A..B-1,
    # kept as the key (A, s) with s = B - A - 1 (0: one pair, 1: two)
    kt = np.int32 if (2 * nb) ** 3 < 2**31 else np.int64
    keys = np.zeros(idx.shape[0], kt)
    pow2 = (b & (b - 1)) == 0 and (nb & (nb - 1)) == 0
    sh = b.bit_length() - 1
    for d in (2, 1, 0):          # z, y, x: key = ((A_z*2 + s_z) * 2nb + A_y*2 + s_y) * 2nb + ...
        p = idx[:, d].astype(kt) >> 1
        if pow2:                 # floor division and periodic wrap by shifts and masks
            A = (p - r) >> sh
            s = ((p + r) >> sh) - A - 1
            A &= nb - 1
        else:
            A = np.floor_divide(p - r, b)
            s = np.floor_divide(p + r, b) - A - 1
            A = np.mod(A, nb)
        keys *= 2 * nb
        keys += (A << 1) | s
    seen = np.zeros((2 * nb) ** 3, bool)
    seen[keys] = True
    # pairs: a pair a of an axis comes from the key (a, any s) and from (a - 1, s = 1)
    pr = seen.reshape(nb, 2, nb, 2, nb, 2)
    pr = pr[:, 0] | pr[:, 1] | np.roll(pr[:, 1], 1, axis=0)                       # z
    pr = pr[:, :, 0] | pr[:, :, 1] | np.roll(pr[:, :, 1], 1, axis=1)              # y
    pr = pr[:, :, :, 0] | pr[:, :, :, 1] | np.roll(pr[:, :, :, 1], 1, axis=2)     # x
    az, ay, ax = np.nonzero(pr)
    return np.stack([ax * b + n, ay * b + n, az * b + n], 1).astype(np.int32)


def _carried_cells(idx, M_coarse: int, grow: int):
    """Carried tags as cells (coarse parents grown by ``grow``), for clustering
    parameters the block form does not cover."""
    c = np.unique(idx.astype(np.int64) // 2, axis=0)
    r = np.arange(-grow, grow + 1)
    off = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    out = (c[:, None, :] + off[None, :, :]).reshape(-1, 3) % M_coarse
    return np.unique(out, axis=0).astype(np.int32)


def merge_tags(a, b):
    """Both tag lists in one (clustering counts a cell tagged twice once)."""
    a = np.asarray(a, np.int32).reshape(-1, 3)
    b = np.asarray(b, np.int32).reshape(-1, 3)
    if not len(b):
        return a
    return np.concatenate([a, b])


def regrid(h, max_level: int, layout_for=None, efficiency: float = 0.7, max_level_bytes: int | None = None,
           log=None, timing: dict | None = None, start: int = 1, carry: bool = True):
    """Rebuild levels start..max_level from tags (levels below start are kept).

    ``layout_for(lev, ntag, idx)`` may return the boxes of level lev+1 from the tag list;
    by default the library clusters (Berger-Rigoutsos) the blocks the tags meet, marked on
    the GPU (``tag_blocks``, ``cluster_blocks``: no tag list crosses to the host).  With
    ``carry``, the tags of every existing finer level are taken first, on the hierarchy as
    it stands, and each level's blocks are joined by those the grown parents of the level
    above it meet (what ``carried_tags`` gives as a cell list): levels are
    rebuilt coarsest first, and a level l+1 built from level l's tags alone could be too
    small to nest the refinement of a tag level l+1 holds near its edge, which clustering
    would then drop.  ``max_level_bytes`` caps the device arena of any one new level: a
    layout above it is not built, and that level and every finer one are removed instead
    (a field that has blown up tags nearly every plaquette, and refining all of it would
    not fit in memory).  ``timing``, if given, accumulates host seconds spent in tagging,
    clustering and layout changes.  Returns the tag counts (each level's own).
    """
    counts = []
    nbuf = h.params.n_error_buf
    carried = {}      # level -> bitset of its blocks met by the finer level's grown tag parents
    if carry and layout_for is None:
        t0 = time.perf_counter()
        for lev in range(max(1, start), min(h.num_levels(), max_level)):
            n, bits = h.tag_blocks(lev, 1 + nbuf, halve=True)
            if n:
                carried[lev - 1] = bits
        if timing is not None:
            timing["tag"] = timing.get("tag", 0.0) + time.perf_counter() - t0
    for lev in range(max(0, start - 1), max_level):
        if lev >= h.num_levels():
            break
        t0 = time.perf_counter()
        if layout_for is not None:
            ntag, idx = h.tag(lev)
        else:      # tagged blocks: the level's own tags grown by n_error_buf, the carried ones joined
            ntag, bits = h.tag_blocks(lev, nbuf, bits=carried.get(lev))
        t1 = time.perf_counter()
        counts.append(ntag)
        if layout_for is not None:
            boxes = layout_for(lev, ntag, idx)
        else:
            boxes = h.cluster_blocks(lev, bits, efficiency)
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


def local_regrid(h, max_level: int, log=None, timing: dict | None = None):
    """Local regrid (section II, "Local versus global regrid"): every existing box stays;
    from the coarsest level up, the tags of level l grow level l+1 (creating it if it is
    the next level below max_level) where they come within n_error_buf cells of its
    boundary, and coarser levels grow where the added boxes need the nesting gap.  Changed
    levels are laid out again coarsest first (old cells kept, new ones interpolated).
    Returns {level: cells added}."""
    p = h.params
    bf, nbuf, mb = p.blocking_factor, p.n_error_buf, p.max_box
    added_cells = {}
    for lev in range(max_level):
        if lev >= h.num_levels():
            break
        t0 = time.perf_counter()
        ntag, idx = h.tag(lev)
        t1 = time.perf_counter()
        fine = lev + 1
        cur = h.boxes.get(fine, []) if fine < h.num_levels() else []
        add = {}
        new = shamr.local_tag_boxes(p.n0 << fine, cur, idx, bf, nbuf, mb) if ntag else []
        if new:
            add[fine] = new
            k = lev
            while new and k >= 1:
                new = shamr.local_nest_boxes(p.n0 << k, new, h.boxes[k], bf, mb)
                if new:
                    add[k] = new
                k -= 1
        t2 = time.perf_counter()
        for k in sorted(add):
            old = h.boxes.get(k, []) if k < h.num_levels() else []
            h.set_layout(k, list(old) + add[k])
            added_cells[k] = added_cells.get(k, 0) + sum(
                (b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1) for b in add[k])
        if timing is not None:
            t3 = time.perf_counter()
            for key, v in (("tag", t1 - t0), ("cluster", t2 - t1), ("layout", t3 - t2)):
                timing[key] = timing.get(key, 0.0) + v
        if log is not None and add:
            log(f"local regrid from level {lev}: added " + ", ".join(f"{len(v)} boxes to level {k}"
                                                                  for k, v in sorted(add.items())))
    return added_cells


class RegridPolicy:
    """Choice between a local and a global regrid (section II, "Local versus global
    regrid"): the volume added to each level by local regrids since the last global one,
    as a fraction dV_l of the level's volume then, triggers a global regrid once some dV_l
    exceeds eps_strong, starting at the lowest level with dV_l >= eps_weak (that level and
    every finer one are rebuilt from the tags of the level below); so does the
    max_local-th consecutive local regrid (then from level 1).  Defaults as in the paper:
    10 %, 5 %, 10."""

    def __init__(self, eps_strong: float = 0.10, eps_weak: float = 0.05, max_local: int = 10):
        self.eps_s, self.eps_w, self.max_local = eps_strong, eps_weak, max_local
        self.base = {}
        self.added = {}
        self.nlocal = 0

    def after_global(self, cells_per_level):
        """cells_per_level[l] = cells of level l right after a global regrid."""
        self.base = {k: int(v) for k, v in enumerate(cells_per_level) if k >= 1}
        self.added = {}
        self.nlocal = 0

    def after_local(self, added_cells):
        for k, v in added_cells.items():
            self.added[k] = self.added.get(k, 0) + int(v)
        self.nlocal += 1

    def fractions(self):
        out = {}
        for k in set(self.base) | set(self.added):
            b, a = self.base.get(k, 0), self.added.get(k, 0)
            out[k] = a / b if b else (float("inf") if a else 0.0)
        return out

    def decide(self):
        """("local", None), or ("global", l): rebuild levels >= l (l >= 1) from the tags of
        level l-1."""
        if self.nlocal >= self.max_local:
            return "global", 1
        dv = self.fractions()
        if any(v > self.eps_s for v in dv.values()):
            return "global", max(1, min(k for k, v in dv.items() if v >= self.eps_w))
        return "local", None

