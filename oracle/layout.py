"""Box-layout checks and a plain block layout (oracle; test infrastructure only).

Rules from the paper (section II and II.C, appendix E "AMR parameters"):
* every box side is a multiple of the blocking factor (boxes start on multiples too);
* every tagged cell is refined together with a buffer of ``n_error_buf`` cells;
* a fine level is properly nested in the coarse level with a gap of at least one fine
  blocking factor: the coarsened fine boxes grown by bf/2 coarse cells lie inside the
  coarse level (periodically);
* boxes are chopped to at most ``max_box`` cells per side.

``block_layout`` is the simplest layout obeying these rules: every bf-block of the fine
level whose coarse footprint holds a buffered tag and whose gap fits inside the coarse
level becomes part of a box, blocks merged along x up to ``max_box``.
"""
from __future__ import annotations

import numpy as np

from .amr import boxes_mask, coarsen_mask, dilate, erode


def check_layout(fine_boxes, fine_M: int, coarse_valid: np.ndarray, bf: int, max_box: int,
                 tags: np.ndarray | None = None, n_error_buf: int = 0):
    """Return a list of violated rules (empty if the layout is proper)."""
    errs = []
    for b in fine_boxes:
        lo = np.array(b[:3])
        hi = np.array(b[3:]) + 1
        if np.any(lo % bf) or np.any(hi % bf):
            errs.append(f"box {b} not aligned to blocking factor {bf}")
        if np.any(hi - lo > max_box):
            errs.append(f"box {b} larger than {max_box}")
    try:
        fv = boxes_mask(fine_boxes, fine_M)
    except ValueError as e:
        return errs + [str(e)]
    cfoot = coarsen_mask(fv)
    if not np.all(coarse_valid[dilate(cfoot, bf // 2)]):
        errs.append("fine level not properly nested (gap bf/2 coarse cells)")
    if tags is not None:
        allowed = erode(coarse_valid, bf // 2)
        want = dilate(tags.astype(bool) & coarse_valid, n_error_buf) & allowed
        # blocks of the coarse level that a proper layout may hold in full
        if not np.all(cfoot[want & _block_allowed(allowed, bf // 2)]):
            errs.append("buffered tags not covered")
    return errs


def _block_allowed(allowed: np.ndarray, b: int) -> np.ndarray:
    """Cells whose whole b-block lies in ``allowed``."""
    M = allowed.shape[0]
    blk = allowed.reshape(M // b, b, M // b, b, M // b, b).all(axis=(1, 3, 5))
    return blk.repeat(b, 0).repeat(b, 1).repeat(b, 2)


def block_layout(tags: np.ndarray, coarse_valid: np.ndarray, bf: int, max_box: int,
                 n_error_buf: int):
    """Fine boxes (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi) covering the buffered tags."""
    b = bf // 2                                   # coarse cells per fine blocking factor
    M = tags.shape[0]
    allowed = erode(coarse_valid, b)
    want = dilate(tags.astype(bool) & coarse_valid, n_error_buf)
    nb = M // b
    sel = want.reshape(nb, b, nb, b, nb, b).any(axis=(1, 3, 5))
    ok = allowed.reshape(nb, b, nb, b, nb, b).all(axis=(1, 3, 5))
    sel &= ok
    boxes = []
    run_max = max(1, max_box // bf)
    for kz in range(nb):
        for ky in range(nb):
            kx = 0
            while kx < nb:
                if not sel[kz, ky, kx]:
                    kx += 1
                    continue
                k0 = kx
                while kx < nb and sel[kz, ky, kx] and kx - k0 < run_max:
                    kx += 1
                boxes.append((k0 * bf, ky * bf, kz * bf, kx * bf - 1, ky * bf + bf - 1,
                              kz * bf + bf - 1))
    return boxes
