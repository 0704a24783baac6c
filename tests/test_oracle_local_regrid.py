"""Pins of the oracle's local regrid (section II, "Local versus global regrid"): nothing is
added for tags well inside the refined region, a tag at the boundary adds exactly the
blocks its buffer reaches, the result covers every buffered tag, never removes a box,
wraps periodically, keeps every level properly nested (checked with the independent layout
checker, coarser levels expanded where needed) and merges blocks along x."""
import numpy as np
import pytest

from oracle.amr import boxes_mask, coarsen_mask, dilate, refine_mask
from oracle.layout import check_layout
from oracle.local_regrid import blocks_to_boxes, local_regrid


def _cube(lo, hi):
    return (lo, lo, lo, hi, hi, hi)


def test_tags_inside_add_nothing():
    # level 1 covers coarse cells 8..23; tags at least n_error_buf inside need nothing
    boxes = [[_cube(0, 31)], [_cube(16, 47)]]
    tags = np.array([[12, 12, 12], [14, 18, 16], [10, 10, 21]])
    assert local_regrid(boxes, 32, 0, tags, 8, 2, 64) == {}


def test_boundary_tag_adds_the_blocks_its_buffer_reaches():
    # tag at coarse (23, 16, 16), buffer 2: refined x range 42..51 needs fine block 6 (48..55);
    # y and z ranges 28..37 need blocks 3 and 4
    boxes = [[_cube(0, 31)], [_cube(16, 47)]]
    out = local_regrid(boxes, 32, 0, np.array([[23, 16, 16]]), 8, 2, 64)
    assert out == {1: [(48, 24, 24, 55, 39, 39)]}                # 1 x 2 x 2 blocks, merged


def test_blocks_merge_along_x_up_to_max_box():
    new = np.zeros((8, 8, 8), dtype=bool)
    new[1, 2, 0:7] = True
    assert blocks_to_boxes(new, 8, 24) == [(0, 16, 8, 23, 23, 15), (24, 16, 8, 47, 23, 15),
                                           (48, 16, 8, 55, 23, 15)]


def test_blocks_merge_in_y_and_z():
    new = np.zeros((8, 8, 8), dtype=bool)
    new[0:2, 0:5, 0:2] = True                   # 2 x 5 x 2 blocks: y extent capped at 3 blocks
    new[3, 0, 4] = True                         # a lone block
    assert blocks_to_boxes(new, 8, 24) == [(0, 0, 0, 15, 23, 15), (0, 24, 0, 15, 39, 15),
                                           (32, 0, 24, 39, 7, 31)]
    # every block exactly once
    m = np.zeros((64,) * 3, dtype=bool)
    for b in blocks_to_boxes(new, 8, 24):
        assert not m[b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1].any()
        m[b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = True
    assert m.sum() == new.sum() * 512


def test_periodic_wrap():
    boxes = [[_cube(0, 31)], [(0, 0, 0, 15, 15, 15)]]
    out = local_regrid(boxes, 32, 0, np.array([[0, 3, 3]]), 8, 2, 64)
    xs = sorted({b[0] for b in out[1]})
    assert 56 in xs                                         # x = -2..-1 wraps to the last block


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_tags_covered_nested_and_nothing_removed(seed):
    rng = np.random.default_rng(seed)
    n0, bf, nbuf = 32, 8, 2
    l1 = [(16, 16, 16, 31, 31, 31), (32, 16, 16, 47, 39, 31)]
    l2 = [(40, 40, 40, 55, 55, 55)]
    boxes = [[_cube(0, n0 - 1)], l1, l2]
    v1 = boxes_mask(l1, 2 * n0)
    cand = np.argwhere(v1)                                  # [z, y, x] of level-1 cells
    pick = cand[rng.choice(len(cand), 6, replace=False)]
    tags = pick[:, ::-1]                                    # (x, y, z)
    out = local_regrid(boxes, n0, 1, tags, bf, nbuf, 32)
    new2 = l2 + out.get(2, [])
    new1 = l1 + out.get(1, [])
    # every buffered tag is refined
    tm = np.zeros((2 * n0,) * 3, dtype=bool)
    tm[pick[:, 0], pick[:, 1], pick[:, 2]] = True
    need = refine_mask(dilate(tm, nbuf))
    assert np.all(boxes_mask(new2, 4 * n0)[need])
    # old boxes kept, added ones disjoint (boxes_mask raises on overlaps)
    boxes_mask(new1, 2 * n0)
    # both refined levels properly nested, checked independently
    v0 = np.ones((n0,) * 3, dtype=bool)
    assert check_layout(new1, 2 * n0, v0, bf, 32) == []
    assert check_layout(new2, 4 * n0, boxes_mask(new1, 2 * n0), bf, 32) == []


def test_expands_the_coarser_level_for_nesting():
    # a tag near the boundary of level 1 needs level-2 blocks whose nesting gap leaves
    # level 1: level 1 grows too, only by blocks that the gap reaches
    n0 = 32
    l1 = [(8, 8, 8, 39, 39, 39)]
    l2 = [(32, 32, 32, 47, 47, 47)]
    v0 = np.ones((n0,) * 3, dtype=bool)
    assert check_layout(l2, 4 * n0, boxes_mask(l1, 2 * n0), 8, 64) == []      # a proper start
    out = local_regrid([[_cube(0, n0 - 1)], l1, l2], n0, 1, np.array([[37, 24, 24]]), 8, 2, 64)
    assert 1 in out and 2 in out
    new1 = l1 + out[1]
    assert check_layout(new1, 2 * n0, v0, 8, 64) == []
    assert check_layout(l2 + out[2], 4 * n0, boxes_mask(new1, 2 * n0), 8, 64) == []
    need = dilate(coarsen_mask(boxes_mask(out[2], 4 * n0)), 4)
    for b in out[1]:
        assert need[b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1].any(), b


def test_unaligned_boxes_are_refused():
    with pytest.raises(ValueError):
        local_regrid([[_cube(0, 31)], [(2, 0, 0, 17, 15, 15)]], 32, 0, np.array([[1, 1, 1]]), 8, 1, 64)
