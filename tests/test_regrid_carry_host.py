"""Host-side check of the driver's tag carry (no GPU): levels are rebuilt coarsest first,
so a tag that level 1 holds away from everything level 0 tags would lose its refinement
(the rebuilt level 1 would not contain it, and clustering drops tags whose refinement
cannot nest); carried down to level 0 it keeps it.  Layouts come from the library's
Berger-Rigoutsos (host code) and are checked with the oracle's layout rules."""
import numpy as np
import pytest

from oracle.amr import boxes_mask, coarsen_mask
from oracle.layout import check_layout
from paper_2404_02950_amd import driver

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")

M0, BF, MAX_BOX, NBUF = 32, 8, 64, 2


def _blob(lo, hi):
    r = [np.arange(a, b + 1) for a, b in zip(lo, hi)]
    x, y, z = np.meshgrid(*r, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.int32)


def _rebuild(carry):
    t0 = _blob((10, 10, 10), (13, 13, 13))            # level-0 tags (coarse cells)
    t1 = _blob((44, 24, 24), (46, 26, 26))            # tags level 1 holds now, far from t0's refinement
    level0 = [(0, 0, 0, M0 - 1, M0 - 1, M0 - 1)]
    if carry == "library":                            # carried inside the clustering call
        l1 = shamr.cluster_boxes(M0, level0, t0, BF, MAX_BOX, NBUF, carried=t1)
        l2 = shamr.cluster_boxes(2 * M0, l1, t1, BF, MAX_BOX, NBUF) if l1 else []
        return t1, l1, l2
    tags0 = driver.merge_tags(t0, driver.carried_tags(t1, M0)) if carry else t0
    l1 = shamr.cluster_boxes(M0, level0, tags0, BF, MAX_BOX, NBUF)
    l2 = shamr.cluster_boxes(2 * M0, l1, t1, BF, MAX_BOX, NBUF) if l1 else []
    return t1, l1, l2


def _blocks_met(cells, M, grow, b=4):
    """Blocks of b cells that cells grown by ``grow`` meet (periodic), by brute force."""
    out = set()
    for x, y, z in np.asarray(cells).reshape(-1, 3).tolist():
        rng = [range(c - grow, c + grow + 1) for c in (x, y, z)]
        for cx in rng[0]:
            for cy in rng[1]:
                for cz in rng[2]:
                    out.add(((cx % M) // b, (cy % M) // b, (cz % M) // b))
    return out


def test_carried_tags_meet_the_blocks_of_the_grown_parents():
    # clustering grows each tag by n_error_buf = 2 and tags the blocks of bf/2 = 4 cells
    # it meets: the carried list must meet exactly the blocks the coarse parents grown by
    # 1 + 2 meet (fine tags at every residue mod 8, at both periodic ends, and a cluster)
    rng = np.random.default_rng(3)
    fine = np.concatenate([np.array([[0, 0, 0], [1, 1, 1], [9, 4, 63], [63, 62, 61], [5, 13, 22]], np.int32),
                           rng.integers(0, 64, (40, 3), dtype=np.int32)])
    c = driver.carried_tags(fine, 32)
    parents = fine // 2
    assert _blocks_met(c, 32, 2) == _blocks_met(parents, 32, 3)
    # far fewer cells than the grown parents: one per pair of blocks
    assert len(c) < len(driver._carried_cells(fine, 32, 1))
    assert _blocks_met(driver._carried_cells(fine, 32, 1), 32, 2) == _blocks_met(parents, 32, 3)
    assert len(driver.carried_tags(np.zeros((0, 3), np.int32), 32)) == 0
    m = driver.merge_tags(fine[:3], fine[:1])
    assert len(m) == 4


def test_carried_tags_of_many_fine_tags_are_fast():
    import time
    rng = np.random.default_rng(4)
    fine = rng.integers(0, 1024, (20_000_000, 3), dtype=np.int32)
    t0 = time.perf_counter()
    c = driver.carried_tags(fine, 512)
    assert time.perf_counter() - t0 < 20.0
    assert c.shape[1] == 3 and len(c) <= (512 // 4) ** 3


@pytest.mark.parametrize("carry", [False, True, "library"])
def test_a_level_one_tag_keeps_its_refinement_only_when_carried(carry):
    t1, l1, l2 = _rebuild(carry)
    assert not check_layout(l1, 2 * M0, np.ones((M0,) * 3, bool), BF, MAX_BOX)
    l1_valid = boxes_mask(l1, 2 * M0)
    if l2:
        assert not check_layout(l2, 4 * M0, l1_valid, BF, MAX_BOX)
    refined = coarsen_mask(boxes_mask(l2, 4 * M0)) if l2 else np.zeros((2 * M0,) * 3, bool)
    # every tagged level-1 cell and its buffer refined by level 2
    want = np.zeros((2 * M0,) * 3, bool)
    for x, y, z in t1:
        want[(z - NBUF):(z + NBUF + 1), (y - NBUF):(y + NBUF + 1), (x - NBUF):(x + NBUF + 1)] = True
    covered = bool(np.all(refined[want]))
    assert covered == bool(carry)


def _random_layout(rng, M, n):
    """n boxes of whole blocking-factor blocks, disjoint (first come first kept)."""
    occ = np.zeros((M // BF,) * 3, bool)
    out = []
    for _ in range(50 * n):
        if len(out) == n:
            break
        lo = rng.integers(0, M // BF, 3)
        sz = rng.integers(1, 5, 3)
        hi = np.minimum(lo + sz, M // BF)
        if occ[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].any():
            continue
        occ[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
        out.append(tuple(int(v) for v in np.concatenate([lo * BF, hi * BF - 1])))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_carried_inside_the_clustering_equals_the_carried_list(seed):
    # the library marks the blocks met by the fine tags' grown parents itself: the boxes
    # must equal those of clustering the level's tags joined by carried_tags (whose block
    # set is pinned by brute force above), on level 0 and on a refined level, with tags
    # at the periodic ends and fine tags far from and next to the level's own tags
    rng = np.random.default_rng(seed)
    for M, level in ((32, [(0, 0, 0, 31, 31, 31)]), (64, None)):
        if level is None:
            level = _random_layout(rng, M, 12)
        valid = boxes_mask(level, M)
        cells = np.argwhere(valid)[:, ::-1].astype(np.int32)          # (x, y, z)
        tags = cells[rng.choice(len(cells), min(len(cells), 40), replace=False)]
        fine = rng.integers(0, 2 * M, (60, 3), dtype=np.int32)
        fine = np.concatenate([fine, 2 * tags[:10] + 1, np.array([[0, 0, 0], [2 * M - 1] * 3], np.int32)])
        for eff in (0.5, 0.7, 0.9):
            want = shamr.cluster_boxes(M, level, driver.merge_tags(tags, driver.carried_tags(fine, M)), BF,
                                       MAX_BOX, NBUF, eff)
            got = shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF, eff, carried=fine)
            assert got == want, (M, eff)
        assert shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF, carried=fine[:0]) == \
            shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF)


def test_carried_cells_outside_the_finer_level_are_refused():
    level0 = [(0, 0, 0, M0 - 1, M0 - 1, M0 - 1)]
    for bad in ([2 * M0, 0, 0], [0, -1, 0]):
        with pytest.raises(shamr.ShError):
            shamr.cluster_boxes(M0, level0, _blob((1, 1, 1), (2, 2, 2)), BF, MAX_BOX, NBUF,
                                carried=np.array([bad], np.int32))
    with pytest.raises(shamr.ShError):
        shamr.cluster_boxes(M0, level0, _blob((1, 1, 1), (2, 2, 2)), BF, MAX_BOX, NBUF,
                            carried=_blob((1, 1, 1), (2, 2, 2)), grow=-1)


def _blob_tags(rng, M, n):
    blobs = [np.floor(c + rng.normal(0, M / 16, (n // 4, 3))).astype(np.int64) % M
             for c in rng.integers(0, M, (4, 3))]
    faces = np.array([[0, 5, 7], [M - 1, 5, 7], [3, 0, M - 1], [M - 1, M - 1, M - 1], [0, 0, 0]])
    run = np.stack([np.arange(M), np.full(M, 9), np.full(M, M - 2)], 1)
    tags = np.unique(np.concatenate(blobs + [faces, run]), axis=0).astype(np.int32)
    return tags[np.lexsort((tags[:, 0], tags[:, 1], tags[:, 2]))]


def _one_by_one(fn):
    import os
    os.environ["SHAMR_DENSE_MARKING"] = "0"
    try:
        return fn()
    finally:
        del os.environ["SHAMR_DENSE_MARKING"]


@pytest.mark.parametrize("M,seed", [(256, 0), (256, 1), (512, 2)])
def test_long_tag_lists_mark_the_same_blocks(M, seed):
    # from one tag per 32 blocks on, a level's own tags are marked through octant bitsets;
    # marking them one by one (the dense form switched off) gives the same boxes, on the
    # whole domain and on a refined layout, with tags on the periodic faces and in runs;
    # long carried lists (marked one by one) equal clustering numpy's carried cell list
    rng = np.random.default_rng(seed)
    nb = M // (BF // 2)
    tags = _blob_tags(rng, M, nb ** 3 // 32 + 500)
    fine = _blob_tags(rng, 2 * M, nb ** 3 // 32 + 500)
    assert len(tags) >= nb ** 3 // 32 and len(fine) >= nb ** 3 // 32
    few = tags[::97]
    for level in ([(0, 0, 0, M - 1, M - 1, M - 1)], _random_layout(rng, M, 40)):
        own = shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF, 0.7)
        assert own == _one_by_one(lambda: shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF, 0.7))
        car = shamr.cluster_boxes(M, level, few, BF, MAX_BOX, NBUF, 0.7, carried=fine)
        assert car == _one_by_one(lambda: shamr.cluster_boxes(M, level, few, BF, MAX_BOX, NBUF, 0.7, carried=fine))
        joined = driver.merge_tags(few, driver.carried_tags(fine, M))
        assert car == _one_by_one(lambda: shamr.cluster_boxes(M, level, joined, BF, MAX_BOX, NBUF, 0.7))
        assert own or level[0][3] != M - 1


def _octants_of(cells, M, r, halve=False):
    """Octant bitsets (8, nwords) of tagged cells: the bit of each cell's block (of its
    parent's, halved) in every octant its cube [c - r, c + r] reaches (per axis: -1 when
    the offset in the block is < r, +1 when offset + r >= b)."""
    b = BF // 2
    nb = M // b
    nw = shamr.block_words(M, BF)
    flat = np.zeros((8, nw * 64), bool)
    for c in np.asarray(cells).reshape(-1, 3):
        c = c >> 1 if halve else c
        opts = [[s for s, ok in ((0, v % b < r), (1, v % b + r >= b)) if ok] for v in c]
        k = (c[2] // b * nb + c[1] // b) * nb + c[0] // b
        for ox in opts[0]:
            for oy in opts[1]:
                for oz in opts[2]:
                    flat[ox | oy << 1 | oz << 2, k] = True
    return np.packbits(flat, axis=1, bitorder="little").view(np.uint64)


@pytest.mark.parametrize("M,seed", [(64, 0), (64, 1), (256, 2)])
def test_octant_bitsets_grown_cluster_like_tag_lists(M, seed):
    # the host half of block tagging: octant bitsets of a level's own tags (grown by 2)
    # and of carried fine tags (parents grown by 3), each grown by one block towards its
    # octant and ORed, cluster into the boxes of the tag lists (rows of whole words at
    # 256, set bit by set bit at 64), on level 0 and on a refined layout
    rng = np.random.default_rng(20 + seed)
    for level in ([(0, 0, 0, M - 1, M - 1, M - 1)], _random_layout(rng, M, 12)):
        valid = np.argwhere(boxes_mask(level, M))[:, ::-1].astype(np.int32)
        tags = valid[rng.choice(len(valid), min(len(valid), 400), replace=False)]
        tags = np.concatenate([tags, valid[:3], valid[-3:]])
        fine = rng.integers(0, 2 * M, (300, 3), dtype=np.int32)
        fine = np.concatenate([fine, np.array([[0, 0, 0], [2 * M - 1] * 3], np.int32)])
        bits = shamr.dilate_octants(M, _octants_of(tags, M, NBUF), BF)
        assert shamr.cluster_boxes_bits(M, level, bits, BF, MAX_BOX) == shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF)
        shamr.dilate_octants(M, _octants_of(fine, M, 1 + NBUF, halve=True), BF, bits=bits)
        want = shamr.cluster_boxes(M, level, tags, BF, MAX_BOX, NBUF, carried=fine, grow=1)
        assert shamr.cluster_boxes_bits(M, level, bits, BF, MAX_BOX) == want
    nw = shamr.block_words(M, BF)
    assert shamr.cluster_boxes_bits(M, [(0, 0, 0, M - 1, M - 1, M - 1)], np.zeros(nw, np.uint64)) == []
    with pytest.raises(shamr.ShError):
        shamr.cluster_boxes_bits(M, [(0, 0, 0, M - 1, M - 1, M - 1)], np.zeros(nw - 1, np.uint64))
