"""Local regrid on the host (no GPU): the library's box computation equals the oracle's on
random layouts and tags (box lists compared exactly, level by level through the nesting
expansion), bad inputs are refused, the driver lays changed levels out coarsest first,
and the local/global regrid policy follows its thresholds.

What the equality pins: the paper defines which cells a local regrid must add (every
tagged cell with its buffer refined, the coarser levels grown for nesting, nothing
removed) but not how added blocks are merged into boxes.  Those properties are pinned on
the oracle alone (tests/test_oracle_local_regrid.py: coverage, nesting, no removal,
periodic wrap); the merge order (x runs, then y, then z) is a choice made once for both
sides, so on box lists the equality below checks that the library implements that
choice, not the paper."""
import numpy as np
import pytest

from oracle.amr import boxes_mask
from oracle.layout import block_layout
from oracle.local_regrid import local_regrid as oracle_local_regrid
from oracle.tagging import tag_cells
from synth import string_loop_state

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402


def _library_local_regrid(level_boxes, n0, lev, tags, bf, nbuf, max_box):
    """The driver's composition of the two library calls, on plain box lists."""
    fine = lev + 1
    cur = level_boxes[fine] if fine < len(level_boxes) else []
    out = {}
    new = shamr.local_tag_boxes(n0 << fine, cur, tags, bf, nbuf, max_box)
    if new:
        out[fine] = new
        k = lev
        while new and k >= 1:
            new = shamr.local_nest_boxes(n0 << k, new, level_boxes[k], bf, max_box)
            if new:
                out[k] = new
            k -= 1
    return out


def _layouts(seed, n0=32, bf=8, max_box=32):
    U = string_loop_state(n0, float(n0), seed=seed, nloops=2, rmin=4.0, rmax=6.0, taper_in=2.0, taper_out=9.0)
    v0 = np.ones((n0,) * 3, dtype=bool)
    l1 = block_layout(tag_cells(U[0], U[1]).astype(bool), v0, bf, max_box, 2)
    v1 = boxes_mask(l1, 2 * n0)
    # a level 2 from a thinned-out tag set on level 1 (every 7th level-1 cell)
    t1 = np.zeros((2 * n0,) * 3, dtype=bool)
    t1.flat[::7] = True
    l2 = block_layout(t1 & v1, v1, bf, max_box, 1)
    return [[(0, 0, 0, n0 - 1, n0 - 1, n0 - 1)], l1, l2], v1


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("lev,nbuf", [(0, 2), (1, 1), (1, 3)])
def test_library_equals_oracle(seed, lev, nbuf):
    n0, bf, max_box = 32, 8, 32
    boxes, v1 = _layouts(seed, n0, bf, max_box)
    rng = np.random.default_rng(seed * 10 + lev)
    valid = np.ones((n0,) * 3, dtype=bool) if lev == 0 else v1
    cells = np.argwhere(valid)
    tags = cells[rng.choice(len(cells), 40, replace=False)][:, ::-1]      # (x, y, z)
    want = oracle_local_regrid(boxes, n0, lev, tags, bf, nbuf, max_box)
    got = _library_local_regrid(boxes, n0, lev, tags, bf, nbuf, max_box)
    assert got == want
    assert want, "the random tags should grow something"


def test_new_level_and_no_tags():
    n0 = 32
    boxes = [[(0, 0, 0, n0 - 1, n0 - 1, n0 - 1)]]
    tags = np.array([[5, 6, 7], [20, 21, 22]])
    assert _library_local_regrid(boxes, n0, 0, tags, 8, 2, 64) == oracle_local_regrid(boxes, n0, 0, tags, 8, 2, 64)
    assert shamr.local_tag_boxes(2 * n0, [], np.zeros((0, 3)), 8, 2, 64) == []


def test_bad_inputs_are_refused():
    with pytest.raises(shamr.ShError):
        shamr.local_tag_boxes(64, [(4, 0, 0, 19, 15, 15)], [(1, 1, 1)], 8, 2, 64)     # not block aligned
    with pytest.raises(shamr.ShError):
        shamr.local_tag_boxes(64, [], [(32, 1, 1)], 8, 2, 64)                       # tag outside
    with pytest.raises(shamr.ShError):
        shamr.local_nest_boxes(32, [(0, 0, 0, 7, 7, 7)], [(0, 0, 0, 9, 7, 7)], 8, 64)


class _Fake:
    """Stands in for shamr.Hierarchy (boxes, tags and layout calls only)."""

    class P:
        n0, blocking_factor, n_error_buf, max_box = 32, 8, 2, 64

    def __init__(self, boxes, tags):
        self.params = self.P()
        self.boxes = {k: list(v) for k, v in enumerate(boxes)}
        self._tags = tags
        self.calls = []

    def num_levels(self):
        return len(self.boxes)

    def tag(self, lev):
        t = np.asarray(self._tags.get(lev, np.zeros((0, 3))), np.int32)
        return len(t), t

    def set_layout(self, lev, boxes):
        self.calls.append(lev)
        self.boxes[lev] = list(boxes)


def test_driver_lays_out_coarsest_first_and_counts_cells():
    n0 = 32
    l1 = [(8, 8, 8, 39, 39, 39)]
    l2 = [(32, 32, 32, 47, 47, 47)]
    tags = {1: np.array([[37, 24, 24]])}
    h = _Fake([[(0, 0, 0, n0 - 1, n0 - 1, n0 - 1)], l1, l2], tags)
    added = driver.local_regrid(h, 2)
    want = oracle_local_regrid([[(0, 0, 0, 31, 31, 31)], l1, l2], n0, 1, tags[1], 8, 2, 64)
    assert h.calls == sorted(want)                               # level 1 before level 2
    for k, v in want.items():
        assert h.boxes[k][-len(v):] == v
        assert added[k] == sum((b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1) for b in v)


def test_regrid_policy():
    p = driver.RegridPolicy(eps_strong=0.10, eps_weak=0.05, max_local=3)
    p.after_global([1000, 400, 200])
    assert p.decide() == ("local", None)
    p.after_local({2: 8})                                        # 4 % on level 2
    assert p.decide() == ("local", None)
    p.after_local({1: 24, 2: 16})                                # level 1: 6 %, level 2: 12 %
    assert p.decide() == ("global", 1)                           # from the lowest level >= 5 %
    p.after_global([1000, 420, 230])
    p.after_local({})
    p.after_local({})
    assert p.decide() == ("local", None)
    p.after_local({})
    assert p.decide() == ("global", 1)                           # max_local consecutive local regrids
    q = driver.RegridPolicy()
    q.after_global([1000, 400])
    q.after_local({2: 64})                                       # a level that did not exist
    assert q.decide() == ("global", 2)
