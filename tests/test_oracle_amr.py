"""Pins of the AMR oracle: interpolation identities, averaging, subcycling order and the
two-level full-coverage equivalence with a single fine level."""
import numpy as np
import pytest

from oracle.amr import (Hierarchy, average_down_arrays, boxes_mask, coarsen_mask, dilate,
                        interp_cells, schedule, time_interp)
from oracle.layout import block_layout, check_layout
from oracle.level import run_single_level
from oracle.tagging import tag_cells
from synth import gaussian_random_pair, state_from_psi, string_loop_state


def _fine_indices(Mf):
    f = np.arange(Mf)
    return [a.ravel() for a in np.meshgrid(f, f, f, indexing="ij")]


def test_interp_reproduces_linear_fields_exactly():
    Mc = 8
    I = np.arange(Mc, dtype=float)
    Z, Y, X = np.meshgrid(I, I, I, indexing="ij")
    a, b, c, d = 3.0, 2.0, -5.0, 7.0
    C = a + b * (X + 0.5) + c * (Y + 0.5) + d * (Z + 0.5)   # linear in the cell centre
    fz, fy, fx = _fine_indices(2 * Mc)
    inner = (fz >= 2) & (fz < 2 * Mc - 2) & (fy >= 2) & (fy < 2 * Mc - 2) & (fx >= 2) & (fx < 2 * Mc - 2)
    fz, fy, fx = fz[inner], fy[inner], fx[inner]
    got = interp_cells(C, fz, fy, fx)
    want = a + b * (fx + 0.5) / 2 + c * (fy + 0.5) / 2 + d * (fz + 0.5) / 2
    assert np.array_equal(got, want)


def test_interp_children_mean_equals_parent_and_average_down_inverts():
    rng = np.random.default_rng(0)
    Mc = 8
    C = rng.integers(-1000, 1000, size=(Mc, Mc, Mc)).astype(float)
    fz, fy, fx = _fine_indices(2 * Mc)
    F = interp_cells(C, fz, fy, fx).reshape(2 * Mc, 2 * Mc, 2 * Mc)
    assert np.array_equal(average_down_arrays(F), C)


def test_average_down_exact_on_integers_and_order():
    rng = np.random.default_rng(1)
    F = rng.integers(-2**20, 2**20, size=(8, 8, 8)).astype(float)
    A = average_down_arrays(F)
    want = F.reshape(4, 2, 4, 2, 4, 2).sum(axis=(1, 3, 5)) / 8.0
    assert np.array_equal(A, want)


def test_time_interp_endpoints_and_midpoint():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 4, 4))
    b = rng.standard_normal((4, 4, 4))
    assert np.array_equal(time_interp(a, b, 0.0), a)
    assert np.array_equal(time_interp(None, b, 1.0), b)
    ai = rng.integers(-100, 100, (4, 4, 4)).astype(float)
    bi = rng.integers(-100, 100, (4, 4, 4)).astype(float)
    assert np.array_equal(time_interp(ai, bi, 0.25), 0.75 * ai + 0.25 * bi)
    assert np.array_equal(time_interp(ai, bi, 0.5), (ai + bi) / 2)


def test_schedule_reproduces_fig2_numbering():
    # Fig. 2: 1D, two refinement levels, three-stage integrator; fine-level ghost fills at
    # 5, 7, 9, ..., synchronisations at 21, 38, 39, 39 operations in all.  Level-0 fills
    # are periodic copies, not fills from a coarse level, and are not numbered.
    ops = [o for o in schedule(2, 3) if not (o[0] == "fill" and o[1] == 0)]
    assert len(ops) == 39
    fills = [i + 1 for i, o in enumerate(ops) if o[0] == "fill"]
    syncs = [i + 1 for i, o in enumerate(ops) if o[0] == "sync"]
    stages = [i + 1 for i, o in enumerate(ops) if o[0] == "stage"]
    assert fills[:3] == [5, 7, 9]
    assert syncs == [21, 38, 39]
    assert stages[:4] == [1, 2, 3, 4]
    # stages per level: 3 on level 0, 2x3 on level 1, 4x3 on level 2
    per = {0: 0, 1: 0, 2: 0}
    for o in ops:
        if o[0] == "stage":
            per[o[1]] += 1
    assert per == {0: 3, 1: 6, 2: 12}


def _random_hier(n0, max_level, seed, dtype=np.float64, beta=2):
    p1, p2 = gaussian_random_pair(n0, float(n0), seed)
    h = Hierarchy(n0, float(n0), 0.25, 0.1, max_level, dtype=dtype, beta=beta)
    h.set_level0(state_from_psi(p1, p2))
    return h


def test_two_level_full_coverage_equals_single_fine_level():
    n0 = 8
    h = _random_hier(n0, 1, seed=4)
    M1 = 2 * n0
    # level 1 covers the whole periodic domain, split into 8 boxes
    boxes = [(x, y, z, x + 7, y + 7, z + 7) for z in (0, 8) for y in (0, 8) for x in (0, 8)]
    h.set_layout(1, boxes)
    assert not h.levels[1].ghost.any()
    U1 = h.levels[1].U.copy()
    for _ in range(3):
        h.coarse_step()
        assert np.array_equal(h.levels[0].U, np.stack([average_down_arrays(c) for c in h.levels[1].U]))
        assert h.time(0) == h.time(1)
    ref = run_single_level(U1, 6, 0.1, 0.125, 0.5)
    assert np.array_equal(h.levels[1].U, ref)
    assert M1 == h.levels[1].M


def test_amr_u1_rotation_commutes_bitwise_and_sync_times_align():
    n0 = 16
    h = _random_hier(n0, 2, seed=6, beta=0)
    h.set_layout(1, [(8, 8, 8, 23, 23, 15), (8, 8, 16, 15, 15, 23)])
    h.set_layout(2, [(20, 20, 20, 27, 27, 27)])

    def rot(U):
        return np.stack([-U[1], U[0], -U[3], U[2]])

    g = Hierarchy(n0, float(n0), 0.25, 0.1, 2, beta=0)
    g.set_level0(rot(h.levels[0].U))
    g.set_layout(1, h.levels[1].boxes)
    g.set_layout(2, h.levels[2].boxes)
    for _ in range(2):
        h.coarse_step()
        g.coarse_step()
    for lev in range(3):
        v = h.levels[lev].valid
        assert np.array_equal(rot(h.levels[lev].U)[:, v], g.levels[lev].U[:, v])
    assert h.time(0) == h.time(1) == h.time(2)


def test_vacuum_is_a_fixed_point_of_the_amr_step():
    n0 = 16
    h = Hierarchy(n0, float(n0), 0.25, 0.1, 2)
    U0 = np.zeros((4, n0, n0, n0))
    U0[0] = 1.0
    h.set_level0(U0)
    h.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    h.set_layout(2, [(24, 24, 24, 39, 39, 31)])
    h.coarse_step()
    h.coarse_step()
    for L in h.levels:
        assert np.all(L.U[0][L.valid] == 1.0) and np.all(L.U[1:][:, L.valid] == 0.0)


def _smooth_state(n, L):
    i = np.arange(n) * L / n
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    p1 = 0.5 * np.cos(2 * np.pi * X / L) + 0.3 * np.sin(2 * np.pi * (Y + Z) / L)
    p2 = 0.4 * np.sin(2 * np.pi * (X - Z) / L)
    return state_from_psi(p1, p2)


def test_amr_patch_converges_to_the_uniformly_fine_run():
    # free field, one refined patch vs a fully refined level 1, same physical time: the
    # difference comes from the coarse/fine boundary and must shrink with resolution
    # (linear interpolation leaves an O(1) truncation error in one cell layer, so the
    # expected rate is about first order)
    errs = []
    for n0 in (16, 32):
        L = 16.0
        U0 = _smooth_state(n0, L)
        q = n0 // 2
        res = []
        for boxes in ([(q, q, q, 3 * q - 1, 3 * q - 1, 3 * q - 1)], [(0, 0, 0, 2 * n0 - 1, 2 * n0 - 1, 2 * n0 - 1)]):
            h = Hierarchy(n0, L, 0.25, 0.1, 1, alpha=0.0, lam=0.0, beta=0)
            h.set_level0(U0)
            h.set_layout(1, boxes)
            for _ in range(n0 // 4):
                h.coarse_step()
            res.append(h.levels[1])
        v = res[0].valid
        errs.append(np.max(np.abs(res[0].U[:, v] - res[1].U[:, v])))
    assert errs[0] < 0.02 and errs[0] / errs[1] > 1.3, errs


def test_block_layout_is_proper_and_checker_rejects_bad_layouts():
    n0 = 32
    U = string_loop_state(n0, float(n0), seed=3, nloops=1, rmin=5.0, rmax=6.0,
                          taper_in=2.0, taper_out=9.0)
    tags = tag_cells(U[0], U[1])
    assert tags.sum() > 0
    cv = np.ones((n0,) * 3, bool)
    boxes = block_layout(tags, cv, 8, 16, 2)
    assert boxes
    assert check_layout(boxes, 2 * n0, cv, 8, 16, tags, 2) == []
    # a second level nested in the first
    v1 = coarsen_mask(boxes_mask(boxes, 2 * n0))
    assert v1.sum() > 0
    # misaligned / oversized / overlapping layouts are rejected
    assert check_layout([(4, 0, 0, 11, 7, 7)], 2 * n0, cv, 8, 16)
    assert check_layout([(0, 0, 0, 31, 7, 7)], 2 * n0, cv, 8, 16)
    assert check_layout([(0, 0, 0, 7, 7, 7), (0, 0, 0, 7, 7, 7)], 2 * n0, cv, 8, 16)
    # not nested: a level-2 box touching the edge of a level-1 patch
    lev1 = boxes_mask([(16, 16, 16, 31, 31, 31)], 2 * n0)
    assert check_layout([(32, 32, 32, 39, 39, 39)], 4 * n0, lev1, 8, 16)
    assert check_layout([(40, 40, 40, 47, 47, 47)], 4 * n0, lev1, 8, 16) == []
    # uncovered tags are reported
    assert check_layout(boxes[1:], 2 * n0, cv, 8, 16, tags, 2)


def test_dilate_periodic():
    m = np.zeros((8, 8, 8), bool)
    m[0, 0, 0] = True
    d = dilate(m, 1)
    assert d.sum() == 27 and d[7, 7, 7] and d[1, 1, 1]


def test_fp32_amr_step_runs_and_tracks_fp64():
    n0 = 16
    p1, p2 = gaussian_random_pair(n0, float(n0), 12, kmax_frac=0.25)
    U0 = state_from_psi(p1, p2)
    out = []
    for dt in (np.float64, np.float32):
        h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, beta=0, dtype=dt)
        h.set_level0(U0)
        h.set_layout(1, [(8, 8, 8, 23, 23, 23)])
        for _ in range(3):
            h.coarse_step()
        out.append(h.levels[1].U[:, h.levels[1].valid].astype(np.float64))
    assert np.max(np.abs(out[0] - out[1])) < 1e-5


@pytest.mark.parametrize("bad", ["outside", "overlap"])
def test_boxes_mask_rejects(bad):
    with pytest.raises(ValueError):
        if bad == "outside":
            boxes_mask([(0, 0, 0, 8, 7, 7)], 8)
        else:
            boxes_mask([(0, 0, 0, 3, 3, 3), (2, 2, 2, 5, 5, 5)], 8)
