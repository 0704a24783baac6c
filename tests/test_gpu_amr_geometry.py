"""GPU parity against the oracle at the box geometry of the AMR workloads.

The AMR workloads lay out refined levels with a blocking factor of 8 and boxes of up to
64^3 (section II.C clustering; appendix E "AMR parameters": blocking_factor, max_grid_size),
over a level 0 that advances with the fused step.  These cases reach that geometry on a
lattice the oracle finishes in seconds: level 0 is one 32^3 box (a multiple of every fused
footprint, so the fused step runs there), max_box is 64, and three levels are stepped:

* first on a hand-placed layout whose refined boxes are 64 cells wide and 16-32 cells
  deep in y and z (the block-row stage kernel runs on boxes at least 64 wide; one level-1
  box spans the periodic x range and so is its own x neighbour; boxes touch across faces,
  so same-level copies run between them);
* then, after one regrid, on layouts clustered by the library's Berger-Rigoutsos from the
  oracle's tags (boxes up to 48 x 40 x 32 here), each checked against the layout rules.

Every level is compared with the oracle bit for bit after every coarse step and after the
regrid; the tag masks that drive the regrid are compared bit for bit too.  Cases: FP64
and FP32 storage, RK4 and SSPRK3, level 0 on the fused and on the per-stage kernels, and
the 13-point Laplacian with Kreiss-Oliger dissipation (which level 0 runs per stage).
"""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier
from oracle.layout import check_layout
from synth import string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise  # noqa: E402

N0, BF, MAX_BOX, NBUF = 32, 8, 64, 2
# level 1 (64^3): a 64 x 32 x 32 box spanning x, a 16^3 box on its +y face, a 16 x 8 x 8 box
L1_BOXES = [(0, 8, 8, 63, 39, 39), (16, 40, 16, 31, 55, 31), (40, 48, 40, 55, 55, 47)]
# level 2 (128^3): a 64 x 32 x 24 box and a 16^3 box on its +x face, nested in the first
# level-1 box with the gap of half a blocking factor
L2_BOXES = [(16, 24, 24, 79, 55, 47), (80, 24, 24, 95, 39, 39)]

CASES = {
    "f64-rk4-fused": dict(prec=0, integrator=4),
    "f32-rk4-fused": dict(prec=1, integrator=4),
    "f64-ssprk3-fused": dict(prec=0, integrator=10),
    "f32-ssprk3-fused": dict(prec=1, integrator=10),
    "f64-rk4-per-stage": dict(prec=0, integrator=4, fuse=0),
    "f64-rk4-lap13-ko2": dict(prec=0, integrator=4, lap_order=2, ko_order=2, ko_eps=0.3),
}


def _initial():
    return string_loop_state(N0, float(N0), seed=7, nloops=2, rmin=5.0, rmax=7.0, taper_in=1.5, taper_out=8.5)


def _compare(hg, ho, what):
    assert hg.num_levels() == len(ho.levels), what
    for lev, L in enumerate(ho.levels):
        G = hg.read_dense(lev)
        v = L.valid
        assert_bitwise(G[:, v], L.U[:, v].astype(np.float64), f"{what}, level {lev}")
        assert hg.level_info(lev)["eta"] == ho.time(lev), what


def _regrid(hg, ho):
    """Tag every level below the finest allowed one, cluster the oracle's tags with the
    library's Berger-Rigoutsos and give the boxes to both sides (coarsest first)."""
    shapes = []
    for lev in range(ho.max_level):
        to = ho.tags(lev)
        tg = hg.tag_mask_dense(lev)
        assert np.array_equal(tg, to), f"tag masks of level {lev} differ in {np.count_nonzero(tg != to)} cells"
        z, y, x = np.nonzero(to)
        M = N0 << lev
        boxes = shamr.cluster_boxes(M, ho.levels[lev].boxes, np.stack([x, y, z], 1), BF, MAX_BOX, NBUF)
        errs = check_layout(boxes, 2 * M, ho.levels[lev].valid, BF, MAX_BOX, tags=to, n_error_buf=NBUF)
        assert not errs, errs
        ho.set_layout(lev + 1, boxes)
        hg.set_layout(lev + 1, boxes)
        shapes += [shamr.box_shape(b) for b in boxes]
        if not boxes:
            break
    return shapes


@pytest.mark.timeout(600)
@pytest.mark.parametrize("poison", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_three_levels_at_workload_geometry(case, poison):
    # with poison, every complete ghost fill is preceded by NaN in the shell it sets
    # (sh_set_debug): a ghost read but never written would show up as NaN here
    kw = dict(CASES[case])
    fuse = kw.pop("fuse", 4)
    prec = kw.pop("prec")
    U0 = _initial()
    dt = np.float64 if prec == 0 else np.float32
    ho = OHier(N0, float(N0), 0.25, 0.1, 2, beta=2, dtype=dt,
               integrator=kw.get("integrator", 4), order=kw.get("lap_order", 1),
               ko_order=kw.get("ko_order", 0), ko_eps=kw.get("ko_eps", 0.0))
    ho.set_level0(U0)
    hg = shamr.Hierarchy(N0, float(N0), 0.25, 0.1, 1.0, 2.0, 2, max_level=2, blocking_factor=BF,
                         max_box=MAX_BOX, n_error_buf=NBUF, prec=prec, **kw)
    hg.set_layout(0, [(0, 0, 0, N0 - 1, N0 - 1, N0 - 1)])
    if fuse != 4:
        hg.set_tuning(fuse=fuse)
    if poison:
        hg.set_debug(True)
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    for lev, boxes in ((1, L1_BOXES), (2, L2_BOXES)):
        assert not check_layout(boxes, N0 << lev, ho.levels[lev - 1].valid, BF, MAX_BOX)
        ho.set_layout(lev, boxes)
        hg.set_layout(lev, boxes)
    _compare(hg, ho, f"{case}: hand-placed layout")
    hg.profile(True)
    for step in range(4):
        if step == 2:
            shapes = _regrid(hg, ho)
            assert len(ho.levels) == 3, "the loops must keep two refined levels"
            # clustered boxes deeper than one blocking factor in y and z
            assert max(s[1] for s in shapes) > BF and max(s[0] for s in shapes) > BF
            _compare(hg, ho, f"{case}: after the regrid")
        driver.coarse_step(hg)
        ho.coarse_step()
        _compare(hg, ho, f"{case}: coarse step {step + 1}")
    prof = hg.profile_read()
    hg.profile(False)
    fused_launches = prof["fused_step"][1]
    if fuse == 4 and kw.get("lap_order", 1) == 1 and kw.get("ko_order", 0) == 0:
        assert fused_launches == 4, "level 0 must advance with the fused step"
    else:
        assert fused_launches == 0
    e, _ = hg.energy()
    np.testing.assert_allclose(e, ho.energy(), rtol=1e-12 if prec == 0 else 1e-6)
    hg.close()


def test_poisoned_coarse_fine_ghosts_wait_for_the_synchronisation():
    # the second sub-step of a fine level ends with its same-level copy; its coarse/fine
    # ghosts are set by the synchronisation that follows, so in between they still hold
    # the debug poison while every same-level ghost and every valid cell is finite
    U0 = _initial()
    hg = shamr.Hierarchy(N0, float(N0), 0.25, 0.1, 1.0, 2.0, 2, max_level=1, blocking_factor=BF, max_box=MAX_BOX)
    hg.set_layout(0, [(0, 0, 0, N0 - 1, N0 - 1, N0 - 1)])
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    boxes = [(16, 16, 16, 31, 31, 31), (32, 16, 16, 47, 31, 31)]   # two boxes sharing a face
    hg.set_layout(1, boxes)
    hg.set_debug(True)
    hg.advance(0)
    hg.advance(1, 0)
    hg.advance(1, 1)
    g = hg.read_boxes(1, ghosts=True)
    for b, a in zip(boxes, g):
        psi = a[:2]
        assert np.all(np.isfinite(psi[:, 1:-1, 1:-1, 1:-1])), "valid cells"
        shared_x = 0 if b[0] == 32 else -1            # the face the two boxes share
        assert np.all(np.isfinite(psi[:, 1:-1, 1:-1, shared_x])), "same-level ghosts"
        assert np.isnan(psi[:, 1:-1, 1:-1, -1 - shared_x]).all(), "coarse/fine ghosts before the sync"
    hg.average_down(1)
    g = hg.read_boxes(1, ghosts=True)
    for a in g:
        assert np.all(np.isfinite(a[:2, 1:-1, 1:-1, :])) and np.all(np.isfinite(a[:2, :, 1:-1, 1:-1]))
    hg.close()

