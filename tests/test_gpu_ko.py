"""GPU parity of Kreiss-Oliger dissipation (dissipation orders 2 and 3, on psi and Pi)
against the oracle, through the C-ABI: the right-hand side alone, single levels with both
integrators, every Laplacian order, ragged boxes and FP32 storage, and three-level
hierarchies with regrids whose fills carry Pi as deep as the dissipation stencil."""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier
from oracle.layout import block_layout
from oracle.level import ko_coef, rhs, run_single_level
from oracle.scalars import stage_scalars
from synth import random_state, string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise, decompose  # noqa: E402

EPS = 0.05


def _level(U0, ko, order=1, integrator=4, boxes=None, prec=shamr.SH_F64, beta=0):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=0, prec=prec, integrator=integrator,
                        lap_order=order, ko_order=ko, ko_eps=EPS)
    h.set_layout(0, boxes if boxes is not None else decompose(n))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


@pytest.mark.parametrize("ko,order", [(2, 1), (3, 1), (2, 2), (3, 3)])
def test_right_hand_side_bitwise(ko, order):
    n = 40
    U0 = random_state(n, float(n), 3)
    rng = np.random.default_rng(1)
    U0[2:] = 0.3 * rng.standard_normal(U0[2:].shape)     # Pi is stencilled too
    h = _level(U0, ko, order, boxes=decompose(n, [[8, 24], [16], [32]]))
    got = np.full((4, n, n, n), np.nan)
    for b, a in zip(h.boxes[0], h.eval_rhs(0)):
        got[:, b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = a
    _, cf, cp = stage_scalars(0.1, 0.25, 0, 2.0, 1.0, 0)
    assert_bitwise(got, rhs(U0, 1.0, cf, cp, order, (ko, ko_coef(ko, EPS, 1.0))), f"rhs ko {ko} order {order}")
    h.close()


@pytest.mark.parametrize("ko", [2, 3])
@pytest.mark.parametrize("integrator,order,prec,kind", [(4, 1, 0, 8), (10, 2, 0, 8), (4, 3, 1, 8), (10, 1, 1, 8),
                                                         (4, 3, 0, 4), (10, 1, 0, 4), (4, 2, 1, 0)])
def test_single_level_bitwise(ko, integrator, order, prec, kind):
    # boxes 64 wide run on block-row tiles of `kind` rows (psi and Pi staged through LDS),
    # the narrower ones on wave rows; kind 0 puts every box on wave rows
    n = 72
    U0 = random_state(n, float(n), 7)
    h = _level(U0, ko, order, integrator, boxes=decompose(n, [[64], [36], [40]]), prec=prec)
    h.set_tuning(kind=kind)
    h.profile(True)
    ref = run_single_level(U0.astype(np.float32) if prec else U0, 4, 0.1, 0.25, 1.0, beta=0, integrator=integrator,
                           order=order, ko_order=ko, ko_eps=EPS)
    for _ in range(4):
        h.advance(0)
    prof = h.profile_read()
    assert prof["fused_step"][1] == 0 and prof["stage1"][1] == 4
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), f"ko {ko} integrator {integrator} order {order}")
    h.close()


def _amr(ko, order, interp, integrator=4, prec=0):
    n = 24
    U0 = string_loop_state(n, float(n), seed=5, nloops=2, rmin=3.5, rmax=4.5, taper_in=2.0, taper_out=7.0)
    hg = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 0, max_level=2, prec=prec, max_box=32,
                         integrator=integrator, lap_order=order, interp=interp, ko_order=ko, ko_eps=EPS)
    hg.set_layout(0, decompose(n))
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    ho = OHier(n, float(n), 0.25, 0.1, 2, beta=0, dtype=np.float64 if prec == 0 else np.float32,
               integrator=integrator, order=order, interp=interp, ko_order=ko, ko_eps=EPS)
    ho.set_level0(U0)
    return hg, ho


def _regrid(hg, ho):
    for lev in range(ho.max_level):
        if lev >= len(ho.levels):
            break
        to = ho.tags(lev)
        assert np.array_equal(hg.tag_mask_dense(lev), to), f"tags differ on level {lev}"
        boxes = block_layout(to, ho.levels[lev].valid, 8, 32, 2)
        ho.set_layout(lev + 1, boxes)
        hg.set_layout(lev + 1, boxes)
        if not boxes:
            break


@pytest.mark.parametrize("ko,order,interp,integrator,prec", [(2, 1, 1, 4, 0), (3, 2, 4, 10, 0), (2, 1, 4, 4, 1)])
def test_three_level_hierarchy_with_regrids(ko, order, interp, integrator, prec):
    hg, ho = _amr(ko, order, interp, integrator, prec)
    _regrid(hg, ho)
    assert len(ho.levels) == 3
    for step in range(4):
        driver.coarse_step(hg)
        ho.coarse_step()
        for lev, L in enumerate(ho.levels):
            v = L.valid
            assert_bitwise(hg.read_dense(lev)[:, v], L.U.astype(np.float64)[:, v], f"step {step + 1} level {lev}")
        if step % 2 == 1:
            _regrid(hg, ho)
    hg.close()


def test_parameters_are_validated():
    for kw in ({"ko_order": 1, "ko_eps": 0.1}, {"ko_order": 2, "ko_eps": -1.0}, {"ko_order": 2, "ko_eps": np.inf}):
        with pytest.raises(shamr.ShError):
            shamr.Hierarchy(16, 16.0, **kw)
    U0 = random_state(32, 32.0, 1)
    h = _level(U0, 2)
    with pytest.raises(shamr.ShError):
        shamr.Batch([h])
    h.close()
