"""GPU parity of the higher-order Laplacians (appendix A orders 2 and 3: the 13- and
19-point stencils) against the oracle, through the C-ABI: the right-hand side alone, single
levels under every per-stage launch shape with ragged boxes, both integrators, FP32
storage, and a three-level hierarchy with regrids whose refined levels carry ghost shells
as deep as the stencil (the paper's minimal example: order 2 with SSPRK3 type 10 and
truncation-error tagging)."""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier
from oracle.layout import block_layout
from oracle.level import rhs, run_single_level
from oracle.scalars import stage_scalars
from synth import random_state, string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise, decompose  # noqa: E402


def _level(U0, order, integrator=4, boxes=None, prec=shamr.SH_F64, beta=0, **kw):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=0, prec=prec, integrator=integrator,
                        lap_order=order, **kw)
    h.set_layout(0, boxes if boxes is not None else decompose(n))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


@pytest.mark.parametrize("order", [2, 3])
def test_right_hand_side_bitwise(order):
    n = 40
    U0 = random_state(n, float(n), 3)
    h = _level(U0, order, boxes=decompose(n, [[8, 24], [16], [32]]))
    got = np.full((4, n, n, n), np.nan)
    for b, a in zip(h.boxes[0], h.eval_rhs(0)):
        got[:, b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = a
    _, cf, cp = stage_scalars(0.1, 0.25, 0, 2.0, 1.0, 0)
    assert_bitwise(got, rhs(U0, 1.0, cf, cp, order), f"rhs order {order}")
    h.close()


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("integrator", [4, 10])
@pytest.mark.parametrize("kind,nt,zc,n,cuts", [(8, 1, 0, 96, [[64], [36], [50]]), (4, 0, 8, 64, [[32], [16, 40], []]),
                                               (0, 1, 0, 40, [[8, 16], [24], [8]]), (8, 1, 7, 72, [[64], [], [40]])])
def test_single_level_launch_shapes_bitwise(order, integrator, kind, nt, zc, n, cuts):
    U0 = random_state(n, float(n), 7)
    h = _level(U0, order, integrator, boxes=decompose(n, cuts))
    h.set_tuning(kind, nt, zc)
    h.profile(True)
    ref = run_single_level(U0, 4, 0.1, 0.25, 1.0, beta=0, integrator=integrator, order=order)
    for _ in range(4):
        h.advance(0)
    prof = h.profile_read()
    assert prof["fused_step"][1] == 0 and prof["stage1"][1] == 4, "the fused step is the 7-point stencil's"
    assert_bitwise(h.read_dense(0), ref, f"order {order} integrator {integrator} kind {kind}")
    h.close()


@pytest.mark.parametrize("order", [2, 3])
def test_fp32_storage_and_literal_divergence(order):
    n = 48
    U0 = random_state(n, float(n), 9)
    h = _level(U0, order, prec=shamr.SH_F32, boxes=decompose(n, [[16], [32], []]))
    ref = run_single_level(U0.astype(np.float32), 6, 0.1, 0.25, 1.0, beta=0, order=order)
    for _ in range(6):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), f"FP32 order {order}")
    h.close()
    # the literal configuration (beta = 2) through its blow-up: NaN/Inf positions match
    U0 = random_state(32, 32.0, 4)
    h = _level(U0, order, beta=2)
    ref = run_single_level(U0, 60, 0.1, 0.25, 1.0, order=order)
    for _ in range(60):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref, f"literal order {order}")
    assert not np.all(np.isfinite(ref))
    h.close()


def _amr(n, order, integrator, prec=0, beta=0):
    U0 = string_loop_state(n, float(n), seed=5, nloops=2, rmin=3.5, rmax=4.5, taper_in=2.0, taper_out=7.0)
    hg = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=2, prec=prec, max_box=32,
                         integrator=integrator, lap_order=order)
    hg.set_layout(0, decompose(n))
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    ho = OHier(n, float(n), 0.25, 0.1, 2, beta=beta, dtype=np.float64 if prec == 0 else np.float32,
               integrator=integrator, order=order)
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


def _compare(hg, ho, what):
    assert hg.num_levels() == len(ho.levels)
    for lev, L in enumerate(ho.levels):
        v = L.valid
        assert_bitwise(hg.read_dense(lev)[:, v], L.U.astype(np.float64)[:, v], f"{what} level {lev}")


@pytest.mark.parametrize("order,integrator,prec", [(2, 10, 0), (3, 4, 0), (2, 4, 1)])
def test_three_level_hierarchy_with_deep_ghosts(order, integrator, prec):
    hg, ho = _amr(24, order, integrator, prec)
    _regrid(hg, ho)
    assert len(ho.levels) == 3
    for step in range(4):
        driver.coarse_step(hg)
        ho.coarse_step()
        _compare(hg, ho, f"coarse step {step + 1}")
        if step % 2 == 1:
            _regrid(hg, ho)
            _compare(hg, ho, f"regrid after step {step + 1}")
    np.testing.assert_allclose(hg.energy()[0], ho.energy(), rtol=1e-12 if prec == 0 else 1e-6)
    hg.close()


def test_minimal_example_configuration_with_estimates():
    # order 2, SSPRK3 (type 10), estimates with the shadow level, tagging by estimate
    hg, ho = _amr(24, 2, 10)
    crit = 1e-2
    hg.set_tee(True, crit, 1)
    ho.set_tee(True, crit, 1)
    _regrid(hg, ho)
    for rnd in range(2):
        hg.shadow_begin()
        ho.shadow_begin()
        hg.shadow_advance()
        ho.shadow_advance()
        for _ in range(2):
            driver.coarse_step(hg)
            ho.coarse_step()
        hg.shadow_end()
        ho.shadow_end()
        for lev in range(len(ho.levels)):
            assert_bitwise(hg.tee_dense(lev), ho.levels[lev].tee, f"estimate level {lev} round {rnd}")
        hg.set_tee(True, crit, 2)
        ho.set_tee(True, crit, 2)
        _regrid(hg, ho)
        _compare(hg, ho, f"after estimate-driven regrid {rnd}")
    hg.close()


def test_order_is_validated_and_batches_refuse_it():
    with pytest.raises(shamr.ShError):
        shamr.Hierarchy(16, 16.0, lap_order=4)
    U0 = random_state(32, 32.0, 1)
    h = _level(U0, 2)
    with pytest.raises(shamr.ShError):
        shamr.Batch([h])
    h.close()
