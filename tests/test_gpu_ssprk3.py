"""GPU parity of the SSPRK3 integrator (integrator types 3 and 10: three stages, three
state buffers, no accumulator) against the oracle, through the C-ABI: stage scalars,
single levels under every per-stage launch shape and every fused-step shape and variant,
a three-level hierarchy with regrids in FP64 and FP32, the subcycling order of Fig. 2
(drawn for a three-stage integrator), truncation error estimates with the shadow level,
and recorded (graph) steps."""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier, schedule
from oracle.layout import block_layout
from oracle.level import run_single_level
from oracle.scalars import level_time, stage_scalars
from synth import random_state, string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise, decompose  # noqa: E402


def _level(U0, integrator=10, boxes=None, prec=shamr.SH_F64, beta=2, stream=None, **kw):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=0, prec=prec, stream=stream,
                        integrator=integrator, **kw)
    h.set_layout(0, boxes if boxes is not None else decompose(n))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


def test_device_stage_scalars():
    U0 = random_state(8, 8.0, 0)
    h = _level(U0, integrator=3)
    dt = 0.25
    for k in range(4):
        for s in range(3):
            got = h.stage_scalars(0, s)
            eta_s, cf, cp = stage_scalars(level_time(0.1, k, dt), dt, s, 2.0, 1.0, 2, integrator=3)
            assert got[:3] == [eta_s, cf, cp], (k, s)
            assert got[6] == dt
        with pytest.raises(shamr.ShError):
            h.stage_scalars(0, 3)
        h.advance(0)
    h.close()


@pytest.mark.parametrize("integrator", [3, 10])
@pytest.mark.parametrize("fuse", [4, 0])
def test_literal_64cube_bitwise(integrator, fuse):
    # the literal configuration (beta = 2, diverging) through its first 40 steps, fused and
    # per-stage, the whole lattice checked at a few steps (NaN/Inf positions included)
    U0 = random_state(64, 64.0, 1)
    h = _level(U0, integrator=integrator)
    h.set_tuning(fuse=fuse)
    ref = {}
    run_single_level(U0, 40, 0.1, 0.25, 1.0, integrator=integrator,
                     callback=lambda k, U: ref.__setitem__(k, U.copy()) if k in (1, 2, 3, 7, 40) else None)
    for k in range(1, 41):
        h.advance(0)
        if k in ref:
            assert_bitwise(h.read_dense(0), ref[k], f"step {k}")
    assert h.level_info(0)["k"] == 40
    h.close()


@pytest.mark.parametrize("kind,nt,zc,n,cuts", [(8, 1, 0, 64, None), (4, 0, 8, 64, [[32], [16, 40], []]),
                                               (0, 1, 0, 40, [[8, 16], [24], [8]]), (8, 1, 7, 72, [[64], [], [40]])])
def test_launch_shapes_and_ragged_boxes_bitwise(kind, nt, zc, n, cuts):
    U0 = random_state(n, float(n), 7)
    boxes = decompose(n, cuts) if cuts else None
    h = _level(U0, boxes=boxes, beta=0)
    h.set_tuning(kind, nt, zc, fuse=0)
    ref = run_single_level(U0, 7, 0.1, 0.25, 1.0, beta=0, integrator=10)
    for _ in range(7):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref, f"kind {kind} tile_z {zc}")
    h.close()


def test_fp32_storage_bitwise_with_fp32_oracle():
    n = 48
    U0 = random_state(n, float(n), 9)
    h = _level(U0, prec=shamr.SH_F32, beta=0, boxes=decompose(n, [[16], [32], []]))
    ref = run_single_level(U0.astype(np.float32), 9, 0.1, 0.25, 1.0, beta=0, integrator=10)
    for _ in range(9):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), "FP32 storage")
    h.close()


@pytest.mark.parametrize("variant", [0, 1, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("prec,shape,fzc,cuts", [(0, 0, 64, None), (0, 0, 7, [[32], [8, 40], []]),
                                                 (0, 1, 13, [[], [16], [40]]), (0, 2, 9, [[32], [16], [24]]),
                                                 (0, 3, 11, [[16], [8, 40], [24]]), (1, 2, 0, None),
                                                 (1, 0, 5, [[32], [24], [16, 40]])])
def test_fused_three_stage_step_bitwise(prec, shape, fzc, cuts, variant):
    # the fused step with the three SSPRK3 stages in one kernel must give the oracle's bits
    n = 64
    U0 = random_state(n, float(n), 6)
    h = _level(U0, prec=prec, beta=0, boxes=decompose(n, cuts) if cuts else None)
    h.set_tuning(8, 1, 0, fuse=4, fused_shape=shape, fused_tile_z=fzc, fused_variant=variant)
    h.profile(True)
    ref = run_single_level(U0.astype(np.float32) if prec else U0, 5, 0.1, 0.25, 1.0, beta=0, integrator=10)
    for _ in range(5):
        h.advance(0)
    prof = h.profile_read()
    assert prof["fused_step"][1] == 5 and prof["stage1"][1] == 0, prof
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), f"prec={prec} shape={shape} fzc={fzc} variant={variant}")
    h.close()


def test_stage_counts_and_batches_refuse_ssprk3():
    n = 32
    U0 = random_state(n, float(n), 2)
    h = _level(U0, beta=0)
    for fuse, want in ((4, (1, 0, 0, 0, 0)), (0, (0, 1, 1, 1, 0))):
        h.set_tuning(fuse=fuse)
        h.profile(True)
        h.advance(0)
        prof = h.profile_read()
        h.profile(False)
        got = tuple(prof[k][1] for k in ("fused_step", "stage1", "stage2", "stage3", "stage4"))
        assert got == want, (fuse, got)
    with pytest.raises(shamr.ShError):
        shamr.Batch([h])
    h.close()
    with pytest.raises(shamr.ShError):
        shamr.Hierarchy(n, float(n), integrator=5)


def _amr(n, integrator, prec=0, beta=0, stream=None):
    U0 = string_loop_state(n, float(n), seed=5, nloops=2, rmin=3.5, rmax=4.5, taper_in=2.0, taper_out=7.0)
    hg = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=2, prec=prec, max_box=32,
                         integrator=integrator, stream=stream)
    hg.set_layout(0, decompose(n))
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    ho = OHier(n, float(n), 0.25, 0.1, 2, beta=beta, dtype=np.float64 if prec == 0 else np.float32,
               integrator=integrator)
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
        assert hg.level_info(lev)["eta"] == ho.time(lev)


@pytest.mark.parametrize("prec,beta", [(0, 0), (0, 2), (1, 0)])
def test_three_level_hierarchy_with_regrids(prec, beta):
    hg, ho = _amr(24, 10, prec, beta)
    _regrid(hg, ho)
    assert len(ho.levels) == 3
    for step in range(5):
        driver.coarse_step(hg)
        ho.coarse_step()
        _compare(hg, ho, f"coarse step {step + 1}")
        if step % 2 == 1:
            _regrid(hg, ho)
            _compare(hg, ho, f"regrid after step {step + 1}")
    np.testing.assert_allclose(hg.energy()[0], ho.energy(), rtol=1e-12 if prec == 0 else 1e-6)
    hg.close()


def test_trace_follows_the_three_stage_schedule():
    hg, ho = _amr(24, 3)
    _regrid(hg, ho)
    hg.trace(True)
    driver.coarse_step(hg)
    rec = hg.trace_read()
    hg.trace(False)
    role_of = {1: 1, 2: 2, 3: 0}          # the stage-2 input A, the stage-3 input B, the new state
    frac = {1: 1.0, 2: 0.5, 3: 1.0}
    want = []
    for op in schedule(2, 3):
        if op[0] == "stage":
            want.append((1, op[1], op[2]))
        elif op[0] == "fill":
            _, lev, sub, s = op
            if lev > 0:
                want.append((3, lev, role_of[s], int(round(4 * (sub + frac[s]) / 2))))
        else:
            want += [(4, op[1], 0, 0), (3, op[1], 0, 4)]
    got = [(1, lev, a) if op == 1 else ((3, lev, a, b) if op == 3 else (4, lev, 0, 0))
           for op, lev, a, b in rec if op in (1, 3, 4)]
    assert got == want
    hg.close()


def test_estimates_with_the_shadow_level():
    hg, ho = _amr(24, 10)
    crit = 2e-2
    hg.set_tee(True, crit, 1)
    ho.set_tee(True, crit, 1)
    _regrid(hg, ho)
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
        assert_bitwise(hg.tee_dense(lev), ho.levels[lev].tee, f"estimate level {lev}")
    hg.set_tee(True, crit, 3)
    ho.set_tee(True, crit, 3)
    _regrid(hg, ho)
    _compare(hg, ho, "after an estimate-driven regrid")
    hg.close()


def test_recorded_coarse_steps_replay_like_eager_ones():
    import torch
    st = torch.cuda.Stream()
    eager, _ = _amr(24, 10, stream=st)
    rec, ho = _amr(24, 10, stream=st)
    _regrid(rec, ho)
    for lev in range(1, ho.finest + 1):
        eager.set_layout(lev, ho.levels[lev].boxes)
    with rec.capture() as c:
        driver.coarse_step(rec)
    for r in range(4):                      # more replays than the three-slot role cycle
        c.graph.launch()
        driver.coarse_step(eager)
        rec.sync()
        eager.sync()
        for lev in range(eager.num_levels()):
            assert rec.level_info(lev) == eager.level_info(lev)
            assert_bitwise(rec.read_dense(lev), eager.read_dense(lev), f"replay {r} level {lev}")
    c.graph.close()
    rec.close()
    eager.close()
