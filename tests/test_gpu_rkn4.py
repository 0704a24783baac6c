"""GPU parity of RKN4 (integrator type 21, the friction-free EOM) against the oracle, bit
for bit: single levels through the wave-row and block-row stage kernels with the 7- and
13-point Laplacians in FP64 and FP32, a three-level hierarchy with regrids and a shadow
level, and the refusal of friction, dissipation and batching."""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier
from oracle.layout import block_layout
from oracle.level import run_single_level
from synth import random_state, string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise, decompose  # noqa: E402


def _level(U0, boxes, prec=0, order=1, beta=2):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 0.0, beta, max_level=0, prec=prec, integrator=21,
                        lap_order=order)
    h.set_layout(0, boxes)
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


@pytest.mark.parametrize("prec,order,n,cuts", [
    (0, 1, 32, [[8, 16], [24], [8]]),     # wave-row tiles (boxes narrower than 64)
    (1, 1, 32, [[8, 16], [24], [8]]),
    (0, 2, 32, [[16], [8], [24]]),
    (0, 1, 64, None),                     # one 64^3 box: block-row tiles
    (1, 2, 64, [[], [32], []]),
])
def test_single_level_matches_the_oracle(prec, order, n, cuts):
    U0 = random_state(n, float(n), 11)
    h = _level(U0, decompose(n, cuts), prec, order)
    nsteps = 6
    dt = np.float64 if prec == 0 else np.float32
    ref = run_single_level(U0.astype(dt), nsteps, 0.1, 0.25, 1.0, alpha=0.0, lam=1.0, beta=2, integrator=21,
                           order=order)
    for _ in range(nsteps):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), f"RKN4 prec {prec} order {order} n {n}")
    assert h.level_info(0)["eta"] == 0.1 + nsteps * 0.25
    h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_three_levels_with_regrids_and_shadow(prec):
    n = 24
    U0 = string_loop_state(n, float(n), seed=5, nloops=2, rmin=3.5, rmax=4.5, taper_in=2.0, taper_out=7.0)
    dt = np.float64 if prec == 0 else np.float32
    hg = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 0.0, 2, max_level=2, prec=prec, max_box=32, integrator=21,
                         lap_order=2)
    hg.set_layout(0, decompose(n))
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    ho = OHier(n, float(n), 0.25, 0.1, 2, alpha=0.0, beta=2, dtype=dt, integrator=21, order=2)
    ho.set_level0(U0)

    def regrid():
        for lev in range(2):
            if lev >= len(ho.levels):
                break
            to = ho.tags(lev)
            assert np.array_equal(hg.tag_mask_dense(lev), to), f"tags differ on level {lev}"
            boxes = block_layout(to, ho.levels[lev].valid, 8, 32, 2)
            ho.set_layout(lev + 1, boxes)
            hg.set_layout(lev + 1, boxes)
            if not boxes:
                break

    def compare(what):
        assert hg.num_levels() == len(ho.levels)
        for lev, L in enumerate(ho.levels):
            v = L.valid
            assert_bitwise(hg.read_dense(lev)[:, v], L.U[:, v].astype(np.float64), f"{what}, level {lev}")
            assert hg.level_info(lev)["eta"] == ho.time(lev)

    regrid()
    assert len(ho.levels) == 3
    hg.set_tee(True, 1e-2, 3)
    ho.set_tee(True, 1e-2, 3)
    hg.shadow_begin()
    ho.shadow_begin()
    hg.shadow_advance()
    ho.shadow_advance()
    for step in range(4):
        driver.coarse_step(hg)
        ho.coarse_step()
        compare(f"coarse step {step + 1}")
        if step == 1:
            hg.shadow_end()
            ho.shadow_end()
            for lev in range(len(ho.levels)):
                assert_bitwise(hg.tee_dense(lev), ho.levels[lev].tee, f"estimate, level {lev}")
            regrid()
            compare("after the regrid")
    hg.close()


def test_friction_dissipation_and_batching_are_refused():
    n = 16
    with pytest.raises(shamr.ShError) as e:
        shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 2, integrator=21)
    assert e.value.status == shamr.SH_EINVAL
    with pytest.raises(shamr.ShError) as e:
        shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 0.0, 2, integrator=21, ko_order=2, ko_eps=0.1)
    assert e.value.status == shamr.SH_EINVAL
    h = _level(random_state(n, float(n), 2), decompose(n))
    with pytest.raises(shamr.ShError) as e:
        shamr.Batch([h])
    assert e.value.status == shamr.SH_EINVAL
    h.close()
