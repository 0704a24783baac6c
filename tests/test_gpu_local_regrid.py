"""GPU parity of local regrids: a three-level hierarchy advanced with local regrids (the
driver's, through the C-ABI) against the oracle hierarchy regridded with the oracle's local
regrid on the same tags; layouts are compared exactly and states bit for bit, FP64 and
FP32, also with quartic interpolation; then a policy-driven run mixing local and global
regrids stays nested and finite."""
import numpy as np
import pytest

from oracle.amr import Hierarchy as OHier
from oracle.layout import block_layout, check_layout
from oracle.amr import boxes_mask
from oracle.local_regrid import local_regrid as oracle_local_regrid
from synth import string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver  # noqa: E402
from gpu_util import assert_bitwise, decompose  # noqa: E402


def _pair(prec=0, interp=1, n=24):
    U0 = string_loop_state(n, float(n), seed=5, nloops=2, rmin=3.5, rmax=4.5, taper_in=2.0, taper_out=7.0)
    hg = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 0, max_level=2, prec=prec, max_box=32,
                         n_error_buf=2, interp=interp)
    hg.set_layout(0, decompose(n))
    hg.write_dense(0, U0)
    hg.fill_ghosts(0)
    ho = OHier(n, float(n), 0.25, 0.1, 2, beta=0, dtype=np.float64 if prec == 0 else np.float32, interp=interp)
    ho.set_level0(U0)
    # the starting layout: a plain global one on both sides
    for lev in range(2):
        to = ho.tags(lev)
        boxes = block_layout(to, ho.levels[lev].valid, 8, 32, 2)
        ho.set_layout(lev + 1, boxes)
        hg.set_layout(lev + 1, boxes)
    return hg, ho


def _oracle_local(ho, bf=8, nbuf=2, max_box=32):
    for lev in range(ho.max_level):
        if lev >= len(ho.levels):
            break
        tags = np.argwhere(ho.tags(lev))[:, ::-1]
        boxes = [list(L.boxes) for L in ho.levels]
        add = oracle_local_regrid(boxes, ho.n0, lev, tags, bf, nbuf, max_box)
        for k in sorted(add):
            old = list(ho.levels[k].boxes) if k < len(ho.levels) else []
            ho.set_layout(k, old + add[k])


def _compare(hg, ho, what):
    assert hg.num_levels() == len(ho.levels), what
    for lev, L in enumerate(ho.levels):
        assert list(hg.boxes[lev]) == list(L.boxes), f"{what}: layouts differ on level {lev}"
        v = L.valid
        assert_bitwise(hg.read_dense(lev)[:, v], L.U.astype(np.float64)[:, v], f"{what} level {lev}")


@pytest.mark.parametrize("prec,interp", [(0, 1), (1, 1), (0, 4)])
def test_local_regrids_match_the_oracle(prec, interp):
    hg, ho = _pair(prec, interp)
    grown = 0
    for step in range(6):
        driver.coarse_step(hg)
        ho.coarse_step()
        _compare(hg, ho, f"coarse step {step + 1}")
        if step % 2 == 1:
            for lev in range(len(ho.levels)):
                assert np.array_equal(hg.tag_mask_dense(lev), ho.tags(lev)), f"tags differ on level {lev}"
            before = [len(L.boxes) for L in ho.levels]
            added = driver.local_regrid(hg, 2)
            _oracle_local(ho)
            grown += sum(added.values())
            assert [len(L.boxes) for L in ho.levels] >= before
            _compare(hg, ho, f"local regrid after step {step + 1}")
    assert grown > 0, "the moving loops should make the local regrids grow the levels"
    hg.close()


def test_policy_driven_run_stays_nested():
    hg, _ = _pair()
    policy = driver.RegridPolicy(eps_strong=0.10, eps_weak=0.05, max_local=2)
    policy.after_global([hg.level_info(k)["ncells"] for k in range(hg.num_levels())])
    kinds = []
    for step in range(8):
        driver.coarse_step(hg)
        if step % 2 == 1:
            kind, start = policy.decide()
            kinds.append(kind)
            if kind == "local":
                policy.after_local(driver.local_regrid(hg, 2))
            else:
                driver.regrid(hg, 2, start=start)
                policy.after_global([hg.level_info(k)["ncells"] for k in range(hg.num_levels())])
            for lev in range(1, hg.num_levels()):
                coarse = boxes_mask(hg.boxes[lev - 1], 24 << (lev - 1))
                assert check_layout(hg.boxes[lev], 24 << lev, coarse, 8, 64) == [], f"level {lev} after {kind}"
    assert "local" in kinds and "global" in kinds
    for lev in range(hg.num_levels()):
        assert np.all(np.isfinite(hg.read_dense(lev)[:, boxes_mask(hg.boxes[lev], 24 << lev)]))
    hg.close()
