"""The launch-shape autotuner times candidates on a twin: the tuned hierarchy's state and
step count do not move, and stepping with the chosen shape keeps the oracle's bits."""
import pytest

from oracle.level import run_single_level
from synth import random_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import autotune  # noqa: E402
from gpu_util import assert_bitwise, single_level  # noqa: E402


@pytest.mark.parametrize("prec", [shamr.SH_F64, shamr.SH_F32])
def test_autotune_leaves_state_and_keeps_parity(prec):
    n = 64
    U0 = random_state(n, float(n), 21)
    h = single_level(U0, prec=prec, beta=0)
    h.advance(0)
    h.advance(0)
    before = h.read_dense(0)
    cands = autotune.candidates(h.boxes[0])
    assert (8, 1, 0, 4, 0, 0, 5) in cands and (8, 1, 0, 4, 2, 0, 6) in cands
    times = autotune.tune(h, steps=2)
    assert len(times) == len(cands) and all(t > 0 for t in times.values())
    assert h.level_info(0)["k"] == 2
    assert_bitwise(h.read_dense(0), before, "state after tuning")
    for _ in range(3):
        h.advance(0)
    ref = run_single_level(U0.astype("float32") if prec == shamr.SH_F32 else U0, 5, 0.1, 0.25, 1.0, beta=0)
    assert_bitwise(h.read_dense(0), ref, f"5 steps with the tuned shape {next(iter(times))}")
    h.close()


def test_candidates_respect_the_footprints():
    boxes = [(0, 0, 0, 47, 47, 47)]          # 48 wide: only the 16 x 8 footprint divides it
    shapes = {c[4] for c in autotune.candidates(boxes) if c[3] == 4}
    assert shapes == {3}


def test_autotune_of_an_ssprk3_order2_level_keeps_parity():
    # the twin carries the hierarchy's numerics: a 13-point SSPRK3 level is tuned among
    # per-stage shapes only and still gives the oracle's bits
    n = 64
    U0 = random_state(n, float(n), 22)
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 0, max_level=0, integrator=10, lap_order=2)
    h.set_layout(0, [(0, 0, 0, n - 1, n - 1, n - 1)])
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    cands = autotune.candidates(h.boxes[0], h.params)
    assert all(c[3] == 0 for c in cands)
    autotune.tune(h, steps=1)
    for _ in range(3):
        h.advance(0)
    ref = run_single_level(U0, 3, 0.1, 0.25, 1.0, beta=0, integrator=10, order=2)
    assert_bitwise(h.read_dense(0), ref, "3 tuned SSPRK3 order-2 steps")
    h.close()
    p = shamr.Hierarchy(16, 16.0, integrator=10).params
    fused = [c for c in autotune.candidates([(0, 0, 0, 63, 63, 63)], p) if c[3] == 4]
    assert fused and not any(c[6] in (3, 6) for c in fused)
