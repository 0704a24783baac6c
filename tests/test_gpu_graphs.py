"""Recorded level steps (HIP graphs): every replay must give the same bits as issuing the
same steps eagerly, with eager work and synchronisations between the replays; calls that
cannot be recorded are refused during a capture; a graph refuses to run once the layout
it recorded has changed."""
import numpy as np
import pytest

from oracle.layout import block_layout
from oracle.tagging import tag_cells
from synth import random_state, string_loop_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import driver, serve  # noqa: E402
from gpu_util import assert_bitwise, decompose, single_level  # noqa: E402


def _levels(h):
    return [h.read_dense(lev) for lev in range(h.num_levels())]


def _side_stream():
    # a capture needs a stream other than the legacy default stream
    import torch
    return torch.cuda.Stream()


def _level(U0, stream, boxes=None, prec=shamr.SH_F64, beta=0):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=0, prec=prec, stream=stream)
    h.set_layout(0, boxes if boxes is not None else decompose(n))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


@pytest.mark.parametrize("prec,cuts", [(shamr.SH_F64, None), (shamr.SH_F32, None),
                                       (shamr.SH_F64, [[32], [16, 40], None])])
def test_single_level_graph_replays_match_eager(prec, cuts):
    n = 64
    U0 = random_state(n, float(n), 11)
    boxes = decompose(n, [c if c is not None else [] for c in cuts]) if cuts else None
    st = _side_stream()
    eager = _level(U0, st, boxes=boxes, prec=prec)
    rec = _level(U0, st, boxes=boxes, prec=prec)
    with rec.capture() as c:
        for _ in range(3):
            rec.advance(0)
    assert rec.level_info(0)["k"] == 0          # recorded, not run
    assert_bitwise(rec.read_dense(0), eager.read_dense(0), "state untouched by the capture")
    for r in range(4):
        c.graph.launch()
        for _ in range(3):
            eager.advance(0)
        eager.sync()
        rec.sync()
        assert rec.level_info(0)["k"] == 3 * (r + 1)
        assert_bitwise(rec.read_dense(0), eager.read_dense(0), f"replay {r}")
        # eager work between replays: an energy reduction and a read of the state
        assert rec.energy()[0] == eager.energy()[0]
    c.graph.close()
    eager.close()
    rec.close()


def _amr_pair(n=32, beta=0):
    U0 = string_loop_state(n, float(n), 3, nloops=2, rmin=4.0, rmax=6.0, taper_in=2.0, taper_out=8.0)
    hs = []
    st = _side_stream()
    for _ in range(2):
        h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, beta, max_level=2, stream=st)
        h.set_layout(0, [(0, 0, 0, n - 1, n - 1, n - 1)])
        h.write_dense(0, U0)
        h.fill_ghosts(0)
        hs.append(h)
    # the same layout for both, from the oracle's tags of the initial coarse field
    tags = tag_cells(U0[0], U0[1])
    valid = np.ones((n, n, n), bool)
    boxes = block_layout(tags, valid, 8, 32, 2)
    assert boxes
    for h in hs:
        h.set_layout(1, boxes)
    return hs


def test_amr_coarse_step_graph_replays_match_eager():
    eager, rec = _amr_pair()
    with rec.capture() as c:
        driver.coarse_step(rec)
    for r in range(3):
        c.graph.launch()
        driver.coarse_step(eager)
        eager.sync()
        rec.sync()
        for lev in range(eager.num_levels()):
            assert rec.level_info(lev) == eager.level_info(lev)
        for lev, (a, b) in enumerate(zip(_levels(rec), _levels(eager))):
            assert_bitwise(a, b, f"replay {r} level {lev}")
        # eager level steps between replays keep both in lockstep
        driver.coarse_step(rec)
        driver.coarse_step(eager)
    c.graph.close()
    for lev, (a, b) in enumerate(zip(_levels(rec), _levels(eager))):
        assert_bitwise(a, b, f"after mixed eager/replayed steps, level {lev}")
    eager.close()
    rec.close()


def test_capture_refuses_unrecordable_calls_and_stale_layouts():
    n = 32
    U0 = random_state(n, float(n), 2)
    st = _side_stream()
    h = _level(U0, st)
    # calls that would synchronise, read back or upload are refused before they touch
    # the device (those that allocate device memory are not tried: an allocation would
    # end the capture)
    with h.capture() as c:
        h.advance(0)
        for call in (h.energy, h.sync, lambda: h.tag(0), lambda: h.profile(True), lambda: h.stage_scalars(0, 1),
                     lambda: h.set_tuning()):
            with pytest.raises(shamr.ShError):
                call()
        with pytest.raises(shamr.ShError):
            h.capture().__enter__()               # no nested capture
        h.advance(0)
    assert h.level_info(0)["k"] == 0
    c.graph.launch()
    h.sync()
    assert h.level_info(0)["k"] == 2
    ref = _level(U0, st)
    ref.advance(0)
    ref.advance(0)
    assert_bitwise(h.read_dense(0), ref.read_dense(0), "two recorded steps")
    h.set_layout(0, decompose(n, [[16], [], []]))   # new layout: the graph is stale
    with pytest.raises(shamr.ShError):
        c.graph.launch()
    c.graph.close()
    h.close()
    ref.close()
    # the legacy default stream cannot be captured
    h0 = single_level(U0, beta=0)
    with pytest.raises(shamr.ShError):
        h0.capture().__enter__()
    h0.close()


def test_batch_capture_replays_match_solo_runs():
    import torch
    stream = torch.cuda.Stream()
    jobs = []
    for i, n in enumerate((32, 48, 64)):
        j = serve.Job(jid=i, n=n, steps=10, prec=shamr.SH_F64, seed=40 + i, arrival=0.0, beta=0)
        j.U0 = random_state(n, float(n), j.seed)
        jobs.append(j)
    hs = [serve.make_hierarchy(j, stream) for j in jobs]
    b = shamr.Batch(hs)
    g = b.capture(5)
    assert all(h.level_info(0)["k"] == 0 for h in hs)
    g.launch()
    stream.synchronize()
    b.advance()                                   # an eager batch step between replays
    g.launch()
    stream.synchronize()
    for j, h in zip(jobs, hs):
        assert h.level_info(0)["k"] == 11
        j.steps = 11
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(h.read_dense(0), solo, f"job {j.jid}")
    g.close()
    b.close()
    for h in hs:
        h.close()
