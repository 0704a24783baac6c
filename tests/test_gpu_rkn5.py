"""GPU parity of RKN5 (integrator type 22, the friction-free EOM, single periodic levels)
against the oracle, bit for bit: the wave-row and block-row stage kernels with the 7- and
13-point Laplacians (appendix B's stencil) in FP64 and FP32 over enough steps to cycle the
three state slots, the stage times of the potential, recorded steps, and the refusals
(friction, dissipation, refined levels, the shadow level, batching)."""
import numpy as np
import pytest

from oracle.level import run_single_level
from synth import random_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from gpu_util import assert_bitwise, decompose  # noqa: E402


def _level(U0, boxes, prec=0, order=1, beta=2, eta0=0.1, stream=None):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, eta0, 1.0, 0.0, beta, max_level=0, prec=prec, integrator=22,
                        lap_order=order, stream=stream)
    h.set_layout(0, boxes)
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


@pytest.mark.parametrize("prec,order,n,cuts", [
    (0, 1, 32, [[8, 16], [24], [8]]),     # wave-row tiles (boxes narrower than 64)
    (1, 1, 32, [[8, 16], [24], [8]]),
    (0, 2, 32, [[16], [8], [24]]),
    (1, 2, 32, [[16], [], [24]]),
    (0, 1, 64, None),                     # one 64^3 box: block-row tiles
    (1, 2, 64, [[], [32], []]),
])
def test_single_level_matches_the_oracle(prec, order, n, cuts):
    U0 = random_state(n, float(n), 13)
    h = _level(U0, decompose(n, cuts), prec, order)
    nsteps = 7                            # the slots cycle every three steps
    dt = np.float64 if prec == 0 else np.float32
    ref = run_single_level(U0.astype(dt), nsteps, 0.1, 0.25, 1.0, alpha=0.0, lam=1.0, beta=2, integrator=22,
                           order=order)
    for _ in range(nsteps):
        h.advance(0)
    assert_bitwise(h.read_dense(0), ref.astype(np.float64), f"RKN5 prec {prec} order {order} n {n}")
    assert h.level_info(0)["eta"] == 0.1 + nsteps * 0.25
    assert h.level_info(0)["k"] == nsteps
    h.close()


def test_recorded_steps_equal_eager_steps():
    import torch
    n = 32
    U0 = random_state(n, float(n), 4)
    eager = _level(U0, decompose(n, [[16], [], []]), eta0=0.3)
    rec = _level(U0, decompose(n, [[16], [], []]), eta0=0.3, stream=torch.cuda.Stream())
    with rec.capture() as c:
        for _ in range(3):
            rec.advance(0)
    for rep in range(2):
        c.graph.launch()
        for _ in range(3):
            eager.advance(0)
        assert_bitwise(rec.read_dense(0), eager.read_dense(0), f"replay {rep}")
    c.graph.close()
    ref = run_single_level(U0, 6, 0.3, 0.25, 1.0, alpha=0.0, lam=1.0, beta=2, integrator=22)
    assert_bitwise(eager.read_dense(0), ref, "six steps against the oracle")
    rec.close()
    eager.close()


def test_refusals():
    n = 16
    for kw in (dict(alpha=2.0), dict(ko_order=2, ko_eps=0.1), dict(max_level=1)):
        alpha = kw.pop("alpha", 0.0)
        with pytest.raises(shamr.ShError) as e:
            shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, alpha, 2, integrator=22, **kw)
        assert e.value.status == shamr.SH_EINVAL, kw
    h = _level(random_state(n, float(n), 2), decompose(n))
    with pytest.raises(shamr.ShError) as e:
        shamr.Batch([h])
    assert e.value.status == shamr.SH_EINVAL
    with pytest.raises(shamr.ShError) as e:
        h.shadow_begin()
    assert e.value.status == shamr.SH_EINVAL
    h.close()
