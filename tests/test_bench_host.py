"""Host-side pieces of bench.py that need no GPU: the multi-core oracle baseline cuts the
lattice into z-slabs with extra planes and steps each slab with the oracle unchanged; the
kept planes must equal the whole-lattice oracle step bit for bit."""
import numpy as np
import pytest

import bench
from oracle.level import ko_coef, rk4_step, ssprk3_step
from synth import random_state


def _whole(U, integrator, order, ko_order, ko_eps):
    step = rk4_step if integrator == 4 else ssprk3_step
    ko = (ko_order, ko_coef(ko_order, ko_eps, 1.0)) if ko_order else None
    return step(U, 0.1, 0.25, 1.0, 2.0, 1.0, 2, order=order, ko=ko)


@pytest.mark.parametrize("integrator,order,ko_order,nslabs", [(4, 1, 0, 4), (10, 1, 0, 8), (4, 2, 3, 2)])
def test_slab_decomposition_equals_whole_lattice_step(integrator, order, ko_order, nslabs):
    U = random_state(16, 16.0, 3)
    ko_eps = 0.2 if ko_order else 0.0
    _, got = bench.oracle_step_slabs(U, nslabs, 1, integrator, order, ko_order, ko_eps, keep=True)
    ref = _whole(U, integrator, order, ko_order, ko_eps)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_slab_decomposition_in_worker_processes():
    U = random_state(16, 16.0, 4)
    _, got = bench.oracle_step_slabs(U, 4, 2, keep=True)
    assert np.array_equal(got, _whole(U, 4, 1, 0, 0.0))
    # the timed form returns one checksum per slab
    _, sums = bench.oracle_step_slabs(U, 4, 2)
    assert len(sums) == 4 and np.isfinite(sums).all()


def test_first_slab_only_and_host_description():
    U = random_state(16, 16.0, 5)
    _, one = bench.oracle_step_slabs(U, 8, 1, first_only=True, keep=True)
    assert np.array_equal(one, _whole(U, 4, 1, 0, 0.0)[:, :2])
    nproc, workers, model = bench.host_cpu()
    assert 1 <= workers <= min(nproc, 16) and isinstance(model, str) and model
