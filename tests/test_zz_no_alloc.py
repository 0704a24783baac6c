"""The allocation-free tagging entry point (sh_tag_cells_noalloc) against sh_tag_cells,
called through the C-ABI: the same count, list and mask on two calls in a row, the
second on a smaller level, and a capacity above its fixed maximum refused on the host."""
import ctypes

import numpy as np
import pytest

from synth import random_state, state_from_psi, straight_strings

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from gpu_util import decompose  # noqa: E402

CAP_MAX = 1 << 20


def _level(U0, boxes=None):
    n = U0.shape[-1]
    h = shamr.Hierarchy(n, float(n), 0.25, 0.1, 1.0, 2.0, 2, max_level=1)
    h.set_layout(0, boxes or decompose(n))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


def _call(fn, h, cap):
    torch = h.torch
    nv = h.level_info(0)["ncells"]
    mask = torch.zeros(nv, dtype=torch.uint8, device="cuda")
    idx = np.full((max(cap, 1), 3), -7, np.int32)
    n = ctypes.c_int64(-1)
    st = fn(h.h, 0, ctypes.c_void_p(mask.data_ptr()), idx.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n))
    return st, n.value, idx, mask.cpu().numpy()


def test_noalloc_tagging_matches_sh_tag_cells_twice():
    lib = shamr.load()
    big = _level(random_state(48, 48.0, 8), decompose(48, [[16, 24], [8], [40]]))
    p1, p2 = straight_strings(32, 10.37, 21.61)
    small = _level(state_from_psi(p1, p2))
    results = []
    for h in (big, small):
        st_ref, n_ref, idx_ref, m_ref = _call(lib.sh_tag_cells, h, 1 << 18)
        st, n, idx, m = _call(lib.sh_tag_cells_noalloc, h, 1 << 18)
        assert st_ref == shamr.SH_OK and st == shamr.SH_OK, shamr.load().sh_last_error()
        assert n == n_ref and n > 0
        assert np.array_equal(idx[:n], idx_ref[:n_ref])
        assert np.array_equal(m, m_ref)
        results.append(n)
    assert results[1] < results[0]
    assert results[1] == 16 * 32  # two straight strings pierce 16 plaquette corners per plane
    # a partial list: only the first cap entries are written
    st, n, idx, _ = _call(lib.sh_tag_cells_noalloc, small, 100)
    assert st == shamr.SH_OK and n == 16 * 32
    _, _, idx_ref, _ = _call(lib.sh_tag_cells, small, 1 << 18)
    assert np.array_equal(idx[:100], idx_ref[:100])
    big.close()
    small.close()


def test_noalloc_tagging_refuses_a_capacity_above_its_maximum():
    lib = shamr.load()
    p1, p2 = straight_strings(32, 10.37, 21.61)
    h = _level(state_from_psi(p1, p2))
    idx = np.empty((1, 3), np.int32)
    n = ctypes.c_int64(-1)
    st = lib.sh_tag_cells_noalloc(h.h, 0, None, idx.ctypes.data_as(ctypes.c_void_p), CAP_MAX + 1, ctypes.byref(n))
    assert st == shamr.SH_EINVAL
    assert b"allocation-free maximum" in lib.sh_last_error()
    h.close()
