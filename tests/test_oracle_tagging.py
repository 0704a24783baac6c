"""Pins of the plaquette tagging oracle.

Straight strings with a known pierced-plaquette set, agreement of the crossing rule
with an independent wrapped-phase (atan2) sum, the sign flip under conjugation and
hand-built single vortices.
"""
import numpy as np
import pytest

from oracle.tagging import plaquette_windings, plaquette_windings_atan2, tag_cells
from synth import gaussian_random_pair, straight_strings, string_loop_state


@pytest.mark.parametrize("n,x0,y0", [(16, 3.37, 5.61), (32, 10.37, 21.61), (24, 0.5, 7.25)])
def test_straight_strings_pierced_set(n, x0, y0):
    p1, p2 = straight_strings(n, x0, y0)
    W = plaquette_windings(p1, p2)
    assert np.count_nonzero(W["x"]) == 0 and np.count_nonzero(W["y"]) == 0
    Wz = W["z"]
    # exactly four pierced xy plaquettes per z plane, at the cells bracketing the zeros
    assert np.all(np.count_nonzero(Wz, axis=(1, 2)) == 4)
    xs = sorted({int(np.floor(x0)) % n, int(np.floor(x0 + n / 2)) % n})
    ys = sorted({int(np.floor(y0)) % n, int(np.floor(y0 + n / 2)) % n})
    for z in range(n):
        yy, xx = np.nonzero(Wz[z])
        assert sorted(set(xx.tolist())) == xs and sorted(set(yy.tolist())) == ys
    # each pierced plaquette tags its 4 corners: 16 cells per plane
    tags = tag_cells(p1, p2)
    assert tags.sum() == 16 * n


def test_crossing_rule_matches_atan2_on_random_fields():
    p1, p2 = gaussian_random_pair(16, 16.0, seed=11)
    a = plaquette_windings(p1, p2)
    b = plaquette_windings_atan2(p1, p2)
    total = 0
    for n in "xyz":
        assert np.array_equal(a[n], b[n])
        assert np.all(np.abs(a[n]) <= 1)
        total += np.count_nonzero(a[n])
    assert total > 50          # a random field is full of strings


def test_string_loops_close_and_conjugation_flips_sign():
    U = string_loop_state(48, 48.0, seed=2, nloops=1, rmin=6.0, rmax=8.0, delta=0.0,
                          taper_in=3.0, taper_out=14.0)
    a = plaquette_windings(U[0], U[1])
    b = plaquette_windings_atan2(U[0], U[1])
    c = plaquette_windings(U[0], -U[1])
    for n in "xyz":
        assert np.array_equal(a[n], b[n])
        assert np.array_equal(c[n], -a[n])
    # a closed loop: the net flux through every lattice plane x = const vanishes
    for n, ax in (("x", 2), ("y", 1), ("z", 0)):
        assert np.all(a[n].sum(axis=tuple(i for i in range(3) if i != ax)) == 0)
    assert sum(np.count_nonzero(a[n]) for n in "xyz") > 20


def test_single_vortex_winding_sign():
    # z = (x - 0.5) + i (y - 0.5) on the 2x2 corner block, 1 elsewhere: the plaquette with
    # lower corner (0, 0) winds +1 (counter-clockwise); periodicity forces compensating
    # windings elsewhere, so every xy plane carries zero net winding
    n = 8
    i = np.arange(n, dtype=float)
    X = np.broadcast_to(i[None, None, :], (n, n, n))
    Y = np.broadcast_to(i[None, :, None], (n, n, n))
    p1 = np.where((X < 2) & (Y < 2), X - 0.5, 1.0)
    p2 = np.where((X < 2) & (Y < 2), Y - 0.5, 0.0)
    W = plaquette_windings(p1, p2)
    assert np.all(W["z"][:, 0, 0] == 1)
    assert np.all(W["z"].sum(axis=(1, 2)) == 0)
    assert np.count_nonzero(W["x"]) == 0 and np.count_nonzero(W["y"]) == 0
    Wc = plaquette_windings(p1, -p2)
    assert np.all(Wc["z"][:, 0, 0] == -1)
    t = tag_cells(p1, p2)
    assert np.all(t[:, :2, :2] == 1)


def test_origin_on_edge_counts_zero_and_zero_corner_rule():
    # corner values exactly 0 fall under the y <= 0 branch: a plaquette whose corners are
    # 0, 1, 1+i, i has the origin at a corner and is not pierced
    n = 4
    p1 = np.ones((n, n, n))
    p2 = np.zeros((n, n, n))
    p1[0, 0, 0] = 0.0
    W = plaquette_windings(p1, p2)
    for k in "xyz":
        assert np.count_nonzero(W[k]) == 0
