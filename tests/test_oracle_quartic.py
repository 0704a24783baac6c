"""Pins of the oracle's quartic conservative interpolation (interpolation type 4 of
appendix E, the paper's default): the 1-D child weights against an independent solve of
the five-cell moment system, exactness on cell averages of separable quartics (and not
one degree higher), conservation, and a regrid that fills new fine cells exactly."""
import numpy as np
import pytest

from oracle.amr import Hierarchy, average_down_arrays, interp_cells, interp_support


def _moment_weights():
    """Child averages of the quartic with prescribed averages over cells -2..2 (unit
    width, centred at 0), as weights on those averages; solved here with numpy."""
    A = np.array([[((j + 0.5) ** (m + 1) - (j - 0.5) ** (m + 1)) / (m + 1) for m in range(5)] for j in range(-2, 3)])
    Ainv = np.linalg.inv(A)                               # coefficients = Ainv @ averages
    lo = np.array([(0.0 - (-0.5) ** (m + 1)) / (m + 1) * 2 for m in range(5)])
    hi = np.array([(0.5 ** (m + 1) - 0.0) / (m + 1) * 2 for m in range(5)])
    return lo @ Ainv, hi @ Ainv


def test_one_dimensional_weights_solve_the_moment_system():
    wl, wh = _moment_weights()
    Mc = 8
    for j in range(5):
        C = np.zeros((Mc, Mc, Mc))
        C[4, 4, 2 + j] = 1.0                              # unit average in x-cell 2+j (offset j-2)
        fx = np.array([8, 9])                             # the two x-children of coarse x-cell 4
        got = interp_cells(C, np.array([8, 8]), np.array([8, 8]), fx, kind=4)
        # along y and z the parent's own cell has weight 1 in both children
        assert np.allclose(got, [wl[j], wh[j]], atol=1e-15), (j, got)


def _prim(coef, x):
    """Antiderivative of sum_m coef[m] x^m."""
    return sum(c * x ** (m + 1) / (m + 1) for m, c in enumerate(coef))


def _cell_avgs(coef, n, h):
    e = np.arange(n + 1) * h
    return (_prim(coef, e[1:]) - _prim(coef, e[:-1])) / h


@pytest.mark.parametrize("deg,exact", [(4, True), (5, False)])
def test_separable_polynomial_cell_averages(deg, exact):
    rng = np.random.default_rng(deg)
    Mc, H = 12, 1.0
    px, py, pz = (rng.uniform(-1, 1, deg + 1) for _ in range(3))
    cx, cy, cz = (_cell_avgs(p, Mc, H) for p in (px, py, pz))
    fx_, fy_, fz_ = (_cell_avgs(p, 2 * Mc, H / 2) for p in (px, py, pz))
    C = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    want = fz_[:, None, None] * fy_[None, :, None] * fx_[None, None, :]
    idx = np.arange(4, 2 * Mc - 4)                        # parents 2..Mc-3: no periodic wrap
    fz, fy, fx = np.meshgrid(idx, idx, idx, indexing="ij")
    got = interp_cells(C, fz.ravel(), fy.ravel(), fx.ravel(), kind=4).reshape(fz.shape)
    err = np.max(np.abs(got - want[4:-4, 4:-4, 4:-4])) / np.max(np.abs(want))
    if exact:
        assert err < 1e-12, err
    else:
        assert err > 1e-6, err
    # linear conservative interpolation is exact only on linear data
    lin = interp_cells(C, fz.ravel(), fy.ravel(), fx.ravel(), kind=1).reshape(fz.shape)
    assert np.max(np.abs(lin - want[4:-4, 4:-4, 4:-4])) / np.max(np.abs(want)) > 1e-6


def test_children_average_to_the_parent():
    rng = np.random.default_rng(1)
    Mc = 8
    C = rng.standard_normal((Mc, Mc, Mc))
    f = np.arange(2 * Mc)
    fz, fy, fx = np.meshgrid(f, f, f, indexing="ij")
    F = interp_cells(C, fz.ravel(), fy.ravel(), fx.ravel(), kind=4).reshape(fz.shape)
    assert np.max(np.abs(average_down_arrays(F) - C)) < 1e-14


def test_support_is_the_five_cube():
    m = interp_support(np.array([9]), np.array([9]), np.array([9]), 16, kind=4)
    assert m.sum() == 125 and m[2:7, 2:7, 2:7].all()


def test_regrid_fills_new_cells_exactly_and_checks_the_wider_support():
    rng = np.random.default_rng(3)
    n0, L = 16, 16.0
    px, py, pz = (rng.uniform(-0.1, 0.1, 5) for _ in range(3))
    cx, cy, cz = (_cell_avgs(p, n0, 1.0) for p in (px, py, pz))
    fx_, fy_, fz_ = (_cell_avgs(p, 2 * n0, 0.5) for p in (px, py, pz))
    U0 = np.zeros((4, n0, n0, n0))
    U0[0] = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    h = Hierarchy(n0, L, 0.25, 0.1, 1, alpha=0.0, lam=0.0, beta=0, interp=4)   # free field: no overflow
    h.set_level0(U0)
    h.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    L1 = h.levels[1]
    want = fz_[:, None, None] * fy_[None, :, None] * fx_[None, None, :]
    assert np.max(np.abs(L1.U[0][L1.valid] - want[L1.valid])) < 1e-13 * np.max(np.abs(want))
    h.coarse_step()                                      # fills with the quartic run
    assert np.all(np.isfinite(L1.U[0][L1.valid]))
    # a level 2 whose quartic support leaves level 1 is refused
    with pytest.raises(ValueError):
        h.set_layout(2, [(18, 18, 18, 45, 45, 45)])
