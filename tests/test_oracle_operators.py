"""Pins of the oracle's higher-order Laplacians (appendix A, orders 2 and 3: the 13- and
19-point stencils) and of the ghost depth they need on refined levels: exactness on
polynomials up to the stencils' degree (and inexactness just above it), the plane-wave
eigenvalue in closed form, the convergence rate, the fully discrete free field, and a
refined level whose ghost cells (as deep as the stencil) must be interpolated at the
right times for it to stay exact."""
import numpy as np
import pytest

from oracle.amr import Hierarchy, ghost_mask, boxes_mask
from oracle.level import lap, lap7, run_single_level
from synth import plane_wave, state_from_psi


def _grid(n, origin=-4):
    i = np.arange(n, dtype=np.float64) + origin
    return np.meshgrid(i, i, i, indexing="ij")       # z, y, x in index units


@pytest.mark.parametrize("order,deg", [(2, 5), (3, 7)])
def test_exact_on_polynomials_up_to_the_stencil_degree(order, deg):
    # central differences of order 2p are exact for polynomials of degree <= 2p + 1
    n, r = 16, order
    z, y, x = _grid(n)
    u = x ** deg - 2 * y ** (deg - 1) + 3 * z ** (deg - 2) + x * y * z
    want = deg * (deg - 1) * x ** (deg - 2) - 2 * (deg - 1) * (deg - 2) * y ** (deg - 3) \
        + 3 * (deg - 2) * (deg - 3) * z ** (deg - 4)
    got = lap(u, 1.0, order)
    inner = (slice(r, -r),) * 3                        # away from the periodic wrap
    scale = np.max(np.abs(u[inner]))
    assert np.max(np.abs(got[inner] - want[inner])) < 1e-13 * scale * 10 ** order
    # one degree more is not exact: the leading error term of the stencil appears
    v = x ** (deg + 1)
    err = lap(v, 1.0, order)[inner] - (deg + 1) * deg * x[inner] ** (deg - 1)
    # leading error c * dx^(2p) * u^(2p+2) per axis: c = -1/90 (order 2), +1/560 (order 3)
    c = {2: -1.0 / 90.0, 3: 1.0 / 560.0}[order]
    fact = np.prod(np.arange(1, deg + 2, dtype=np.float64))   # (deg + 1)! = u^(deg+1)
    assert np.allclose(err, c * fact, rtol=1e-6), (err.min(), err.max(), c * fact)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_plane_wave_eigenvalue_closed_form(order):
    n, L = 24, 24.0 * 0.7
    dx = L / n
    k = 2 * np.pi / L * np.array([3.0, -5.0, 2.0])
    u = plane_wave(n, L, k)
    th = k * dx
    if order == 1:
        per_axis = 2 * (np.cos(th) - 1)
    elif order == 2:
        per_axis = (4 / 3) * 2 * (np.cos(th) - 1) - (1 / 12) * 2 * (np.cos(2 * th) - 1)
    else:
        per_axis = 1.5 * 2 * (np.cos(th) - 1) - 0.15 * 2 * (np.cos(2 * th) - 1) + (1 / 90) * 2 * (np.cos(3 * th) - 1)
    lam = np.sum(per_axis) / dx ** 2
    np.testing.assert_allclose(lap(u, 1.0 / dx ** 2, order), lam * u, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("order,rate", [(1, 4.0), (2, 16.0), (3, 64.0)])
def test_convergence_rate(order, rate):
    # error of the discrete Laplacian of sin(2 pi x / L) on refinement: 2^(2 order)
    L = 8.0
    errs = []
    for n in (16, 32):
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        u = np.broadcast_to(np.sin(2 * np.pi * x / L), (n, n, n)).copy()
        exact = -(2 * np.pi / L) ** 2 * u
        errs.append(np.max(np.abs(lap(u, 1.0 / dx ** 2, order) - exact)))
    assert abs(errs[0] / errs[1] / rate - 1) < 0.05, errs[0] / errs[1]


def test_order_one_is_the_seven_point_stencil():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((8, 8, 8))
    assert np.array_equal(lap(u, 2.5, 1), lap7(u, 2.5))


@pytest.mark.parametrize("order", [2, 3])
def test_free_field_fully_discrete_solution(order):
    # lambda = alpha = 0: one integer mode evolves by the RK4 step matrix of its eigenvalue
    n, L, dt = 16, 16.0, 0.2
    dx = L / n
    k = 2 * np.pi / L * np.array([1.0, 2.0, -3.0])
    cosk = plane_wave(n, L, k)
    w2 = -np.mean(lap(cosk, 1.0 / dx ** 2, order)[cosk > 0.5] / cosk[cosk > 0.5])
    A = np.array([[0.0, 1.0], [-w2, 0.0]]) * dt
    A2 = A @ A
    M = np.eye(2) + A + A2 / 2 + A2 @ A / 6 + A2 @ A2 / 24
    nsteps = 30
    a, b = np.linalg.matrix_power(M, nsteps) @ np.array([1.0, 0.0])
    U = run_single_level(state_from_psi(cosk, np.zeros_like(cosk)), nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0,
                         beta=0, order=order)
    np.testing.assert_allclose(U[0], a * cosk, atol=1e-11)
    np.testing.assert_allclose(U[2], b * cosk, atol=1e-11 * np.sqrt(w2))


def test_ghost_mask_depth():
    valid = boxes_mask([(4, 4, 4, 11, 11, 11)], 16)
    for d in (1, 2, 3):
        g = ghost_mask(valid, d)
        assert g.sum() == (8 + 2 * d) ** 3 - 8 ** 3
        assert not (g & valid).any()


@pytest.mark.parametrize("order,integrator", [(2, 4), (3, 4), (2, 10)])
def test_deep_ghost_fills_keep_a_linear_in_time_field_exact(order, integrator):
    # psi' = Pi, Pi' = 0 with a uniform field: every stage is exact and so is the linear
    # time interpolation of the coarse level, so the fine level stays uniform only if all
    # of its ghost cells down to the stencil's depth are interpolated at the right time
    n0, L = 16, 16.0
    y0 = (0.2, -0.1, 0.5, 0.3)
    U0 = np.stack([np.full((n0,) * 3, v) for v in y0])
    h = Hierarchy(n0, L, 0.25, 0.3, 1, alpha=0.0, lam=0.0, beta=0, integrator=integrator, order=order)
    h.set_level0(U0)
    h.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    L1 = h.levels[1]
    assert L1.ghost.sum() == (16 + 2 * order) ** 3 - 16 ** 3
    for step in range(2):
        h.coarse_step()
        t = (step + 1) * 0.25
        for c, want in enumerate((y0[0] + y0[2] * t, y0[1] + y0[3] * t, y0[2], y0[3])):
            assert np.max(np.abs(L1.U[c][L1.valid] - want)) < 1e-14, (step, c)
    # a hierarchy that leaves the deepest ghost layer stale is caught by the same check
    bad = Hierarchy(n0, L, 0.25, 0.3, 1, alpha=0.0, lam=0.0, beta=0, integrator=integrator, order=order)
    bad.set_level0(U0)
    bad.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    bad.levels[1].ghost = ghost_mask(bad.levels[1].valid, order - 1)
    with np.errstate(invalid="ignore"):
        bad.coarse_step()
    B1 = bad.levels[1]
    assert not np.all(np.abs(B1.U[0][B1.valid] - (y0[0] + y0[2] * 0.25)) < 1e-6)
