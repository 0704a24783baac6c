"""Pins of the oracle's SSPRK3 integrator (three-stage, third-order, strong-stability-
preserving; appendix E's integrator list) against forms written independently of it:
the Butcher tableau of the method on the uniform-field ODE, its stability polynomial on
the free lattice, third-order convergence, the stage times seen by the coarse-to-fine
fills, and the self-shadow estimate of a free plane wave."""
import numpy as np
import pytest

from oracle.amr import Hierarchy, average_down_arrays
from oracle.level import run_single_level
from oracle.scalars import stage_fractions, stage_scalars
from synth import plane_wave, state_from_psi


def _f_uniform(t, y, alpha, lam, beta):
    p1, p2, q1, q2 = y
    g = lam * t**beta * (p1 * p1 + p2 * p2 - 1)
    return np.array([q1, q2, -alpha / t * q1 - g * p1, -alpha / t * q2 - g * p2])


def _butcher_ssprk3(y0, eta0, dt, nsteps, alpha, lam, beta):
    """Butcher form: c = (0, 1, 1/2), a21 = 1, a31 = a32 = 1/4, b = (1/6, 1/6, 2/3)."""
    y = np.array(y0, dtype=float)
    for k in range(nsteps):
        t = eta0 + k * dt
        k1 = _f_uniform(t, y, alpha, lam, beta)
        k2 = _f_uniform(t + dt, y + dt * k1, alpha, lam, beta)
        k3 = _f_uniform(t + dt / 2, y + dt / 4 * (k1 + k2), alpha, lam, beta)
        y = y + dt * (k1 / 6 + k2 / 6 + 2 * k3 / 3)
    return y


def _uniform_state(y0, n=4):
    U0 = np.empty((4, n, n, n))
    for c in range(4):
        U0[c] = y0[c]
    return U0


@pytest.mark.parametrize("integrator", [3, 10])
def test_uniform_field_matches_the_butcher_tableau(integrator):
    y0 = (0.3, -0.2, 0.1, 0.05)
    eta0, dt, nsteps = 0.5, 0.05, 60
    U = run_single_level(_uniform_state(y0), nsteps, eta0, dt, 1.0, alpha=2.0, lam=1.0, beta=2,
                         integrator=integrator)
    ref = _butcher_ssprk3(y0, eta0, dt, nsteps, 2.0, 1.0, 2)
    for c in range(4):
        assert np.all(U[c] == U[c].flat[0])
        assert abs(U[c].flat[0] - ref[c]) < 1e-13 * max(1.0, abs(ref[c]))


def test_uniform_field_third_order_convergence():
    y0 = (0.3, -0.2, 0.1, 0.05)
    eta0, T = 0.5, 2.0
    exact = _butcher_ssprk3(y0, eta0, T / 4096, 4096, 2.0, 1.0, 2)
    errs = []
    for nsteps in (40, 80):
        U = run_single_level(_uniform_state(y0, 2), nsteps, eta0, T / nsteps, 1.0, integrator=3)
        errs.append(np.max(np.abs(U[:, 0, 0, 0] - exact)))
    ratio = errs[0] / errs[1]
    assert 6.5 < ratio < 9.5, ratio


def _step_matrix(omega2, h):
    """Any three-stage third-order RK applied to y' = A y: I + hA + (hA)^2/2 + (hA)^3/6."""
    A = np.array([[0.0, 1.0], [-omega2, 0.0]]) * h
    A2 = A @ A
    return np.eye(2) + A + A2 / 2 + A2 @ A / 6


def _omega2(k, d):
    return (4.0 / d**2) * np.sum(np.sin(k * d / 2) ** 2)


@pytest.mark.parametrize("dt", [0.25, 0.1])
def test_free_field_matches_the_stability_polynomial(dt):
    n, L = 16, 16.0
    dx = L / n
    k = 2 * np.pi / L * np.array([1.0, 2.0, -3.0])
    cosk = plane_wave(n, L, k)
    U0 = state_from_psi(cosk, np.zeros_like(cosk))
    nsteps = 40
    U = run_single_level(U0, nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0, beta=0, integrator=3)
    a, b = np.linalg.matrix_power(_step_matrix(_omega2(k, dx), dt), nsteps) @ np.array([1.0, 0.0])
    np.testing.assert_allclose(U[0], a * cosk, atol=1e-12 * nsteps)
    np.testing.assert_allclose(U[2], b * cosk, atol=1e-12 * nsteps * np.sqrt(_omega2(k, dx)))
    assert np.all(U[1] == 0.0) and np.all(U[3] == 0.0)


def test_stage_times():
    assert stage_fractions(3) == stage_fractions(10) == (0.0, 1.0, 0.5)
    eta_n, dt = 1.1, 0.25
    for s, c in enumerate((0.0, 1.0, 0.5)):
        eta_s, cf, cp = stage_scalars(eta_n, dt, s, 2.0, 1.0, 2, integrator=3)
        assert eta_s == eta_n + c * dt and cf == 2.0 / eta_s and cp == eta_s * eta_s
    with pytest.raises(ValueError):
        stage_fractions(5)


def test_fills_interpolate_at_the_stage_times():
    # A uniform field moving linearly in time (psi' = Pi, Pi' = 0) is integrated exactly by
    # every stage of the method, and the coarse level's linear-in-time interpolation is
    # exact for it, so a fine level whose ghost cells are filled at the right stage times
    # stays uniform and exact.  Filling at another fraction (RK4's 1/2 for the second
    # stage, say) puts a jump at the level edge that the Laplacian turns into an error.
    n0, L, eta0 = 8, 8.0, 0.3
    y0 = (0.2, -0.1, 0.5, 0.3)
    h = Hierarchy(n0, L, 0.25, eta0, 1, alpha=0.0, lam=0.0, beta=0, integrator=3)
    h.set_level0(_uniform_state(y0, n0))
    h.set_layout(1, [(4, 4, 4, 11, 11, 11)])
    for step in range(3):
        h.coarse_step()
        t = (step + 1) * 0.25
        L1 = h.levels[1]
        for c, want in enumerate((y0[0] + y0[2] * t, y0[1] + y0[3] * t, y0[2], y0[3])):
            got = L1.U[c][L1.valid]
            assert np.max(np.abs(got - want)) < 1e-14, (step, c)
    # the same hierarchy under wrong stage fractions departs from the exact value
    bad = Hierarchy(n0, L, 0.25, eta0, 1, alpha=0.0, lam=0.0, beta=0, integrator=3)
    bad.cs = (0.0, 0.5, 0.5)
    bad.set_level0(_uniform_state(y0, n0))
    bad.set_layout(1, [(4, 4, 4, 11, 11, 11)])
    bad.coarse_step()
    L1 = bad.levels[1]
    assert np.max(np.abs(L1.U[0][L1.valid] - (y0[0] + y0[2] * 0.25))) > 1e-6


def _centred_cos(M, L, k, amp):
    x = (np.arange(M) + 0.5) * (L / M)
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return amp * np.cos(k[0] * xx + k[1] * y + k[2] * z)


def _full_cover_boxes(M, b=8):
    return [(x, y, z, x + b - 1, y + b - 1, z + b - 1)
            for z in range(0, M, b) for y in range(0, M, b) for x in range(0, M, b)]


def test_free_plane_wave_self_shadow_estimate_closed_form():
    n0, L, amp = 16, 16.0, 0.7
    k = 2 * np.pi / L * np.array([2.0, 1.0, 1.0])
    dx0, dt0 = L / n0, 0.25
    zero = np.zeros((n0,) * 3)
    h = Hierarchy(n0, L, 0.25, 0.1, 1, alpha=0.0, lam=0.0, beta=0, integrator=10)
    h.set_level0(np.stack([_centred_cos(n0, L, k, amp), zero, zero, zero]))
    h.set_layout(1, _full_cover_boxes(2 * n0))
    h.levels[1].U[:] = 0.0
    h.levels[1].U[0] = _centred_cos(2 * n0, L, k, amp)
    h.set_tee(True)
    h.coarse_step()
    Mc = _step_matrix(_omega2(k, dx0), dt0)
    Mf = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0 / 2), dt0 / 2), 2)
    P = np.prod(np.cos(k * dx0 / 4))
    coef = max(abs(Mc[0, 0] - P * Mf[0, 0]), abs(Mc[1, 0] - P * Mf[1, 0]))
    ref = coef * np.abs(_centred_cos(n0, L, k, 1.0)) * amp
    got = average_down_arrays(h.levels[1].tee)
    assert coef > 1e-6
    assert np.max(np.abs(got - ref)) < 1e-12
