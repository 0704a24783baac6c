"""Pins of the single-level oracle against closed forms and independent formulations.

Each test fixes the oracle to something other than its own formula: exact Laplacians of
quadratics, the 7-point eigenvalue of a plane wave, the exact fully discrete RK4
solution of the free field, a textbook-form RK4 of the uniform-field ODE, fourth-order
convergence, exact fixed points and the U(1) symmetry.
"""
import numpy as np
import pytest

from oracle.energy import energy
from oracle.level import lap7, rhs, rk4_step, run_single_level
from oracle.scalars import level_time, stage_scalars, int_power
from synth import gaussian_random_pair, plane_wave, quadratic_field, state_from_psi


@pytest.mark.parametrize("coeffs", [(1, 2, 3, 0, 0, 0), (3, -1, 2, 5, -4, 7), (0, 0, 0, 1, 1, 1)])
@pytest.mark.parametrize("inv_dx2", [1.0, 4.0, 16.0])
def test_laplacian_of_quadratic_is_exact(coeffs, inv_dx2):
    # integer quadratic in index units: 7-point Laplacian = 2(a+b+c) exactly (in index units)
    u = quadratic_field((12, 10, 14), coeffs, origin=(-1, -1, -1))
    lap = lap7(u, inv_dx2)[1:-1, 1:-1, 1:-1]   # interior: unaffected by the periodic wrap
    a, b, c = coeffs[:3]
    assert np.all(lap == 2.0 * (a + b + c) * inv_dx2)


def test_laplacian_plane_wave_eigenvalue():
    n, L = 24, 24.0 * 0.7
    dx = L / n
    k = 2 * np.pi / L * np.array([3.0, -5.0, 2.0])
    u = plane_wave(n, L, k)
    lam = -(4.0 / dx**2) * np.sum(np.sin(k * dx / 2) ** 2)
    np.testing.assert_allclose(lap7(u, 1.0 / dx**2), lam * u, atol=1e-12 * abs(lam))


def _free_field_amp(omega, dt, nsteps):
    """Exact fully discrete RK4 amplification of (psi, Pi) for psi'' = -omega^2 psi."""
    y = omega * dt
    J = np.array([[0.0, 1.0], [-omega * omega, 0.0]])
    M = (1 - y * y / 2 + y**4 / 24) * np.eye(2) + (dt - omega * omega * dt**3 / 6) * J
    return np.linalg.matrix_power(M, nsteps) @ np.array([1.0, 0.0])


@pytest.mark.parametrize("dt", [0.25, 0.1])
def test_rk4_free_field_matches_exact_discrete_solution(dt):
    # lambda = 0, alpha = 0: the lattice is linear; one integer mode evolves by M^n exactly
    n, L = 16, 16.0
    dx = L / n
    k = 2 * np.pi / L * np.array([1.0, 2.0, -3.0])
    omega = np.sqrt((4.0 / dx**2) * np.sum(np.sin(k * dx / 2) ** 2))
    cosk = plane_wave(n, L, k)
    U0 = state_from_psi(cosk, np.zeros_like(cosk))
    nsteps = 40
    U = run_single_level(U0, nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0, beta=0)
    a, b = _free_field_amp(omega, dt, nsteps)
    np.testing.assert_allclose(U[0], a * cosk, atol=1e-12 * nsteps)
    np.testing.assert_allclose(U[2], b * cosk, atol=1e-12 * nsteps * omega)
    assert np.all(U[1] == 0.0) and np.all(U[3] == 0.0)


def test_free_field_energy_factor_closed_form():
    # E_n / E_0 = |R(iy)|^(2n), |R(iy)|^2 = 1 - y^6/72 + y^8/576 (exact discrete energy)
    n, L, dt = 16, 16.0, 0.3
    dx = L / n
    k = 2 * np.pi / L * np.array([2.0, 1.0, 1.0])
    omega = np.sqrt((4.0 / dx**2) * np.sum(np.sin(k * dx / 2) ** 2))
    y = omega * dt
    fac = 1 - y**6 / 72 + y**8 / 576
    U0 = state_from_psi(plane_wave(n, L, k), np.zeros((n, n, n)))
    e0 = energy(U0, dx, 0.0)[3]
    nsteps = 25
    U = run_single_level(U0, nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0, beta=0)
    e1 = energy(U, dx, 0.0)[3]
    assert abs(e1 / e0 - fac**nsteps) < 1e-12
    # and the closed-form starting energy: (N^3/4) omega^2 dx^3 for a unit cosine
    assert abs(e0 - n**3 / 4 * omega**2 * dx**3) < 1e-10 * e0


def _textbook_rk4_uniform(y0, eta0, dt, nsteps, alpha, lam, beta):
    """Uniform field: psi_i' = Pi_i, Pi_i' = -(alpha/eta) Pi_i - lam eta^beta psi_i(r2-1).

    Butcher form y + h/6 (k1 + 2k2 + 2k3 + k4), written independently of the oracle.
    """
    def f(t, y):
        p1, p2, q1, q2 = y
        g = lam * t**beta * (p1 * p1 + p2 * p2 - 1)
        return np.array([q1, q2, -alpha / t * q1 - g * p1, -alpha / t * q2 - g * p2])

    y = np.array(y0, dtype=float)
    for k in range(nsteps):
        t = eta0 + k * dt
        k1 = f(t, y)
        k2 = f(t + dt / 2, y + dt / 2 * k1)
        k3 = f(t + dt / 2, y + dt / 2 * k2)
        k4 = f(t + dt, y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_uniform_field_matches_textbook_rk4():
    y0 = (0.3, -0.2, 0.1, 0.05)
    U0 = np.empty((4, 4, 4, 4))
    for c in range(4):
        U0[c] = y0[c]
    eta0, dt, nsteps = 0.5, 0.05, 60
    U = run_single_level(U0, nsteps, eta0, dt, 1.0, alpha=2.0, lam=1.0, beta=2)
    ref = _textbook_rk4_uniform(y0, eta0, dt, nsteps, 2.0, 1.0, 2)
    for c in range(4):
        assert np.all(U[c] == U[c].flat[0])          # stays uniform
        assert abs(U[c].flat[0] - ref[c]) < 1e-13 * max(1.0, abs(ref[c]))


def test_uniform_field_fourth_order_convergence():
    y0 = (0.3, -0.2, 0.1, 0.05)
    eta0, T = 0.5, 2.0
    exact = _textbook_rk4_uniform(y0, eta0, T / 2048, 2048, 2.0, 1.0, 2)
    errs = []
    for nsteps in (20, 40):
        U0 = np.empty((4, 2, 2, 2))
        for c in range(4):
            U0[c] = y0[c]
        U = run_single_level(U0, nsteps, eta0, T / nsteps, 1.0)
        errs.append(np.max(np.abs(U[:, 0, 0, 0] - exact)))
    ratio = errs[0] / errs[1]
    assert 13.0 < ratio < 19.0, ratio


@pytest.mark.parametrize("psi", [(0.0, 0.0), (1.0, 0.0), (0.0, -1.0)])
def test_fixed_points_exact(psi):
    U0 = np.zeros((4, 6, 6, 6))
    U0[0], U0[1] = psi
    U = run_single_level(U0, 10, 0.1, 0.25, 1.0)
    assert np.array_equal(U, U0)


def test_u1_quarter_turn_commutes_bitwise():
    p1, p2 = gaussian_random_pair(12, 12.0, seed=3)
    rng = np.random.default_rng(4)
    U0 = state_from_psi(p1, p2, 0.1 * rng.standard_normal(p1.shape), 0.1 * rng.standard_normal(p1.shape))

    def rot(U):
        return np.stack([-U[1], U[0], -U[3], U[2]])

    a = run_single_level(rot(U0), 5, 0.1, 0.25, 1.0)
    b = rot(run_single_level(U0, 5, 0.1, 0.25, 1.0))
    assert np.array_equal(a, b)


def test_static_background_energy_drift_is_fourth_order():
    # alpha = beta = 0: the semi-discrete system conserves the lattice energy exactly;
    # RK4 drifts at O(dt^4) or better, so halving dt cuts the drift by >= ~16
    p1, p2 = gaussian_random_pair(12, 12.0, seed=5)
    U0 = state_from_psi(p1, p2)
    e0 = energy(U0, 1.0, 1.0)[3]
    drifts = []
    for dt in (0.1, 0.05):
        nsteps = int(round(2.0 / dt))
        U = run_single_level(U0, nsteps, 0.1, dt, 1.0, alpha=0.0, lam=1.0, beta=0)
        drifts.append(abs(energy(U, 1.0, 1.0)[3] - e0))
    assert drifts[0] / drifts[1] > 14.0, drifts


def test_stage_scalars_definitions():
    eta_n, dt = 0.1 + 7 * 0.25, 0.25
    assert level_time(0.1, 7, 0.25) == eta_n
    for s, c in enumerate((0.0, 0.5, 0.5, 1.0)):
        eta_s, cf, cp = stage_scalars(eta_n, dt, s, 2.0, 1.0, 2)
        assert eta_s == eta_n + c * dt
        assert cf == 2.0 / eta_s
        assert cp == eta_s * eta_s
    assert int_power(3.0, 0) == 1.0 and int_power(3.0, 3) == 27.0


def test_rhs_matches_eom_pointwise():
    # independent per-cell evaluation of eq. EOM2 at a few cells of a random state
    p1, p2 = gaussian_random_pair(8, 8.0, seed=1)
    rng = np.random.default_rng(2)
    U = state_from_psi(p1, p2, rng.standard_normal(p1.shape), rng.standard_normal(p1.shape))
    eta = 1.7
    K = rhs(U, 1.0, 2.0 / eta, eta * eta)
    for (z, y, x) in [(0, 0, 0), (3, 5, 7), (7, 7, 7), (2, 0, 6)]:
        for i in (0, 1):
            ps = U[i]
            lap = sum(ps[(z + dz) % 8, (y + dy) % 8, (x + dx) % 8]
                      for dz, dy, dx in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]) \
                - 6 * ps[z, y, x]
            r2 = U[0, z, y, x] ** 2 + U[1, z, y, x] ** 2
            want = -(2.0 / eta) * U[2 + i, z, y, x] + lap - eta**2 * ps[z, y, x] * (r2 - 1)
            assert abs(K[2 + i, z, y, x] - want) < 1e-12 * (1 + abs(want))
            assert K[i, z, y, x] == U[2 + i, z, y, x]


def test_fp32_mode_tracks_fp64():
    p1, p2 = gaussian_random_pair(12, 12.0, seed=7)
    U0 = state_from_psi(p1, p2)
    a = run_single_level(U0, 10, 0.1, 0.25, 1.0)
    b = run_single_level(U0.astype(np.float32), 10, 0.1, 0.25, 1.0)
    assert b.dtype == np.float32
    rel = np.max(np.abs(b - a)) / np.max(np.abs(a))
    assert rel < 1e-5, rel
