"""Pins of the oracle's RKN4 integrator (integrator type 21 of appendix E, read as
Nystrom's classical three-stage fourth-order method) against forms derived by hand from
its tableau, independently of the oracle: the step matrix of a free lattice mode, fourth
order in time, appendix B's energy convergence of a travelling wave with the 13-point
Laplacian at dt = 0.32 dx, the potential evaluated at the stage times, the stage times of
the coarse-to-fine fills, and the refusal of friction and dissipation."""
import numpy as np
import pytest

from oracle.amr import Hierarchy, average_down_arrays
from oracle.level import run_single_level
from oracle.scalars import stage_fractions


def _step_matrix_rkn4(omega2, h):
    """One step of the tableau on y'' = -omega^2 y, worked out by hand with z = (omega h)^2:
    y_new = (1 - z/2 + z^2/24) y + h (1 - z/6) v,
    v_new = -omega^2 h (1 - z/6 + z^2/96) y + (1 - z/2 + z^2/24) v."""
    z = omega2 * h * h
    d = 1.0 - z / 2.0 + z * z / 24.0
    return np.array([[d, h * (1.0 - z / 6.0)], [-omega2 * h * (1.0 - z / 6.0 + z * z / 96.0), d]])


def _omega2(k, dx, order):
    """-(eigenvalue) of the appendix-A Laplacian for the mode exp(i k.x)."""
    th = np.asarray(k) * dx
    if order == 1:
        return float(np.sum(4.0 * np.sin(th / 2) ** 2)) / dx**2
    # fourth-order second difference (4/3, -1/12, -5/2 per axis)
    return float(-np.sum((8.0 / 3.0) * np.cos(th) - (1.0 / 6.0) * np.cos(2 * th) - 2.5)) / dx**2


def _cos_mode(n, L, k):
    x = (np.arange(n) + 0.5) * (L / n)
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return np.cos(k[0] * xx + k[1] * y + k[2] * z)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dt", [0.25, 0.32])
def test_free_mode_follows_the_hand_derived_step_matrix(order, dt):
    n, L = 16, 16.0
    k = 2 * np.pi / L * np.array([1.0, 2.0, 3.0])
    c = _cos_mode(n, L, k)
    a, b = 0.6, -0.35
    zero = np.zeros_like(c)
    U0 = np.stack([a * c, zero, b * c, zero])
    nsteps = 3
    U = run_single_level(U0, nsteps, 0.1, dt, 1.0, alpha=0.0, lam=0.0, beta=0, integrator=21, order=order)
    M = np.linalg.matrix_power(_step_matrix_rkn4(_omega2(k, 1.0, order), dt), nsteps)
    ya, va = M @ np.array([a, b])
    assert np.max(np.abs(U[0] - ya * c)) < 1e-13
    assert np.max(np.abs(U[2] - va * c)) < 1e-13
    assert not U[1].any() and not U[3].any()


def test_fourth_order_in_time_on_a_free_mode():
    n, L = 8, 8.0
    k = 2 * np.pi / L * np.array([1.0, 0.0, 0.0])
    c = _cos_mode(n, L, k)
    zero = np.zeros_like(c)
    U0 = np.stack([c, zero, zero, zero])
    w = np.sqrt(_omega2(k, 1.0, 1))
    T = 4.0
    errs = []
    for nsteps in (32, 64, 128):
        U = run_single_level(U0, nsteps, 0.1, T / nsteps, 1.0, alpha=0.0, lam=0.0, beta=0, integrator=21)
        errs.append(np.max(np.abs(U[0] - np.cos(w * T) * c)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8) and np.all(rates < 4.6) and rates[1] < rates[0], rates


def _travelling_wave_energy_error(n, periods=10):
    """Appendix B's measure for one travelling wave along x on an n x 1 x 1 lattice:
    13-point Laplacian, dt = 0.32 dx, energy of the final state (spectral gradient)
    against the exact one."""
    L = 1.0
    dx = L / n
    kx = 2 * np.pi / L
    x = (np.arange(n) + 0.5) * dx
    U0 = np.zeros((4, 1, 1, n))
    U0[0, 0, 0] = np.sin(kx * x)
    U0[2, 0, 0] = -kx * np.cos(kx * x)
    T = periods * L
    nsteps = int(round(T / (0.32 * dx)))
    dt = T / nsteps
    U = run_single_level(U0, nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0, beta=0, integrator=21, order=2)
    psi, pi = U[0, 0, 0], U[2, 0, 0]
    kk = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    grad = np.real(np.fft.ifft(1j * kk * np.fft.fft(psi)))
    E = np.sum(0.5 * pi**2 + 0.5 * grad**2) * dx
    return abs(E - 0.5 * kx**2)


def test_appendix_b_energy_convergence_of_rkn4_with_the_13_point_laplacian():
    ns = np.array([16, 32, 64])
    dE = np.array([_travelling_wave_energy_error(n) for n in ns])
    slope = np.polyfit(np.log(ns), np.log(dE), 1)[0]
    # the paper's criterion: a power-law index of about -p or better for an order-p
    # integrator (it fits -4.3 for RKN4 on its 3-D wave packets); this single wave's
    # energy error is led by the step's amplitude error, det(M) - 1 = -(omega h)^6 / 288,
    # so it falls off like dx^5 here
    assert -6.0 < slope < -3.7, (slope, dE)


def test_stage_times_and_fills_follow_the_nodes():
    assert stage_fractions(21) == (0.0, 0.5, 1.0)
    # psi'' = 0 with Pi uniform: psi moves linearly, which every stage integrates exactly,
    # and the fine level stays exact only if its ghosts are filled at the nodes' times
    n0, L, eta0 = 8, 8.0, 0.3
    y0 = (0.2, -0.1, 0.5, 0.3)
    U0 = np.empty((4, n0, n0, n0))
    for c in range(4):
        U0[c] = y0[c]
    h = Hierarchy(n0, L, 0.25, eta0, 1, alpha=0.0, lam=0.0, beta=0, integrator=21)
    h.set_level0(U0)
    h.set_layout(1, [(4, 4, 4, 11, 11, 11)])
    for step in range(3):
        h.coarse_step()
        t = (step + 1) * 0.25
        L1 = h.levels[1]
        for c, want in enumerate((y0[0] + y0[2] * t, y0[1] + y0[3] * t, y0[2], y0[3])):
            assert np.max(np.abs(L1.U[c][L1.valid] - want)) < 1e-14, (step, c)
    bad = Hierarchy(n0, L, 0.25, eta0, 1, alpha=0.0, lam=0.0, beta=0, integrator=21)
    bad.cs = (0.0, 0.5, 0.5)
    bad.set_level0(U0)
    bad.set_layout(1, [(4, 4, 4, 11, 11, 11)])
    bad.coarse_step()
    L1 = bad.levels[1]
    assert np.max(np.abs(L1.U[0][L1.valid] - (y0[0] + y0[2] * 0.25))) > 1e-6


def test_potential_is_taken_at_the_stage_times():
    # uniform field, no gradients: psi'' = -lambda eta^beta (|psi|^2 - 1) psi, checked
    # against the tableau applied by hand to the ODE
    eta0, dt, lam, beta = 0.7, 0.2, 0.8, 2
    y, v = np.array([0.4, -0.3]), np.array([0.1, 0.25])

    def f(t, p):
        return -lam * t**beta * (p @ p - 1.0) * p

    k1 = f(eta0, y)
    k2 = f(eta0 + dt / 2, y + dt / 2 * v + dt * dt / 8 * k1)
    k3 = f(eta0 + dt, y + dt * v + dt * dt / 2 * k2)
    y1 = y + dt * v + dt * dt * (k1 / 6 + k2 / 3)
    v1 = v + dt * (k1 / 6 + 2 * k2 / 3 + k3 / 6)
    U0 = np.empty((4, 4, 4, 4))
    for c, val in enumerate((*y, *v)):
        U0[c] = val
    U = run_single_level(U0, 1, eta0, dt, 1.0, alpha=0.0, lam=lam, beta=beta, integrator=21)
    got = np.array([U[c].flat[0] for c in range(4)])
    assert np.max(np.abs(got - np.concatenate([y1, v1]))) < 1e-15
    for c in range(4):
        assert np.all(U[c] == U[c].flat[0])


def test_two_level_full_coverage_equals_single_fine_level():
    n0 = 8
    rng = np.random.default_rng(3)
    U0 = rng.standard_normal((4, n0, n0, n0)) * 0.3
    h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, alpha=0.0, beta=0, integrator=21)
    h.set_level0(U0)
    h.set_layout(1, [(x, y, z, x + 7, y + 7, z + 7) for z in (0, 8) for y in (0, 8) for x in (0, 8)])
    U1 = h.levels[1].U.copy()
    for _ in range(2):
        h.coarse_step()
        assert np.array_equal(h.levels[0].U, np.stack([average_down_arrays(c) for c in h.levels[1].U]))
    ref = run_single_level(U1, 4, 0.1, 0.125, 0.5, alpha=0.0, beta=0, integrator=21)
    assert np.array_equal(h.levels[1].U, ref)


def test_friction_and_dissipation_are_refused():
    with pytest.raises(ValueError):
        Hierarchy(8, 8.0, 0.25, 0.1, 1, alpha=2.0, integrator=21)
    with pytest.raises(ValueError):
        Hierarchy(8, 8.0, 0.25, 0.1, 1, alpha=0.0, integrator=21, ko_order=2, ko_eps=0.1)
    with pytest.raises(ValueError):
        run_single_level(np.zeros((4, 4, 4, 4)), 1, 0.1, 0.1, 1.0, alpha=2.0, integrator=21)
