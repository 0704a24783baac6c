"""Pins of the oracle's RKN5 integrator (integrator type 22 of appendix E, read as a
four-stage fifth-order Runge-Kutta-Nystrom tableau), independently of the oracle: the
tableau's order conditions up to order five in exact fractions, fifth order in time on a
free lattice mode against its closed form, appendix B's energy convergence of a travelling
wave with the 13-point Laplacian at dt = 0.32 dx (the paper's index for RKN5 is -4.0,
limited by that fourth-order Laplacian), one step of a uniform field against the tableau
applied by hand to the ODE (the potential at the stage times), and the refusals."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.amr import Hierarchy
from oracle.level import run_single_level
from oracle.scalars import RKN5_TABLEAU, stage_fractions


def _tableau():
    c = [Fr(*x) for x in RKN5_TABLEAU["c"]]
    a = {k: Fr(*v) for k, v in RKN5_TABLEAU["a"].items()}
    bb = [Fr(*x) for x in RKN5_TABLEAU["bbar"]]
    b = [Fr(*x) for x in RKN5_TABLEAU["b"]]
    A = [[a.get((i + 1, j + 1), Fr(0)) for j in range(4)] for i in range(4)]
    return c, A, bb, b


def test_tableau_satisfies_the_order_conditions_up_to_five():
    # Nystrom order conditions for y'' = f(y) (Hairer, Norsett, Wanner, section II.14),
    # velocity weights b through order 5 and position weights bbar through order 4
    c, A, bb, b = _tableau()
    n = range(4)
    assert [float(x) for x in c] == list(stage_fractions(22))
    for i in n:
        assert sum(A[i]) == c[i] ** 2 / 2                       # row sums
        assert all(A[i][j] == 0 for j in range(i, 4))            # explicit
    Ac = [sum(A[i][j] * c[j] for j in n) for i in n]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in n) for i in n]
    for q in range(5):
        assert sum(b[i] * c[i] ** q for i in n) == Fr(1, q + 1)
    assert sum(b[i] * Ac[i] for i in n) == Fr(1, 24)
    assert sum(b[i] * c[i] * Ac[i] for i in n) == Fr(1, 30)
    assert sum(b[i] * Ac2[i] for i in n) == Fr(1, 60)
    for q in range(4):
        assert sum(bb[i] * c[i] ** q for i in n) == Fr(1, (q + 1) * (q + 2))
    assert sum(bb[i] * Ac[i] for i in n) == Fr(1, 120)
    assert all(bb[i] == b[i] * (1 - c[i]) for i in n)


def _cos_mode(n, L, k):
    x = (np.arange(n) + 0.5) * (L / n)
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return np.cos(k[0] * xx + k[1] * y + k[2] * z)


def test_fifth_order_in_time_on_a_free_mode():
    n, L = 8, 8.0
    k = 2 * np.pi / L * np.array([1.0, 0.0, 0.0])
    c = _cos_mode(n, L, k)
    zero = np.zeros_like(c)
    U0 = np.stack([c, zero, zero, zero])
    w = np.sqrt(4.0 * np.sin(k[0] / 2) ** 2)      # the 7-point Laplacian's eigenvalue
    T = 4.0
    errs = []
    for nsteps in (16, 32, 64):
        U = run_single_level(U0, nsteps, 0.1, T / nsteps, 1.0, alpha=0.0, lam=0.0, beta=0, integrator=22)
        errs.append(np.max(np.abs(U[0] - np.cos(w * T) * c)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 4.6) and np.all(rates < 5.8), (rates, errs)


def _travelling_wave_energy_error(n, periods=10):
    """Appendix B's measure for one travelling wave along x: 13-point Laplacian, dt = 0.32
    dx, energy of the final state (spectral gradient) against the exact one."""
    L = 1.0
    dx = L / n
    kx = 2 * np.pi / L
    x = (np.arange(n) + 0.5) * dx
    U0 = np.zeros((4, 1, 1, n))
    U0[0, 0, 0] = np.sin(kx * x)
    U0[2, 0, 0] = -kx * np.cos(kx * x)
    T = periods * L
    nsteps = int(round(T / (0.32 * dx)))
    U = run_single_level(U0, nsteps, 0.1, T / nsteps, dx, alpha=0.0, lam=0.0, beta=0, integrator=22, order=2)
    psi, pi = U[0, 0, 0], U[2, 0, 0]
    kk = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    grad = np.real(np.fft.ifft(1j * kk * np.fft.fft(psi)))
    E = np.sum(0.5 * pi**2 + 0.5 * grad**2) * dx
    return abs(E - 0.5 * kx**2)


def test_appendix_b_energy_convergence_of_rkn5_with_the_13_point_laplacian():
    ns = np.array([16, 32, 64])
    dE = np.array([_travelling_wave_energy_error(n) for n in ns])
    slope = np.polyfit(np.log(ns), np.log(dE), 1)[0]
    # the paper's criterion: an index of about -4 or better (it fits -4.0 for RKN5 on its
    # 3-D wave packets, where the fourth-order Laplacian's dispersion limits it); for this
    # single wave the energy error falls off like dx^5, as it does for RKN4
    assert -6.0 < slope < -3.7, (slope, dE)


def test_one_step_of_a_uniform_field_is_the_tableau_by_hand():
    # uniform field, no gradients: psi'' = -lambda eta^beta (|psi|^2 - 1) psi; the four
    # stages written out from the tableau, each acceleration at eta_n + c_i h
    eta0, h, lam, beta = 0.7, 0.2, 0.8, 2
    y, v = np.array([0.4, -0.3]), np.array([0.1, 0.25])

    def f(t, p):
        return -lam * t**beta * (p @ p - 1.0) * p

    k1 = f(eta0, y)
    k2 = f(eta0 + h / 5, y + h / 5 * v + h * h * (k1 / 50))
    k3 = f(eta0 + 2 * h / 3, y + 2 * h / 3 * v + h * h * (-k1 / 27 + 7 * k2 / 27))
    k4 = f(eta0 + h, y + h * v + h * h * (3 * k1 / 10 - 2 * k2 / 35 + 9 * k3 / 35))
    y1 = y + h * v + h * h * (k1 / 24 + 25 * k2 / 84 + 9 * k3 / 56)
    v1 = v + h * (k1 / 24 + 125 * k2 / 336 + 27 * k3 / 56 + 5 * k4 / 48)
    U0 = np.empty((4, 4, 4, 4))
    for c, val in enumerate((*y, *v)):
        U0[c] = val
    U = run_single_level(U0, 1, eta0, h, 1.0, alpha=0.0, lam=lam, beta=beta, integrator=22)
    got = np.array([U[c].flat[0] for c in range(4)])
    assert np.max(np.abs(got - np.concatenate([y1, v1]))) < 1e-15
    for c in range(4):
        assert np.all(U[c] == U[c].flat[0])


def test_friction_dissipation_and_hierarchies_are_refused():
    U0 = np.zeros((4, 4, 4, 4))
    with pytest.raises(ValueError):
        run_single_level(U0, 1, 0.1, 0.25, 1.0, alpha=2.0, integrator=22)
    with pytest.raises(ValueError):
        run_single_level(U0, 1, 0.1, 0.25, 1.0, alpha=0.0, integrator=22, ko_order=2, ko_eps=0.1)
    with pytest.raises(ValueError):
        Hierarchy(8, 8.0, 0.25, 0.1, 1, alpha=0.0, beta=0, integrator=22)
