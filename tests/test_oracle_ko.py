"""Pins of the oracle's Kreiss-Oliger dissipation (section II, "Kreiss-Oliger dissipation";
dissipation order 2 or 3, read as p = 3 or 5): the operator annihilates polynomials up to
degree p and gives (p+1)! on x^(p+1), damps a plane wave at the closed-form rate, enters
the free-field step on both psi and Pi with that rate, and on a refined level needs ghost
cells of psi and Pi as deep as its stencil."""
import numpy as np
import pytest

from oracle.amr import Hierarchy
from oracle.level import ko_coef, ko_term, run_single_level
from synth import plane_wave, state_from_psi


def _grid(n, origin=-5):
    i = np.arange(n, dtype=np.float64) + origin
    return np.meshgrid(i, i, i, indexing="ij")


@pytest.mark.parametrize("d", [2, 3])
def test_differences_of_polynomials(d):
    p = 2 * d - 1
    z, y, x = _grid(16)
    inner = (slice(d, -d),) * 3
    u = x ** p - 3 * y ** (p - 1) + 2 * z ** 2 + x * y * z           # degree <= p: annihilated
    assert np.all(ko_term(u, d, 1.0)[inner] == 0.0)
    v = x ** (p + 1) + y ** (p + 1)                                # two axes of (p+1)! each
    fact = float(np.prod(np.arange(1, p + 2)))
    assert np.all(ko_term(v, d, 1.0)[inner] == 2 * fact)


@pytest.mark.parametrize("d", [2, 3])
def test_plane_wave_damping_rate(d):
    n, L, eps = 24, 24.0 * 0.7, 0.05
    dx = L / n
    k = 2 * np.pi / L * np.array([3.0, -5.0, 2.0])
    u = plane_wave(n, L, k)
    p = 2 * d - 1
    rate = (eps / dx) * np.sum(np.sin(k * dx / 2) ** (p + 1))      # Q = -rate * u
    got = ko_term(u, d, ko_coef(d, eps, dx))
    np.testing.assert_allclose(got, -rate * u, atol=1e-13)
    # the paper's form: (-1)^((p+3)/2) eps dx^p / 2^(p+1) times the (p+1)-st differences
    assert ko_coef(d, eps, dx) == pytest.approx((-1) ** ((p + 3) // 2) * eps / (2 ** (p + 1) * dx), rel=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_free_field_step_matrix_with_dissipation(d):
    # psi' = Pi - g psi, Pi' = -w^2 psi - g Pi for one lattice mode: RK4 step matrix of A
    n, L, dt, eps = 16, 16.0, 0.2, 0.3
    dx = L / n
    k = 2 * np.pi / L * np.array([1.0, 2.0, -3.0])
    cosk = plane_wave(n, L, k)
    w2 = (4.0 / dx ** 2) * np.sum(np.sin(k * dx / 2) ** 2)
    g = (eps / dx) * np.sum(np.sin(k * dx / 2) ** (2 * d))
    A = np.array([[-g, 1.0], [-w2, -g]]) * dt
    A2 = A @ A
    M = np.eye(2) + A + A2 / 2 + A2 @ A / 6 + A2 @ A2 / 24
    nsteps = 25
    a, b = np.linalg.matrix_power(M, nsteps) @ np.array([1.0, 0.0])
    U = run_single_level(state_from_psi(cosk, np.zeros_like(cosk)), nsteps, 0.1, dt, dx, alpha=0.0, lam=0.0,
                         beta=0, ko_order=d, ko_eps=eps)
    np.testing.assert_allclose(U[0], a * cosk, atol=1e-12)
    np.testing.assert_allclose(U[2], b * cosk, atol=1e-11)
    assert g > 1e-3                                                 # the damping is not negligible


@pytest.mark.parametrize("d", [2, 3])
def test_refined_level_needs_deep_psi_and_pi_ghosts(d):
    # a uniform field moving linearly in time is a fixed point of the dissipation; the
    # refined level stays exact only if psi and Pi ghosts are filled d cells deep
    n0, L = 16, 16.0
    y0 = (0.2, -0.1, 0.5, 0.3)
    U0 = np.stack([np.full((n0,) * 3, v) for v in y0])
    h = Hierarchy(n0, L, 0.25, 0.3, 1, alpha=0.0, lam=0.0, beta=0, ko_order=d, ko_eps=0.1)
    h.set_level0(U0)
    h.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    L1 = h.levels[1]
    assert L1.ghost.sum() == (16 + 2 * d) ** 3 - 16 ** 3
    for step in range(2):
        h.coarse_step()
        t = (step + 1) * 0.25
        for c, want in enumerate((y0[0] + y0[2] * t, y0[1] + y0[3] * t, y0[2], y0[3])):
            assert np.max(np.abs(L1.U[c][L1.valid] - want)) < 1e-14, (step, c)

    class PsiGhostsOnly(Hierarchy):
        def fill(self, lev, X, alpha):
            saved, self.ko_order = self.ko_order, 0
            try:
                super().fill(lev, X, alpha)
            finally:
                self.ko_order = saved

    bad = PsiGhostsOnly(n0, L, 0.25, 0.3, 1, alpha=0.0, lam=0.0, beta=0, ko_order=d, ko_eps=0.1)
    bad.set_level0(U0)
    bad.set_layout(1, [(8, 8, 8, 23, 23, 23)])
    with np.errstate(invalid="ignore"):
        bad.coarse_step()
    B1 = bad.levels[1]
    assert not np.all(np.abs(B1.U[2][B1.valid] - y0[2]) < 1e-6)
