"""Lattice energy of the two-component field (oracle; test infrastructure only).

Appendix B measures convergence with the total wave energy (kinetic plus gradient
energy).  For the axion-string field the per-cell energy density is

    e = 1/2 (Pi1^2 + Pi2^2)
      + 1/2 sum_i sum_d (psi_i(x + e_d) - psi_i(x))^2 / dx^2        (forward differences)
      + c_pot/4 (psi1^2 + psi2^2 - 1)^2

with c_pot = lambda eta^beta, the potential whose psi-derivative is the potential term
of eq. EOM2.  With alpha = beta = 0 this is the conserved Hamiltonian of the 7-point
semi-discrete system (the 7-point Laplacian is minus the adjoint of the forward
difference).  The total is sum(e) dx^3 over the counted cells.
"""
from __future__ import annotations

import numpy as np


def energy_density_terms(U: np.ndarray, inv_dx2: float, c_pot: float):
    """Per-cell (kinetic, gradient, potential) densities of a periodic dense state, FP64."""
    p1 = U[0].astype(np.float64)
    p2 = U[1].astype(np.float64)
    q1 = U[2].astype(np.float64)
    q2 = U[3].astype(np.float64)
    kin = 0.5 * (q1 * q1 + q2 * q2)
    g = np.zeros_like(p1)
    for p in (p1, p2):
        for ax in (2, 1, 0):
            d = np.roll(p, -1, axis=ax) - p
            g = g + d * d
    grad = 0.5 * g * inv_dx2
    r2m1 = (p1 * p1 + p2 * p2) - 1.0
    pot = 0.25 * c_pot * (r2m1 * r2m1)
    return kin, grad, pot


def energy(U: np.ndarray, dx: float, c_pot: float, mask: np.ndarray | None = None):
    """[kinetic, gradient, potential, total] summed over ``mask`` (all cells if None)."""
    kin, grad, pot = energy_density_terms(U, 1.0 / (dx * dx), c_pot)
    vol = dx * dx * dx
    out = []
    for t in (kin, grad, pot):
        out.append(float(np.sum(t if mask is None else t[mask], dtype=np.float64)) * vol)
    out.append(out[0] + out[1] + out[2])
    return out


def nonfinite_count(U: np.ndarray, mask: np.ndarray | None = None) -> int:
    """Number of counted cells holding a non-finite value in any component."""
    bad = ~np.all(np.isfinite(U), axis=0)
    return int(np.count_nonzero(bad if mask is None else bad & mask))
