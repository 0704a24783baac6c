"""Plaquette string tagging (oracle; test infrastructure only).

The paper's problem-specific tagging hook (section "Problem-specific cell tagging")
returns true for a cell that must be refined.  Here the criterion is that the phase of
z = psi1 + i psi2 winds by 2 pi around a plaquette of the lattice, i.e. a string pierces
it.  A cell is tagged iff any of the 12 plaquettes having it as a corner is pierced.

Plaquette with lower corner c and normal n, in-plane axes (a, b) = (y, z), (z, x), (x, y)
for n = x, y, z: corners v0 = c, v1 = c + e_a, v2 = c + e_a + e_b, v3 = c + e_b.

Winding number by the crossing rule for the origin (D. Sunday, "Inclusion of a point
in a polygon", 2001): for each directed edge p -> q,
    +1 if y_p <= 0 < y_q and x_p y_q - x_q y_p > 0   (upward crossing, origin to the left)
    -1 if y_q <= 0 < y_p and x_p y_q - x_q y_p < 0   (downward crossing, origin to the right)
with both products rounded separately.  An origin exactly on an edge counts 0; the rule
agrees with (1/2pi) sum of wrapped phase differences whenever no edge passes through 0.
Inputs are promoted to float64 first (products of float32 values are then exact).
"""
from __future__ import annotations

import numpy as np


def _edge(xp, yp, xq, yq):
    cross = xp * yq - xq * yp
    up = (yp <= 0.0) & (yq > 0.0) & (cross > 0.0)
    down = (yq <= 0.0) & (yp > 0.0) & (cross < 0.0)
    return up.astype(np.int8) - down.astype(np.int8)


def _shift(a, ax):
    """a at c + e_ax (periodic)."""
    return np.roll(a, -1, axis=ax)


# axis numbers in [z, y, x] arrays
_AX = {"x": 2, "y": 1, "z": 0}
_PLANES = {"x": ("y", "z"), "y": ("z", "x"), "z": ("x", "y")}


def plaquette_windings(psi1: np.ndarray, psi2: np.ndarray):
    """Winding numbers W_n[c] (int8) for normals n = x, y, z of a periodic dense lattice."""
    X = psi1.astype(np.float64)
    Y = psi2.astype(np.float64)
    out = {}
    for n, (a, b) in _PLANES.items():
        aa, bb = _AX[a], _AX[b]
        x0, y0 = X, Y
        x1, y1 = _shift(X, aa), _shift(Y, aa)
        x2, y2 = _shift(x1, bb), _shift(y1, bb)
        x3, y3 = _shift(X, bb), _shift(Y, bb)
        W = (_edge(x0, y0, x1, y1) + _edge(x1, y1, x2, y2)
             + _edge(x2, y2, x3, y3) + _edge(x3, y3, x0, y0))
        out[n] = W.astype(np.int8)
    return out


def plaquette_windings_atan2(psi1: np.ndarray, psi2: np.ndarray):
    """Same windings from (1/2pi) sum of phase differences wrapped to (-pi, pi].

    Independent of the crossing rule; valid where no edge passes through the origin.
    """
    ph = np.arctan2(psi2.astype(np.float64), psi1.astype(np.float64))

    def wrap(d):
        return d - 2.0 * np.pi * np.ceil((d - np.pi) / (2.0 * np.pi))

    out = {}
    for n, (a, b) in _PLANES.items():
        aa, bb = _AX[a], _AX[b]
        p0 = ph
        p1 = _shift(ph, aa)
        p2 = _shift(p1, bb)
        p3 = _shift(ph, bb)
        s = wrap(p1 - p0) + wrap(p2 - p1) + wrap(p3 - p2) + wrap(p0 - p3)
        out[n] = np.rint(s / (2.0 * np.pi)).astype(np.int8)
    return out


def tag_cells(psi1: np.ndarray, psi2: np.ndarray, windings=None) -> np.ndarray:
    """uint8 mask: 1 where any of the cell's 12 incident plaquettes has W != 0."""
    W = plaquette_windings(psi1, psi2) if windings is None else windings
    tag = np.zeros(psi1.shape, dtype=bool)
    for n, (a, b) in _PLANES.items():
        P = W[n] != 0
        aa, bb = _AX[a], _AX[b]
        # cell c is a corner of the plaquettes with lower corner c, c-e_a, c-e_b, c-e_a-e_b
        Pa = np.roll(P, 1, axis=aa)
        tag |= P | Pa | np.roll(P, 1, axis=bb) | np.roll(Pa, 1, axis=bb)
    return tag.astype(np.uint8)
