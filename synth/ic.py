"""Seeded initial states for the two-component axion-string field.

Every array is indexed ``[z, y, x]`` (C order, x fastest) and is float64.  A full state
is a ``(4, nz, ny, nx)`` array holding ``psi1, psi2, Pi1, Pi2`` (the two scalars and
their conformal-time derivatives, minimal example section, eq. EOM1/EOM2).

Recipes
-------
* ``gaussian_random_pair``: each psi_i is white noise filtered to the modes with
  0 < |k| < kmax_frac * (pi/dx), then both are scaled by one common factor so that
  <psi1^2 + psi2^2> = 1.  Pi_i = 0.
* ``string_loop_state``: closed string loops (phase winding once around a circle of
  radius R, amplitude tanh(d/2) with d the distance to the core) plus a small multiple
  ``delta`` of the random pair, so that no extra strings appear away from the cores.
* ``straight_strings`` / ``plane_wave`` / ``quadratic_field``: closed-form fields used
  as test inputs with known answers.
"""
from __future__ import annotations

import numpy as np


def _kgrid(n: int, dx: float):
    """Signed angular wavenumbers for a full/real FFT grid of n points and spacing dx."""
    k_full = 2.0 * np.pi * np.fft.fftfreq(n, d=dx)
    k_half = 2.0 * np.pi * np.fft.rfftfreq(n, d=dx)
    return k_full, k_half


def gaussian_random_pair(n: int, L: float, seed: int, kmax_frac: float = 0.5,
                         rng: np.random.Generator | None = None):
    """Two Gaussian random fields with flat power for 0 < |k| < kmax_frac*pi/dx.

    Returns ``(psi1, psi2)`` scaled so that mean(psi1^2 + psi2^2) == 1.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    dx = L / n
    kmax = kmax_frac * np.pi / dx
    k_full, k_half = _kgrid(n, dx)
    kz = k_full[:, None, None]
    ky = k_full[None, :, None]
    kx = k_half[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    keep = (k2 < kmax * kmax) & (k2 > 0.0)
    out = []
    for _ in range(2):
        w = rng.standard_normal((n, n, n))
        W = np.fft.rfftn(w)
        W[~keep] = 0.0
        out.append(np.fft.irfftn(W, s=(n, n, n), axes=(0, 1, 2)))
    s = 1.0 / np.sqrt(np.mean(out[0] ** 2 + out[1] ** 2))
    return out[0] * s, out[1] * s


def state_from_psi(psi1: np.ndarray, psi2: np.ndarray,
                   pi1: np.ndarray | None = None, pi2: np.ndarray | None = None) -> np.ndarray:
    """Stack (psi1, psi2, Pi1, Pi2) into a (4, ...) float64 state; Pi defaults to 0."""
    st = np.zeros((4,) + psi1.shape, dtype=np.float64)
    st[0] = psi1
    st[1] = psi2
    if pi1 is not None:
        st[2] = pi1
    if pi2 is not None:
        st[3] = pi2
    return st


def random_state(n: int, L: float, seed: int) -> np.ndarray:
    """The single-level initial state: Gaussian random pair, zero momenta."""
    p1, p2 = gaussian_random_pair(n, L, seed)
    return state_from_psi(p1, p2)


def string_loop_state(n: int, L: float, seed: int, nloops: int,
                      rmin: float = 20.0, rmax: float = 60.0, delta: float = 0.1,
                      taper_in: float = 8.0, taper_out: float = 40.0) -> np.ndarray:
    """Closed string loops superposed on a small random field (lengths in cells).

    Loop j has radius R ~ U[rmin, rmax], centre ~ U[0, n)^3 and a normal drawn uniformly
    on the sphere, all from the same generator as the random field (drawn after it).
    Its phase theta_j = atan2(z', rho - R) - atan2(z', rho + R) winds once around the
    core circle (rho, z' cylindrical coordinates about the loop axis, minimum image);
    theta_j is tapered by a cos^2 window between |r| = R + taper_in and R + taper_out
    (exactly 0 beyond) so the periodic seam carries no winding.  The amplitude is
    prod_j tanh(d_j / 2), d_j the distance to core j.  Pi = 0.
    """
    rng = np.random.default_rng(seed)
    r1, r2 = gaussian_random_pair(n, L, seed, rng=rng)
    loops = []
    for _ in range(nloops):
        R = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, n, size=3)
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        loops.append((R, c, v))
    if nloops and max(R + taper_out for R, _, _ in loops) >= n / 2:
        raise ValueError("loop plus taper does not fit in half the lattice")
    psi1 = np.empty((n, n, n))
    psi2 = np.empty((n, n, n))
    # outside |r| > R + taper_out a loop contributes nothing: its phase is tapered to 0
    # and, when taper_out/2 exceeds 19.1, tanh(d/2) of the core distance d rounds to 1
    local = taper_out / 2 > 19.1
    idx = np.arange(n, dtype=np.float64)
    for z in range(n):  # slab by slab to bound memory at large n
        amp = np.ones((n, n))
        theta = np.zeros((n, n))
        for R, c, v in loops:
            reach = R + taper_out
            dz = z - c[0]
            dz -= n * np.round(dz / n)
            if local and abs(dz) > reach:
                continue
            if local:
                ys = np.nonzero(np.abs((idx - c[1]) - n * np.round((idx - c[1]) / n)) <= reach)[0]
                xs = np.nonzero(np.abs((idx - c[2]) - n * np.round((idx - c[2]) / n)) <= reach)[0]
            else:
                ys = xs = np.arange(n)
            Y, X = np.meshgrid(idx[ys], idx[xs], indexing="ij")
            d = np.stack([np.full(Y.shape, float(z)) - c[0], Y - c[1], X - c[2]])
            d -= n * np.round(d / n)  # minimum image
            zp = d[0] * v[0] + d[1] * v[1] + d[2] * v[2]
            perp = d - zp[None] * v[:, None, None]
            rho = np.sqrt(np.sum(perp * perp, axis=0))
            dist = np.sqrt((rho - R) ** 2 + zp ** 2)
            th = np.arctan2(zp, rho - R) - np.arctan2(zp, rho + R)
            rr = np.sqrt(np.sum(d * d, axis=0))
            sfr = (rr - (R + taper_in)) / (taper_out - taper_in)
            taper = np.where(sfr >= 1.0, 0.0, np.cos(0.5 * np.pi * np.clip(sfr, 0.0, 1.0)) ** 2)
            sub = np.ix_(ys, xs)
            theta[sub] += th * taper
            amp[sub] *= np.tanh(0.5 * dist)
        psi1[z] = amp * np.cos(theta) + delta * r1[z]
        psi2[z] = amp * np.sin(theta) + delta * r2[z]
    return state_from_psi(psi1, psi2)


def straight_strings(n: int, x0: float = 10.37, y0: float = 21.61):
    """psi1 + i psi2 = sin(2pi(x - x0)/n) + i sin(2pi(y - y0)/n) on an n^3 lattice.

    The zeros are the four z-directed lines x - x0 in {0, n/2}, y - y0 in {0, n/2}
    (mod n); for generic x0, y0 each pierces exactly one xy-plaquette per z-plane.
    """
    i = np.arange(n, dtype=np.float64)
    sx = np.sin(2.0 * np.pi * (i - x0) / n)
    sy = np.sin(2.0 * np.pi * (i - y0) / n)
    psi1 = np.broadcast_to(sx[None, None, :], (n, n, n)).copy()
    psi2 = np.broadcast_to(sy[None, :, None], (n, n, n)).copy()
    return psi1, psi2


def plane_wave(n: int, L: float, kvec, amp: float = 1.0):
    """amp * cos(k . x) sampled at x = (index) * dx, returned as an [z, y, x] array.

    ``kvec`` is (kx, ky, kz).
    """
    dx = L / n
    i = np.arange(n, dtype=np.float64) * dx
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    return amp * np.cos(kvec[0] * X + kvec[1] * Y + kvec[2] * Z)


def quadratic_field(shape, coeffs, origin=(-1, -1, -1)):
    """a x^2 + b y^2 + c z^2 + d xy + e yz + f zx at integer points (dx = 1).

    ``shape`` is (nz, ny, nx) and ``origin`` the (z, y, x) index of element [0, 0, 0];
    integer coefficients keep every value exactly representable.
    """
    a, b, c, d, e, f = coeffs
    z = np.arange(shape[0], dtype=np.float64) + origin[0]
    y = np.arange(shape[1], dtype=np.float64) + origin[1]
    x = np.arange(shape[2], dtype=np.float64) + origin[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return a * X * X + b * Y * Y + c * Z * Z + d * X * Y + e * Y * Z + f * Z * X
