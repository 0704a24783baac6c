"""Right-hand side and classic RK4 step on one dense periodic lattice (oracle).

Test infrastructure only.  Follows the minimal example of the paper (eqs. EOM1 and
EOM2, the ``Rhs`` kernel function of section III.A) with the Laplacian of appendix A at
order 1, 2 or 3 (the 7-, 13- and 19-point stencils: order = ghost cells used per
direction), and integrator type 4 (classic RK4, appendix E) or SSPRK3.

The order-2 and order-3 stencils are the sums over the three axes of the standard
fourth- and sixth-order central second differences (coefficients 4/3, -1/12, -5/2 and
3/2, -3/20, 1/90, -49/18 per axis).  With S_r the sum of the six cells at distance r,

    S_r  = ((u[x-r] + u[x+r]) + (u[y-r] + u[y+r])) + (u[z-r] + u[z+r])
    lap1 = (S_1 - 6 u) * inv_dx2
    lap2 = ((4/3 S_1 + (-1/12) S_2) + (-15/2) u) * inv_dx2
    lap3 = (((3/2 S_1 + (-3/20) S_2) + 1/90 S_3) + (-49/6) u) * inv_dx2

(coefficients rounded once to the storage type).

Kreiss-Oliger dissipation (section II, "Kreiss-Oliger dissipation"): the operator
(-1)^((p+3)/2) eps dx^p / 2^(p+1) (d^(p+1)/dx^(p+1) + ...) is added to the right-hand side
of every component (psi and Pi), with the dissipation order d = 2 or 3 (the ghost cells it
needs) read as p = 2d - 1 and the (p+1)-st derivatives as the standard central
differences (1, -4, 6, -4, 1) / dx^4 and (1, -6, 15, -20, 15, -6, 1) / dx^6, so that

    K_2 = (S_2 + (-4) S_1) + 18 u                         Q = (-eps / (16 dx)) K_2
    K_3 = ((S_3 + (-6) S_2) + 15 S_1) + (-60) u           Q = ( eps / (64 dx)) K_3

with the coefficient formed in float64 and rounded once to the storage type.

Canonical operation order (both the oracle and the HIP path evaluate exactly these
expressions, with no fused multiply-add):

    lap   = lap1, lap2 or lap3 above
    r2    = psi1*psi1 + psi2*psi2
    pot   = c_pot * (r2 - 1)
    k_psi = Pi                                  (+ Q(psi) with dissipation)
    k_Pi  = (lap - c_fric * Pi) - pot * psi     (+ Q(Pi) with dissipation)

and RK4 in accumulator form (U_n the state at the step start, h = dt):

    stage 1: k1 = f(U_n);  acc = U_n + (h/6) k1;   U_a = U_n + (h/2) k1
    stage 2: k2 = f(U_a);  acc = acc + (h/3) k2;   U_b = U_n + (h/2) k2
    stage 3: k3 = f(U_b);  acc = acc + (h/3) k3;   U_a = U_n + h k3
    stage 4: k4 = f(U_a);  U_{n+1} = acc + (h/6) k4

which is the textbook y + h/6 (k1 + 2 k2 + 2 k3 + k4) with the sum formed as it goes.

SSPRK3 (integrator types 3 and 10, appendix E; the Shu-Osher form of the three-stage
third-order strong-stability-preserving method, stage times eta_n + (0, 1, 1/2) h):

    stage 1: U_a     = U_n + h f(U_n)
    stage 2: U_b     = 3/4 U_n + 1/4 (U_a + h f(U_a))
    stage 3: U_{n+1} = 1/3 U_n + 2/3 (U_b + h f(U_b))

RKN4 (integrator type 21, appendix E; appendix B's fourth-order Runge-Kutta-Nystrom
method).  The paper names the method but prints no tableau; it is read as Nystrom's
classical three-stage fourth-order scheme for y'' = f(t, y) (nodes c = (0, 1/2, 1),
a_21 = 1/8, a_31 = 0, a_32 = 1/2, position weights (1/6, 1/3, 0), velocity weights
(1/6, 2/3, 1/6); Hairer, Norsett and Wanner, Solving ODEs I, section II.14).  It applies
to the EOM only when the acceleration does not depend on Pi, i.e. without friction
(alpha = 0) and without dissipation; then with y = psi_n, v = Pi_n, h = dt and the
acceleration a(psi) = lap psi - c_pot (r2 - 1) psi (in the storage type, at the stage
time eta_n + c_s h):

    stage 1: a1 = a(U_n);  acc_psi = (y + h v) + (h^2/6) a1;  acc_Pi = v + (h/6) a1
             Y_psi = (y + (h/2) v) + (h^2/8) a1
    stage 2: a2 = a(Y);    acc_psi = acc_psi + (h^2/3) a2;    acc_Pi = acc_Pi + (2h/3) a2
             Y_psi = (y + h v) + (h^2/2) a2
    stage 3: a3 = a(Y);    psi_{n+1} = acc_psi;               Pi_{n+1} = acc_Pi + (h/6) a3

(the stage states carry Pi_n unchanged; acc is float64; the weights times powers of h
are formed once in float64, see scalars.rkn4_weights).

RKN5 (integrator type 22, appendix E; appendix B's fifth-order Runge-Kutta-Nystrom
method), also without a printed tableau: read as the four-stage fifth-order Nystrom
tableau of scalars.RKN5_TABLEAU (nodes c = (0, 1/5, 2/3, 1); its order conditions up to
order five are checked exactly in the tests).  Same EOM restriction as RKN4.  With
w_ij = a_ij h^2, pb_i = bbar_i h^2, vb_i = b_i h, ch_i = c_i h (scalars.rkn5_weights)
and the stage accelerations a_i = a(Y_i), Y_1 = psi_n:

    stage 1: P = pb_1 a_1;  V = vb_1 a_1;  Y_2 = (y + ch_2 v) + w_21 a_1
             S_3 = w_31 a_1;  S_4 = w_41 a_1
    stage 2: P = P + pb_2 a_2;  V = V + vb_2 a_2;  Y_3 = (y + ch_3 v) + (S_3 + w_32 a_2)
             S_4 = S_4 + w_42 a_2
    stage 3: P = P + pb_3 a_3;  V = V + vb_3 a_3;  Y_4 = (y + h v) + (S_4 + w_43 a_3)
    stage 4: psi_{n+1} = (y + h v) + P;  Pi_{n+1} = v + (V + vb_4 a_4)

(bbar_4 = 0).  P and V are the float64 accumulator; the partial sums S_3 and S_4 of the
later stage arguments are kept in the storage type (they ride in the Pi components of
the stage states, which a Nystrom stage does not otherwise use): exact in FP64 storage,
rounded to float32 in FP32 storage.

Mixed precision (FP32 storage): U_n, U_a, U_b are float32 and the right-hand side is
evaluated in float32 (scalars rounded to float32 once); every update above is done in
float64 from the promoted float32 values and rounded to float32 on store, while ``acc``
stays float64.
"""
from __future__ import annotations

import numpy as np

from .scalars import rk4_weights, rkn4_weights, rkn5_weights, stage_scalars


def lap7(u: np.ndarray, inv_dx2) -> np.ndarray:
    """7-point Laplacian of a periodic [z, y, x] array, in the array's own precision."""
    t = u.dtype.type
    xm = np.roll(u, 1, axis=2)
    xp = np.roll(u, -1, axis=2)
    ym = np.roll(u, 1, axis=1)
    yp = np.roll(u, -1, axis=1)
    zm = np.roll(u, 1, axis=0)
    zp = np.roll(u, -1, axis=0)
    return ((((xm + xp) + (ym + yp)) + (zm + zp)) - t(6.0) * u) * t(inv_dx2)


# per-order coefficients of S_1, S_2, S_3 and of the centre cell (appendix A orders 2, 3)
LAP_COEF = {2: (4.0 / 3.0, -1.0 / 12.0, None, -15.0 / 2.0),
            3: (3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0, -49.0 / 6.0)}


def _S(u: np.ndarray, r: int) -> np.ndarray:
    """Sum of the six cells at distance r, ((x-r + x+r) + (y-r + y+r)) + (z-r + z+r)."""
    return (((np.roll(u, r, axis=2) + np.roll(u, -r, axis=2)) + (np.roll(u, r, axis=1) + np.roll(u, -r, axis=1)))
            + (np.roll(u, r, axis=0) + np.roll(u, -r, axis=0)))


def ko_coef(ko_order: int, eps: float, dx: float) -> float:
    """Coefficient of the Kreiss-Oliger sum K for dissipation order 2 (p = 3) or 3 (p = 5)."""
    if ko_order == 2:
        return -eps / (16.0 * dx)
    if ko_order == 3:
        return eps / (64.0 * dx)
    raise ValueError(f"no dissipation of order {ko_order}")


def ko_term(u: np.ndarray, ko_order: int, coef) -> np.ndarray:
    """Kreiss-Oliger term coef * K of a periodic array, in its own precision."""
    t = u.dtype.type
    if ko_order == 2:
        K = (_S(u, 2) + t(-4.0) * _S(u, 1)) + t(18.0) * u
    elif ko_order == 3:
        K = ((_S(u, 3) + t(-6.0) * _S(u, 2)) + t(15.0) * _S(u, 1)) + t(-60.0) * u
    else:
        raise ValueError(f"no dissipation of order {ko_order}")
    return t(coef) * K


def lap(u: np.ndarray, inv_dx2, order: int = 1) -> np.ndarray:
    """Laplacian of appendix A at the given order (1, 2, 3: 7-, 13-, 19-point) of a
    periodic [z, y, x] array, in the array's own precision."""
    if order == 1:
        return lap7(u, inv_dx2)
    if order not in LAP_COEF:
        raise ValueError(f"no Laplacian of order {order}")
    t = u.dtype.type

    c1, c2, c3, c0 = LAP_COEF[order]
    acc = t(c1) * _S(u, 1) + t(c2) * _S(u, 2)
    if order == 3:
        acc = acc + t(c3) * _S(u, 3)
    return (acc + t(c0) * u) * t(inv_dx2)


def rhs(U: np.ndarray, inv_dx2: float, c_fric: float, c_pot: float, order: int = 1, ko=None) -> np.ndarray:
    """f(U) for eqs. EOM1/EOM2 on a periodic lattice, in U's precision; ``ko`` = (dissipation
    order, coefficient from ko_coef) adds Kreiss-Oliger dissipation to every component."""
    t = U.dtype.type
    p1, p2, q1, q2 = U[0], U[1], U[2], U[3]
    cf = t(c_fric)
    cp = t(c_pot)
    r2 = p1 * p1 + p2 * p2
    pot = cp * (r2 - t(1.0))
    K = np.empty_like(U)
    K[0] = q1
    K[1] = q2
    K[2] = (lap(p1, inv_dx2, order) - cf * q1) - pot * p1
    K[3] = (lap(p2, inv_dx2, order) - cf * q2) - pot * p2
    if ko is not None and ko[0]:
        for c in range(4):
            K[c] = K[c] + ko_term(U[c], ko[0], ko[1])
    return K


def accel(U: np.ndarray, inv_dx2: float, c_pot: float, order: int = 1) -> np.ndarray:
    """Acceleration of psi1, psi2 without friction, lap psi - c_pot (r2 - 1) psi, as a
    (2, ...) array in U's precision."""
    t = U.dtype.type
    p1, p2 = U[0], U[1]
    r2 = p1 * p1 + p2 * p2
    pot = t(c_pot) * (r2 - t(1.0))
    return np.stack([lap(p1, inv_dx2, order) - pot * p1, lap(p2, inv_dx2, order) - pot * p2])


def rkn4_stage(s: int, X: np.ndarray, Un: np.ndarray, acc, eta_n: float, dt: float, inv_dx2: float,
               lam: float, beta: int, order: int = 1):
    """Stage s (0-based) of RKN4 (friction-free EOM): returns (acc, Y), acc the float64
    (4, ...) accumulator (psi then Pi), Y the next stage state (s < 2) or U_{n+1} (s = 2),
    in Un's precision."""
    st = Un.dtype
    hh6, hh3, hh8, hh2, h6, h23, h2, h1 = rkn4_weights(dt)
    _, _, cp = stage_scalars(eta_n, dt, s, 0.0, lam, beta, integrator=21)
    a = accel(X, inv_dx2, cp, order).astype(np.float64)
    y = Un[:2].astype(np.float64)
    v = Un[2:].astype(np.float64)
    Y = np.empty_like(Un)
    if s == 0:
        acc = np.concatenate([(y + h1 * v) + hh6 * a, v + h6 * a])
        Y[:2] = ((y + h2 * v) + hh8 * a).astype(st)
        Y[2:] = Un[2:]
    elif s == 1:
        acc = np.concatenate([acc[:2] + hh3 * a, acc[2:] + h23 * a])
        Y[:2] = ((y + h1 * v) + hh2 * a).astype(st)
        Y[2:] = Un[2:]
    else:
        Y[:2] = acc[:2].astype(st)
        Y[2:] = (acc[2:] + h6 * a).astype(st)
    return acc, Y


def rkn4_step(U: np.ndarray, eta_n: float, dt: float, inv_dx2: float, lam: float, beta: int, fill=None,
              order: int = 1) -> np.ndarray:
    """One RKN4 step of the friction-free EOM; ``fill(s, X)`` as for ``rk4_step``."""
    X, acc = U, None
    for s in range(3):
        if s > 0 and fill is not None:
            fill(s, X)
        acc, X = rkn4_stage(s, X, U, acc, eta_n, dt, inv_dx2, lam, beta, order)
    return X


def rkn5_stage(s: int, X: np.ndarray, Un: np.ndarray, acc, S, eta_n: float, dt: float, inv_dx2: float,
               lam: float, beta: int, order: int = 1):
    """Stage s (0-based) of RKN5 (friction-free EOM).  X: the stage argument (psi in
    X[:2]); acc: the float64 (P, V) accumulator, (4, ...); S: the partial sums in the
    storage type, {3: S_3, 4: S_4} (2 components each).  Returns (acc, S, Y): Y the next
    stage argument's psi (s < 3) or U_{n+1} (s = 3), in Un's precision."""
    st = Un.dtype
    W = rkn5_weights(dt)
    w, pb, vb, ch = W["w"], W["pb"], W["vb"], W["ch"]
    _, _, cp = stage_scalars(eta_n, dt, s, 0.0, lam, beta, integrator=22)
    a = accel(X, inv_dx2, cp, order).astype(np.float64)
    y = Un[:2].astype(np.float64)
    v = Un[2:].astype(np.float64)
    if s == 0:
        acc = np.concatenate([pb[0] * a, vb[0] * a])
        S = {3: (w[(3, 1)] * a).astype(st), 4: (w[(4, 1)] * a).astype(st)}
        return acc, S, ((y + ch[1] * v) + w[(2, 1)] * a).astype(st)
    if s == 1:
        acc = np.concatenate([acc[:2] + pb[1] * a, acc[2:] + vb[1] * a])
        Y = ((y + ch[2] * v) + (S[3].astype(np.float64) + w[(3, 2)] * a)).astype(st)
        S = {3: S[3], 4: (S[4].astype(np.float64) + w[(4, 2)] * a).astype(st)}
        return acc, S, Y
    if s == 2:
        acc = np.concatenate([acc[:2] + pb[2] * a, acc[2:] + vb[2] * a])
        return acc, S, ((y + ch[3] * v) + (S[4].astype(np.float64) + w[(4, 3)] * a)).astype(st)
    Y = np.empty_like(Un)
    Y[:2] = ((y + ch[3] * v) + acc[:2]).astype(st)
    Y[2:] = (v + (acc[2:] + vb[3] * a)).astype(st)
    return acc, S, Y


def rkn5_step(U: np.ndarray, eta_n: float, dt: float, inv_dx2: float, lam: float, beta: int, fill=None,
              order: int = 1) -> np.ndarray:
    """One RKN5 step of the friction-free EOM; ``fill(s, X)`` as for ``rk4_step`` (X holds
    the stage argument's psi in X[:2])."""
    X, acc, S = U, None, None
    for s in range(4):
        if s > 0 and fill is not None:
            fill(s, X)
        acc, S, Y = rkn5_stage(s, X, U, acc, S, eta_n, dt, inv_dx2, lam, beta, order)
        if s < 3:
            X = np.concatenate([Y, U[2:]])
        else:
            X = Y
    return X


def rk4_stage(s: int, X: np.ndarray, Un: np.ndarray, acc, eta_n: float, dt: float,
              inv_dx2: float, alpha: float, lam: float, beta: int, order: int = 1, ko=None):
    """Stage s (0-based) of classic RK4 in accumulator form.

    X is the stage input (U_n itself for s = 0), Un the state at the step start, acc the
    float64 accumulator (ignored for s = 0).  Returns (acc, Y): Y is the next stage input
    for s < 3 and U_{n+1} for s = 3, in the storage precision of Un.
    """
    st = Un.dtype
    h6, h3, h2, h1 = rk4_weights(dt)
    _, cf, cp = stage_scalars(eta_n, dt, s, alpha, lam, beta)
    k = rhs(X, inv_dx2, cf, cp, order, ko).astype(np.float64)
    if s == 3:
        return acc, (acc + h6 * k).astype(st)
    U64 = Un.astype(np.float64)
    if s == 0:
        acc = U64 + h6 * k
        Y = U64 + h2 * k
    elif s == 1:
        acc = acc + h3 * k
        Y = U64 + h2 * k
    else:
        acc = acc + h3 * k
        Y = U64 + h1 * k
    return acc, Y.astype(st)


def check_rkn(alpha: float, ko_order: int):
    """The Nystrom methods (RKN4, RKN5) need an acceleration independent of Pi: no
    friction, no dissipation."""
    if alpha != 0.0 or ko_order:
        raise ValueError("RKN4 and RKN5 integrate the friction-free EOM only (alpha = 0, no dissipation)")


def ssprk3_stage(s: int, X: np.ndarray, Un: np.ndarray, eta_n: float, dt: float, inv_dx2: float,
                 alpha: float, lam: float, beta: int, order: int = 1, ko=None) -> np.ndarray:
    """Stage s (0-based) of SSPRK3: the next stage input (s < 2) or U_{n+1} (s = 2), in
    the storage precision of Un; updates in float64 from promoted values."""
    st = Un.dtype
    _, cf, cp = stage_scalars(eta_n, dt, s, alpha, lam, beta, integrator=10)
    k = rhs(X, inv_dx2, cf, cp, order, ko).astype(np.float64)
    U64 = Un.astype(np.float64)
    if s == 0:
        Y = U64 + dt * k
    elif s == 1:
        Y = 0.75 * U64 + 0.25 * (X.astype(np.float64) + dt * k)
    else:
        Y = (1.0 / 3.0) * U64 + (2.0 / 3.0) * (X.astype(np.float64) + dt * k)
    return Y.astype(st)


def ssprk3_step(U: np.ndarray, eta_n: float, dt: float, inv_dx2: float,
                alpha: float, lam: float, beta: int, fill=None, order: int = 1, ko=None) -> np.ndarray:
    """One SSPRK3 step; ``fill(s, X)`` as for ``rk4_step``."""
    X = U
    for s in range(3):
        if s > 0 and fill is not None:
            fill(s, X)
        X = ssprk3_stage(s, X, U, eta_n, dt, inv_dx2, alpha, lam, beta, order, ko)
    return X


def rk4_step(U: np.ndarray, eta_n: float, dt: float, inv_dx2: float,
             alpha: float, lam: float, beta: int, fill=None, order: int = 1, ko=None) -> np.ndarray:
    """One classic RK4 step of size dt from time eta_n; returns U_{n+1} (U's dtype).

    ``fill(s, X)``, if given, is called on the stage input X before stages s = 1, 2, 3
    (0-based) to set ghost values in place; a periodic single level needs none.
    """
    X = U
    acc = None
    for s in range(4):
        if s > 0 and fill is not None:
            fill(s, X)
        acc, X = rk4_stage(s, X, U, acc, eta_n, dt, inv_dx2, alpha, lam, beta, order, ko)
    return X


def run_single_level(U0: np.ndarray, nsteps: int, eta0: float, dt: float, dx: float,
                     alpha: float = 2.0, lam: float = 1.0, beta: int = 2,
                     callback=None, integrator: int = 4, order: int = 1, ko_order: int = 0,
                     ko_eps: float = 0.0) -> np.ndarray:
    """nsteps steps (RK4; SSPRK3 for integrator 3/10; RKN4 / RKN5 for 21 / 22) of a periodic lattice with the
    Laplacian of the given order and, for ko_order 2 or 3, Kreiss-Oliger dissipation of
    strength ko_eps; step k starts at eta0 + k*dt.

    ``callback(k, U)`` is called after each step with the 1-based step count.
    """
    from .scalars import level_time, stage_fractions
    stage_fractions(integrator)  # validates
    inv_dx2 = 1.0 / (dx * dx)
    ko = (ko_order, ko_coef(ko_order, ko_eps, dx)) if ko_order else None
    if integrator in (21, 22):
        check_rkn(alpha, ko_order)
        nystrom = rkn4_step if integrator == 21 else rkn5_step

        def step(U, eta, dt, inv_dx2, alpha, lam, beta, order=1, ko=None):
            return nystrom(U, eta, dt, inv_dx2, lam, beta, order=order)
    else:
        step = rk4_step if integrator == 4 else ssprk3_step
    U = U0.copy()
    for k in range(nsteps):
        U = step(U, level_time(eta0, k, dt), dt, inv_dx2, alpha, lam, beta, order=order, ko=ko)
        if callback is not None:
            callback(k + 1, U)
    return U
