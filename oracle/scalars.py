"""Time bookkeeping and per-stage scalars (oracle; test infrastructure only).

* Delta x_l = Delta x_0 / 2^l, Delta t_l = cfl * Delta x_l (section II, eq. dtscaling).
* The time of level l after k of its steps is eta0 + k * Delta t_l: one multiply and one
  add from integers, so levels that align in time hold bit-identical times.
* Classic RK4 (integrator type 4) evaluates the right-hand side at eta_n + c_s dt with
  c = (0, 1/2, 1/2, 1); the three-stage SSPRK3 (integrator types 3 and 10, the latter
  the same method stored in fewer buffers) at c = (0, 1, 1/2); the fourth-order
  Runge-Kutta-Nystrom method (integrator type 21) at c = (0, 1/2, 1); the fifth-order
  one (type 22) at c = (0, 1/5, 2/3, 1).
* The EOM (eq. EOM2 with lambda and the friction/potential exponents exposed) is
      dPi_i/deta = lap psi_i - (alpha/eta) Pi_i - lambda eta^beta psi_i (|psi|^2 - 1)
  so each stage needs c_fric = alpha / eta_s and c_pot = lambda * eta_s^beta, the
  power taken by repeated multiplication (beta is a small non-negative integer).
"""
from __future__ import annotations

RK4_C = (0.0, 0.5, 0.5, 1.0)
SSP3_C = (0.0, 1.0, 0.5)
RKN4_C = (0.0, 0.5, 1.0)
RKN5_C = (0.0, 0.2, 2.0 / 3.0, 1.0)


def stage_fractions(integrator: int):
    """c_s of the integrator: 4 = classic RK4, 3 or 10 = SSPRK3, 21 = RKN4, 22 = RKN5."""
    if integrator == 4:
        return RK4_C
    if integrator in (3, 10):
        return SSP3_C
    if integrator == 21:
        return RKN4_C
    if integrator == 22:
        return RKN5_C
    raise ValueError(f"unknown integrator {integrator}")


def level_dx(L: float, n0: int, lev: int) -> float:
    return (L / n0) / float(1 << lev)


def level_dt(L: float, n0: int, cfl: float, lev: int) -> float:
    return cfl * level_dx(L, n0, lev)


def level_time(eta0: float, k: int, dt: float) -> float:
    """Time after k steps of size dt from eta0."""
    return eta0 + float(k) * dt


def int_power(x: float, beta: int) -> float:
    p = 1.0
    for _ in range(beta):
        p = p * x
    return p


def stage_scalars(eta_n: float, dt: float, s: int, alpha: float, lam: float, beta: int, integrator: int = 4):
    """(eta_s, c_fric, c_pot) for stage s of the integrator."""
    eta_s = eta_n + stage_fractions(integrator)[s] * dt
    return eta_s, alpha / eta_s, lam * int_power(eta_s, beta)


def rk4_weights(dt: float):
    """(dt/6, dt/3, dt/2, dt): the classic RK4 stage and accumulation weights."""
    return dt / 6.0, dt / 3.0, dt * 0.5, dt


def rkn4_weights(dt: float):
    """Weights of the RKN4 tableau times powers of dt, each formed once in float64:
    (dt^2/6, dt^2/3, dt^2/8, dt^2/2) for the position and (dt/6, 2dt/3, dt/2, dt) for the
    velocity and the stage positions."""
    hh = dt * dt
    return hh / 6.0, hh / 3.0, hh * 0.125, hh * 0.5, dt / 6.0, (2.0 * dt) / 3.0, dt * 0.5, dt


# RKN5 (integrator type 22): a four-stage fifth-order Runge-Kutta-Nystrom tableau for
# y'' = f(t, y) (Hairer, Norsett and Wanner, Solving ODEs I, section II.14), as exact
# fractions: nodes, the lower-triangular a_ij, position weights bbar, velocity weights b.
RKN5_TABLEAU = {
    "c": ((0, 1), (1, 5), (2, 3), (1, 1)),
    "a": {(2, 1): (1, 50), (3, 1): (-1, 27), (3, 2): (7, 27), (4, 1): (3, 10), (4, 2): (-2, 35), (4, 3): (9, 35)},
    "bbar": ((1, 24), (25, 84), (9, 56), (0, 1)),
    "b": ((1, 24), (125, 336), (27, 56), (5, 48)),
}


def rkn5_weights(dt: float):
    """The RKN5 tableau times powers of dt, each formed once in float64 (numerator times
    the power first, then the division): a dict of the position weights w_ij = a_ij dt^2,
    pb_i = bbar_i dt^2, the velocity weights vb_i = b_i dt and the stage positions
    ch_i = c_i dt."""
    hh = dt * dt
    w = {}
    for (i, j), (num, den) in RKN5_TABLEAU["a"].items():
        v = (abs(num) * hh) / float(den) if abs(num) != 1 else hh / float(den)
        w[(i, j)] = -v if num < 0 else v
    pb = [((num * hh) / float(den) if num != 1 else hh / float(den)) for num, den in RKN5_TABLEAU["bbar"][:3]]
    vb = [((num * dt) / float(den) if num != 1 else dt / float(den)) for num, den in RKN5_TABLEAU["b"]]
    ch = [0.0, dt / 5.0, (2.0 * dt) / 3.0, dt]
    return {"w": w, "pb": pb, "vb": vb, "ch": ch}

