"""Berger-Oliger AMR hierarchy on dense per-level arrays (oracle; test infrastructure).

Representation: level l is one dense periodic array over the whole domain at spacing
dx_l = dx_0 / 2^l, plus a boolean mask of its valid cells (the union of its boxes).
Cells within `depth` cells of the valid region (Chebyshev distance, periodic; depth =
the widest stencil: the Laplacian order of appendix A, 1 for the 7-point stencil, or the
Kreiss-Oliger dissipation order) are its ghost cells.  A
ghost cell that is a valid cell of another box of the same level is simply that cell
here, so same-level ghost copies (periodic images included) are implicit and always
current; the remaining ghost cells are set by coarse-to-fine interpolation.

Paper passages followed:
* Subcycling (section II.A, Fig. 2): level l is advanced by dt_l, then level l+1 twice
  by dt_l/2, then the two levels are synchronised.
* Ghost cells of a fine level are interpolated from the coarse level in space and time,
  at every intermediate stage, using the coarse states at the start and end of the
  coarse step (section II.A).  Spatial scheme: linear conservative (interpolation type
  1, appendix E "AMR parameters"), read here as unlimited central slopes
      f = C_I + sum_d s_d (C_{I+e_d} - C_{I-e_d}) / 2,   s_d = +-1/4 the child offset,
  evaluated as ((C_I + t_x) + t_y) + t_z with t_d = (C_{I+e_d} - C_{I-e_d}) * (+-1/8).
  Temporal: C(alpha) = (1 - alpha) C_old + alpha C_new, interpolated in time first;
  alpha = 0 and alpha = 1 take C_old and C_new themselves.
  Quartic conservative (interpolation type 4, the paper's default) is read as the tensor
  product of the 1-D conservative quartic: the quartic whose averages over the five coarse
  cells I-2..I+2 are the coarse values, averaged over the child half-cells, which gives
      f = C_I + t,  t = (C_{I+1} - C_{I-1}) * (+-11/64) + (C_{I+2} - C_{I-2}) * (-+3/128)
  (upper signs for the upper child); applied along x for the 5 x 5 (y, z) neighbours of
  the parent, then along y for the 5 z neighbours, then along z.  Fine sub-step j in {0, 1}
  at stage fraction c_s has alpha = (j + c_s) / 2; c = (0, 1/2, 1/2, 1) for RK4 and
  (0, 1, 1/2) for SSPRK3 (the three-stage method of appendix E's parameter list).
* Synchronisation (section II.A): the fine level is averaged onto the coarse cells it
  covers, c = ((((f000+f100)+(f010+f110))+((f001+f101)+(f011+f111))) * 1/8), and the
  fine ghost cells are set again with no temporal interpolation (alpha = 1).
* Operation order per level step, reproducing the numbering of Fig. 2: stage 1, then
  (fill, stage) for the remaining stages; after the last stage a fill of the new state
  at the step's end time unless the step is the second sub-step, whose end is the
  synchronisation that sets the ghosts itself.
* Regrid (section II "regridding"): new valid cells keep the old level's values where
  it already had valid cells and are interpolated from the coarse level elsewhere.

* Truncation error estimates (section II.B, "self-shadow"; section IV.C): a fine level
  and its coarse level are evolved independently between synchronisations, so just
  before the fine level is averaged onto the coarse one their difference estimates the
  truncation error.  Read here as the difference at the coarse resolution,
      TEE(X) = max over the four components of |C(X) - avg(children of X)|,
  the average taken in the order above, every fine cell carrying the value of its coarse
  parent (the maximum keeps the first component unless a later one compares greater).
  Level 0 has no coarser level; a shadow level (level 0 averaged onto half its
  resolution, when level 0 has taken an even number of steps) is evolved by one step of
  twice the level-0 step while level 0 takes two, and the same difference between the
  shadow and level 0 gives the estimate on level 0.  Cells are tagged where the estimate
  exceeds a threshold (te_crit, one for all components), alone or together with the
  plaquette criterion.  On a regrid the estimate of kept cells is kept and new cells
  start at 0.
* Per-field estimates and their modifier (section IV.C, "Modifying truncation error
  estimates"): with tee_fields on, each component c keeps its own estimate
  Delta_c(X) = |C_c(X) - avg(children)_c| and a cell is tagged by estimate when
  f_c(Delta_c) > eps_c for some component, with its own threshold eps_c (te_crit_phi)
  and f_c(Delta) = s_c * Delta.  The paper's modifier is a user function with user
  parameters; the one built here is the scaling it uses in appendix D (Delta_phi / max phi
  and Delta_phi' / max phi'), with s_c given by the caller.  ``field_absmax`` gives the
  maxima for that normalisation, read as max |U_c| over the valid cells of every level
  (the whole simulation); ``normalising_scales`` turns them into s_c = 1 / max, leaving a
  component whose maximum is 0 unscaled (s_c = 1).

Interpolation and averaging are done in float64 from promoted values and rounded to
the storage precision on store.
"""
from __future__ import annotations

import numpy as np

from .scalars import level_dt, level_dx, level_time, int_power, stage_fractions
from .level import check_rkn, ko_coef, rk4_stage, rkn4_stage, ssprk3_stage
from .tagging import tag_cells
from .energy import energy as _energy


def boxes_mask(boxes, M: int) -> np.ndarray:
    """Valid mask of boxes (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi), inclusive, in [0, M)."""
    m = np.zeros((M, M, M), dtype=bool)
    for b in boxes:
        xl, yl, zl, xh, yh, zh = (int(v) for v in b)
        if min(xl, yl, zl) < 0 or max(xh, yh, zh) >= M or xl > xh or yl > yh or zl > zh:
            raise ValueError(f"box {b} outside the level domain [0, {M})")
        if m[zl:zh + 1, yl:yh + 1, xl:xh + 1].any():
            raise ValueError(f"box {b} overlaps another box")
        m[zl:zh + 1, yl:yh + 1, xl:xh + 1] = True
    return m


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    """Periodic dilation by r cells in every direction (a (2r+1)^3 cube)."""
    out = mask.copy()
    for ax in range(3):
        cur = out.copy()
        for s in range(1, r + 1):
            cur |= np.roll(out, s, axis=ax) | np.roll(out, -s, axis=ax)
        out = cur
    return out


def erode(mask: np.ndarray, r: int) -> np.ndarray:
    return ~dilate(~mask, r)


def ghost_mask(valid: np.ndarray, depth: int = 1) -> np.ndarray:
    return dilate(valid, depth) & ~valid


def coarsen_mask(fine: np.ndarray) -> np.ndarray:
    """Coarse cells any of whose 8 children is set."""
    return fine.reshape(fine.shape[0] // 2, 2, fine.shape[1] // 2, 2,
                        fine.shape[2] // 2, 2).any(axis=(1, 3, 5))


def refine_mask(coarse: np.ndarray) -> np.ndarray:
    return coarse.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def time_interp(Cold, Cnew, alpha: float) -> np.ndarray:
    """(1 - alpha) C_old + alpha C_new in float64; alpha 0 / 1 return C_old / C_new."""
    if alpha == 1.0:
        return Cnew.astype(np.float64)
    if alpha == 0.0:
        return Cold.astype(np.float64)
    return (1.0 - alpha) * Cold.astype(np.float64) + alpha * Cnew.astype(np.float64)


def _quartic_1d(cm2, cm1, c0, cp1, cp2, upper):
    """1-D conservative quartic child average (float64): c0 + t in the canonical order."""
    a = np.where(upper, 11.0 / 64.0, -11.0 / 64.0)
    b = np.where(upper, -3.0 / 128.0, 3.0 / 128.0)
    return c0 + ((cp1 - cm1) * a + (cp2 - cm2) * b)


def interp_cells_quartic(C: np.ndarray, fz: np.ndarray, fy: np.ndarray, fx: np.ndarray) -> np.ndarray:
    """Quartic conservative interpolation of coarse array C at fine cells (fz, fy, fx)."""
    Mc = C.shape[0]
    Iz, Iy, Ix = fz // 2, fy // 2, fx // 2
    ux, uy, uz = (fx & 1) == 1, (fy & 1) == 1, (fz & 1) == 1

    def at(dz, dy, dx):
        return C[(Iz + dz) % Mc, (Iy + dy) % Mc, (Ix + dx) % Mc]

    hz = []
    for dz in range(-2, 3):
        gy = []
        for dy in range(-2, 3):
            gy.append(_quartic_1d(at(dz, dy, -2), at(dz, dy, -1), at(dz, dy, 0), at(dz, dy, 1), at(dz, dy, 2), ux))
        hz.append(_quartic_1d(gy[0], gy[1], gy[2], gy[3], gy[4], uy))
    return _quartic_1d(hz[0], hz[1], hz[2], hz[3], hz[4], uz)


def interp_cells(C: np.ndarray, fz: np.ndarray, fy: np.ndarray, fx: np.ndarray, kind: int = 1) -> np.ndarray:
    """Conservative interpolation of coarse array C at fine cells (fz, fy, fx): linear
    (kind 1) or quartic (kind 4)."""
    if kind == 4:
        return interp_cells_quartic(C, fz, fy, fx)
    if kind != 1:
        raise ValueError(f"no interpolation of type {kind}")
    Mc = C.shape[0]
    Iz, Iy, Ix = fz // 2, fy // 2, fx // 2
    sx = np.where(fx & 1, 0.125, -0.125)
    sy = np.where(fy & 1, 0.125, -0.125)
    sz = np.where(fz & 1, 0.125, -0.125)
    c0 = C[Iz, Iy, Ix]
    tx = (C[Iz, Iy, (Ix + 1) % Mc] - C[Iz, Iy, (Ix - 1) % Mc]) * sx
    ty = (C[Iz, (Iy + 1) % Mc, Ix] - C[Iz, (Iy - 1) % Mc, Ix]) * sy
    tz = (C[(Iz + 1) % Mc, Iy, Ix] - C[(Iz - 1) % Mc, Iy, Ix]) * sz
    return ((c0 + tx) + ty) + tz


def interp_support(fz, fy, fx, Mc: int, kind: int = 1) -> np.ndarray:
    """Coarse cells (as a mask) read by interp_cells at the given fine cells."""
    m = np.zeros((Mc, Mc, Mc), dtype=bool)
    Iz, Iy, Ix = fz // 2, fy // 2, fx // 2
    if kind == 4:
        for dz in range(-2, 3):
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    m[(Iz + dz) % Mc, (Iy + dy) % Mc, (Ix + dx) % Mc] = True
        return m
    m[Iz, Iy, Ix] = True
    for d in (-1, 1):
        m[Iz, Iy, (Ix + d) % Mc] = True
        m[Iz, (Iy + d) % Mc, Ix] = True
        m[(Iz + d) % Mc, Iy, Ix] = True
    return m


def average_down_arrays(F: np.ndarray) -> np.ndarray:
    """2^3 -> 1 mean of a fine [z, y, x] array (float64), in the canonical order."""
    f = F.astype(np.float64)

    def c(dx, dy, dz):
        return f[dz::2, dy::2, dx::2]

    return ((((c(0, 0, 0) + c(1, 0, 0)) + (c(0, 1, 0) + c(1, 1, 0)))
             + ((c(0, 0, 1) + c(1, 0, 1)) + (c(0, 1, 1) + c(1, 1, 1)))) * 0.125)


def tee_coarse(C: np.ndarray, F: np.ndarray) -> np.ndarray:
    """TEE at the coarse resolution: max over components of |C - avg(F children)|
    (C: (4, M, M, M) coarse state, F: (4, 2M, 2M, 2M) fine state; float64)."""
    t = None
    for c in range(4):
        with np.errstate(all="ignore"):
            d = np.abs(C[c].astype(np.float64) - average_down_arrays(F[c]))
        t = d if t is None else np.where(d > t, d, t)
    return t


def tee_coarse_fields(C: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Per-component TEE at the coarse resolution: (4, M, M, M) array of
    |C_c - avg(F_c children)| (float64)."""
    out = np.empty((4,) + C.shape[1:])
    for c in range(4):
        with np.errstate(all="ignore"):
            out[c] = np.abs(C[c].astype(np.float64) - average_down_arrays(F[c]))
    return out


def normalising_scales(absmax) -> np.ndarray:
    """s_c = 1 / max |U_c| (appendix D's normalisation); 1 where the maximum is 0."""
    m = np.asarray(absmax, dtype=np.float64)
    return np.where(m > 0.0, 1.0 / np.where(m > 0.0, m, 1.0), 1.0)


def refine_values(T: np.ndarray) -> np.ndarray:
    """Each coarse value onto its 2^3 children."""
    return np.repeat(np.repeat(np.repeat(T, 2, axis=0), 2, axis=1), 2, axis=2)


def schedule(finest: int, nstages: int):
    """Operations of one coarse step with levels 0..finest and an nstages integrator.

    ("stage", l, s): RK stage s of level l;  ("fill", l, j, s): ghost fill of level l in
    sub-step j before stage s (s == nstages: the new state at the step end);
    ("sync", l): average level l onto l-1 and refill the ghosts of level l.
    A step of level l >= 1 is the j-th of the two sub-steps of its parent's step.
    """
    ops = []

    def step(lev, sub):
        for s in range(nstages):
            if s > 0:
                ops.append(("fill", lev, sub, s))
            ops.append(("stage", lev, s))
        if lev > 0 and sub == 0:
            ops.append(("fill", lev, sub, nstages))
        if lev < finest:
            step(lev + 1, 0)
            step(lev + 1, 1)
            ops.append(("sync", lev + 1))

    step(0, 0)
    return ops


class Level:
    def __init__(self, M: int, dx: float, dt: float):
        self.M, self.dx, self.dt = M, dx, dt
        self.valid = np.zeros((M, M, M), dtype=bool)
        self.ghost = np.zeros((M, M, M), dtype=bool)
        self.boxes = []
        self.U = None
        self.Uold = None
        self.X = None
        self.acc = None
        self.k = 0
        self.tee = np.zeros((M, M, M))


class Hierarchy:
    """Oracle AMR hierarchy.  Layouts are inputs (``set_layout``); nothing is clustered."""

    def __init__(self, n0: int, L: float, cfl: float, eta0: float, max_level: int,
                 alpha: float = 2.0, lam: float = 1.0, beta: int = 2,
                 dtype=np.float64, check_nesting: bool = True, integrator: int = 4, order: int = 1,
                 interp: int = 1, ko_order: int = 0, ko_eps: float = 0.0):
        self.n0, self.L, self.cfl, self.eta0 = n0, L, cfl, eta0
        self.max_level = max_level
        self.alpha, self.lam, self.beta = alpha, lam, beta
        self.dtype = np.dtype(dtype)
        self.check_nesting = check_nesting
        self.integrator = integrator
        self.cs = stage_fractions(integrator)
        self.order = order  # Laplacian order = ghost depth of the refined levels
        self.interp = interp  # spatial interpolation: 1 linear, 4 quartic (conservative)
        # Kreiss-Oliger dissipation (order 2 or 3, 0 = off): it stencils every component,
        # so fills then cover Pi too, and ghost shells are as deep as the widest stencil
        self.ko_order, self.ko_eps = ko_order, ko_eps
        self.depth = max(order, ko_order)
        if integrator == 21:
            check_rkn(alpha, ko_order)
        if integrator == 22:
            # RKN5 is read for single periodic levels (appendix B's use), where
            # run_single_level integrates it; a hierarchy would need coarse/fine fills at
            # the nodes 1/5 and 2/3 of a step
            raise ValueError("RKN5 (integrator 22) runs on single levels only (oracle.level.run_single_level)")
        self.levels: list[Level] = []
        self.trace: list[tuple] = []
        self.tee_on = False
        self.te_crit = 0.0
        # per-field estimates: thresholds eps_c and modifier scales s_c
        self.tee_fields = False
        self.te_crit_c = np.zeros(4)
        self.te_scale = np.ones(4)
        self.tag_mode = 1  # bit 0: plaquette winding, bit 1: truncation error estimate
        self.shadow: Level | None = None

    # ---- bookkeeping -------------------------------------------------------------
    @property
    def finest(self) -> int:
        return len(self.levels) - 1

    def time(self, lev: int) -> float:
        L = self.levels[lev]
        return level_time(self.eta0, L.k, L.dt)

    def _new_level(self, lev: int) -> Level:
        M = self.n0 << lev
        L = Level(M, level_dx(self.L, self.n0, lev), level_dt(self.L, self.n0, self.cfl, lev))
        L.tee = self._tee_zeros(M)
        return L

    # ---- layout ------------------------------------------------------------------
    def set_level0(self, U0: np.ndarray, boxes=None):
        M = self.n0
        L = self._new_level(0)
        if boxes is None:
            boxes = [(0, 0, 0, M - 1, M - 1, M - 1)]
        L.valid = boxes_mask(boxes, M)
        if not L.valid.all():
            raise ValueError("level 0 must cover the whole domain")
        L.boxes = [tuple(b) for b in boxes]
        L.U = U0.astype(self.dtype).copy()
        self.levels = [L]

    def set_layout(self, lev: int, boxes):
        """Set (or change, or with no boxes remove) the layout of level lev >= 1."""
        if lev < 1 or lev > len(self.levels) or lev > self.max_level:
            raise ValueError("bad level")
        if len(boxes) == 0:
            del self.levels[lev:]
            return
        C = self.levels[lev - 1]
        if lev == len(self.levels):
            L = self._new_level(lev)
            L.k = 2 * C.k
            old_valid = np.zeros((L.M,) * 3, dtype=bool)
            oldU = None
            self.levels.append(L)
        else:
            L = self.levels[lev]
            old_valid = L.valid
            oldU = L.U
        new_valid = boxes_mask(boxes, L.M)
        if self.check_nesting:
            need = dilate(coarsen_mask(new_valid), 1 if self.interp == 1 else 2)
            if not np.all(C.valid[need]):
                raise ValueError("level not nested in its coarse level")
        U = np.full((4, L.M, L.M, L.M), np.nan, dtype=self.dtype)
        keep = new_valid & old_valid
        if oldU is not None:
            U[:, keep] = oldU[:, keep]
        tee = self._tee_zeros(L.M)
        tee[..., keep] = L.tee[..., keep] if L.tee.shape == tee.shape else 0.0
        L.tee = tee
        fresh = new_valid & ~old_valid
        fz, fy, fx = np.nonzero(fresh)
        for c in range(4):
            U[c][fz, fy, fx] = interp_cells(C.U[c].astype(np.float64), fz, fy, fx, self.interp).astype(self.dtype)
        L.valid = new_valid
        L.ghost = ghost_mask(new_valid, self.depth)
        L.boxes = [tuple(b) for b in boxes]
        L.U = U
        L.Uold = None
        self.fill(lev, L.U, 1.0)

    # ---- ghost fill (coarse -> fine) ---------------------------------------------
    def fill(self, lev: int, X: np.ndarray, alpha: float):
        """Set the coarse/fine ghost cells of the psi components of X (level lev)."""
        if lev == 0:
            return
        L, C = self.levels[lev], self.levels[lev - 1]
        fz, fy, fx = np.nonzero(L.ghost)
        if self.check_nesting and fz.size:
            sup = interp_support(fz, fy, fx, C.M, self.interp)
            if not np.all(C.valid[sup]):
                raise ValueError("ghost interpolation reads coarse cells outside the coarse level")
        for c in ((0, 1, 2, 3) if self.ko_order else (0, 1)):
            Cold = C.Uold[c] if C.Uold is not None else None
            Ct = time_interp(Cold, C.U[c], alpha)
            X[c][fz, fy, fx] = interp_cells(Ct, fz, fy, fx, self.interp).astype(X.dtype)

    # ---- stepping ----------------------------------------------------------------
    def coarse_step(self):
        """One coarse step: every level advanced in the order of ``schedule``."""
        nstages = len(self.cs)
        ops = schedule(self.finest, nstages)
        for op in ops:
            self.trace.append(op)
            if op[0] == "stage":
                self._stage(op[1], op[2])
            elif op[0] == "fill":
                _, lev, sub, s = op
                L = self.levels[lev]
                c = 1.0 if s == nstages else self.cs[s]
                self.fill(lev, L.U if s == nstages else L.X, (sub + c) / 2.0)
            else:
                self.average_down(op[1])
                self.fill(op[1], self.levels[op[1]].U, 1.0)

    def _stage(self, lev: int, s: int):
        L = self.levels[lev]
        eta_n = level_time(self.eta0, L.k, L.dt)
        X = L.U if s == 0 else L.X
        last = len(self.cs) - 1
        ko = self._ko(L.dx)
        with np.errstate(all="ignore"):
            if self.integrator == 4:
                L.acc, Y = rk4_stage(s, X, L.U, L.acc if s else None, eta_n, L.dt,
                                     1.0 / (L.dx * L.dx), self.alpha, self.lam, self.beta, self.order, ko)
            elif self.integrator == 21:
                L.acc, Y = rkn4_stage(s, X, L.U, L.acc if s else None, eta_n, L.dt, 1.0 / (L.dx * L.dx),
                                      self.lam, self.beta, self.order)
            else:
                Y = ssprk3_stage(s, X, L.U, eta_n, L.dt, 1.0 / (L.dx * L.dx), self.alpha, self.lam, self.beta,
                                 self.order, ko)
        if s == last:
            L.Uold, L.U, L.X, L.acc = L.U, Y, None, None
            L.k += 1
        else:
            L.X = Y

    def _ko(self, dx: float):
        return (self.ko_order, ko_coef(self.ko_order, self.ko_eps, dx)) if self.ko_order else None

    def average_down(self, fine: int):
        F, C = self.levels[fine], self.levels[fine - 1]
        cov = coarsen_mask(F.valid)
        if self.tee_on:
            if self.tee_fields:
                T = tee_coarse_fields(C.U, F.U)
                F.tee = np.stack([np.where(F.valid, refine_values(T[c]), 0.0) for c in range(4)])
            else:
                T = tee_coarse(C.U, F.U)
                F.tee = np.where(F.valid, refine_values(T), 0.0)
        for c in range(4):
            with np.errstate(all="ignore"):
                avg = average_down_arrays(F.U[c])
            C.U[c][cov] = avg[cov].astype(self.dtype)

    # ---- diagnostics -------------------------------------------------------------
    def set_tee(self, enable: bool, te_crit: float = 0.0, tag_mode: int = 1):
        self.tee_on, self.te_crit, self.tag_mode = bool(enable), float(te_crit), int(tag_mode)
        self._reset_tee(False)

    def set_tee_fields(self, enable: bool, te_crit, scale=(1.0, 1.0, 1.0, 1.0), tag_mode: int = 3):
        """Per-field estimates: tag where scale_c * Delta_c > te_crit_c for some c."""
        self.tee_on, self.tag_mode = bool(enable), int(tag_mode)
        self.te_crit_c = np.asarray(te_crit, dtype=np.float64).reshape(4).copy()
        self.te_scale = np.asarray(scale, dtype=np.float64).reshape(4).copy()
        self._reset_tee(True)

    def set_tee_scale(self, scale):
        """New modifier scales; the estimates already formed are kept."""
        self.te_scale = np.asarray(scale, dtype=np.float64).reshape(4).copy()

    def _tee_zeros(self, M: int) -> np.ndarray:
        return np.zeros((4, M, M, M) if self.tee_fields else (M, M, M))

    def _reset_tee(self, fields: bool):
        """Switching between one estimate per cell and one per component starts the
        estimates again from 0."""
        if fields != self.tee_fields:
            self.tee_fields = fields
            for L in self.levels:
                L.tee = self._tee_zeros(L.M)

    def field_absmax(self) -> np.ndarray:
        """max |U_c| over the valid cells of every level, per component (float64); NaN
        if any of those values is NaN."""
        out = np.zeros(4)
        for c in range(4):
            vals = [np.abs(L.U[c][L.valid].astype(np.float64)) for L in self.levels]
            out[c] = np.max(np.concatenate([v.ravel() for v in vals] + [np.zeros(1)]))
        return out

    def tags(self, lev: int) -> np.ndarray:
        L = self.levels[lev]
        t = np.zeros((L.M,) * 3, dtype=bool)
        if self.tag_mode & 1:
            t |= tag_cells(L.U[0], L.U[1]).astype(bool)
        if self.tag_mode & 2:
            if self.tee_fields:
                for c in range(4):
                    t |= (self.te_scale[c] * L.tee[c]) > self.te_crit_c[c]
            else:
                t |= L.tee > self.te_crit
        return (t & L.valid).astype(np.uint8)

    # ---- shadow level (truncation error estimate of level 0) --------------------
    def shadow_begin(self):
        L0 = self.levels[0]
        if L0.k % 2:
            raise ValueError("the shadow starts when level 0 has taken an even number of steps")
        dx = level_dx(self.L, self.n0, 0) * 2.0
        S = Level(self.n0 // 2, dx, self.cfl * dx)
        S.k = L0.k // 2
        S.k_start = S.k
        S.valid[:] = True
        S.U = np.stack([average_down_arrays(L0.U[c]) for c in range(4)]).astype(self.dtype)
        self.shadow = S

    def shadow_advance(self):
        S = self.shadow
        if S.k != S.k_start:
            raise ValueError("the shadow takes a single step")
        eta_n = level_time(self.eta0, S.k, S.dt)
        X, acc = S.U, None
        ko = self._ko(S.dx)
        with np.errstate(all="ignore"):
            for s in range(len(self.cs)):
                if self.integrator == 4:
                    acc, X = rk4_stage(s, X, S.U, acc, eta_n, S.dt, 1.0 / (S.dx * S.dx), self.alpha, self.lam,
                                       self.beta, self.order, ko)
                elif self.integrator == 21:
                    acc, X = rkn4_stage(s, X, S.U, acc, eta_n, S.dt, 1.0 / (S.dx * S.dx), self.lam, self.beta,
                                        self.order)
                else:
                    X = ssprk3_stage(s, X, S.U, eta_n, S.dt, 1.0 / (S.dx * S.dx), self.alpha, self.lam, self.beta,
                                     self.order, ko)
        S.U = X
        S.k += 1

    def shadow_end(self):
        S, L0 = self.shadow, self.levels[0]
        if S.k != S.k_start + 1 or L0.k != 2 * S.k:
            raise ValueError("level 0 and the shadow are not at the same time after one shadow step")
        if self.tee_fields:
            T = tee_coarse_fields(S.U, L0.U)
            L0.tee = np.stack([refine_values(T[c]) for c in range(4)])
        else:
            L0.tee = refine_values(tee_coarse(S.U, L0.U))
        self.shadow = None

    def covered(self, lev: int) -> np.ndarray:
        """Cells of level lev under a finer level."""
        if lev >= self.finest:
            return np.zeros((self.levels[lev].M,) * 3, dtype=bool)
        return coarsen_mask(self.levels[lev + 1].valid)

    def energy(self):
        """Composite [kin, grad, pot, total] over cells not covered by a finer level."""
        tot = np.zeros(4)
        for lev, L in enumerate(self.levels):
            cp = self.lam * int_power(self.time(lev), self.beta)
            mask = L.valid & ~self.covered(lev)
            with np.errstate(all="ignore"):
                tot += np.array(_energy(L.U, L.dx, cp, mask))
        return tot.tolist()
