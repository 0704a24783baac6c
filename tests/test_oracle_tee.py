"""Pins of the oracle's truncation error estimates (self-shadow and shadow level):
closed forms for a uniform field and for a free plane wave, the tag-mode logic and the
regrid rule for kept cells."""
import numpy as np
import pytest

from oracle.amr import Hierarchy, average_down_arrays, boxes_mask, normalising_scales, refine_values
from oracle.tagging import tag_cells
from synth import random_state


def _full_cover_boxes(M, b=8):
    return [(x, y, z, x + b - 1, y + b - 1, z + b - 1)
            for z in range(0, M, b) for y in range(0, M, b) for x in range(0, M, b)]


def _textbook_rk4(y0, eta0, dt, nsteps, alpha, lam, beta):
    """Uniform field, Butcher form y + h/6 (k1 + 2k2 + 2k3 + k4), independent of the oracle."""
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


def test_uniform_field_tee_is_the_one_step_vs_two_half_steps_difference():
    n0, eta0 = 4, 0.5
    y0 = (0.3, -0.2, 0.1, 0.05)
    h = Hierarchy(n0, float(n0), 0.25, eta0, 1, alpha=2.0, lam=1.0, beta=2)
    h.set_level0(np.stack([np.full((n0,) * 3, v) for v in y0]))
    h.set_layout(1, _full_cover_boxes(2 * n0, 4))
    h.set_tee(True)
    h.coarse_step()
    coarse = _textbook_rk4(y0, eta0, 0.25, 1, 2.0, 1.0, 2)
    fine = _textbook_rk4(y0, eta0, 0.125, 2, 2.0, 1.0, 2)
    ref = np.max(np.abs(coarse - fine))
    tee = h.levels[1].tee
    assert np.all(tee == tee.flat[0])
    assert ref > 1e-9                                 # a real difference, not rounding
    assert abs(tee.flat[0] - ref) < 1e-14


def _step_matrix(omega2, h):
    """Classic RK4 step matrix of y' = A y, A = [[0, 1], [-omega^2, 0]]."""
    A = np.array([[0.0, 1.0], [-omega2, 0.0]]) * h
    A2 = A @ A
    return np.eye(2) + A + A2 / 2 + A2 @ A / 6 + A2 @ A2 / 24


def _omega2(k, d):
    return (4.0 / d**2) * np.sum(np.sin(k * d / 2) ** 2)


def _centred_cos(M, L, k, amp):
    x = (np.arange(M) + 0.5) * (L / M)
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    return amp * np.cos(k[0] * xx + k[1] * y + k[2] * z)


def test_free_plane_wave_tee_closed_form():
    n0, L, amp = 16, 16.0, 0.7
    k = 2 * np.pi / L * np.array([2.0, 1.0, 1.0])
    dx0, dt0 = L / n0, 0.25
    zero = np.zeros((n0,) * 3)
    h = Hierarchy(n0, L, 0.25, 0.1, 1, alpha=0.0, lam=0.0, beta=0)
    h.set_level0(np.stack([_centred_cos(n0, L, k, amp), zero, zero, zero]))
    h.set_layout(1, _full_cover_boxes(2 * n0))
    # both levels start from the exact cosine at their own cell centres
    h.levels[1].U[:] = 0.0
    h.levels[1].U[0] = _centred_cos(2 * n0, L, k, amp)
    h.set_tee(True)
    h.coarse_step()
    Mc = _step_matrix(_omega2(k, dx0), dt0)
    Mf = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0 / 2), dt0 / 2), 2)
    P = np.prod(np.cos(k * dx0 / 4))                  # mean of cos over the 8 children
    coef = max(abs(Mc[0, 0] - P * Mf[0, 0]), abs(Mc[1, 0] - P * Mf[1, 0]))
    ref = coef * np.abs(_centred_cos(n0, L, k, 1.0)) * amp
    got = average_down_arrays(h.levels[1].tee)        # children carry their parent's value
    assert coef > 1e-6
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.array_equal(h.levels[1].tee[::2, ::2, ::2], got)


def test_shadow_level_tee_closed_form_and_timing_checks():
    n0, L, amp = 16, 16.0, 0.4
    k = 2 * np.pi / L * np.array([1.0, 2.0, 0.0])
    dx0, dt0 = L / n0, 0.25
    zero = np.zeros((n0,) * 3)
    h = Hierarchy(n0, L, 0.25, 0.1, 0, alpha=0.0, lam=0.0, beta=0)
    h.set_level0(np.stack([zero, _centred_cos(n0, L, k, amp), zero, zero]))
    h.set_tee(True)
    h.shadow_begin()
    with pytest.raises(ValueError):
        h.shadow_end()                                # level 0 has not moved yet
    h.shadow_advance()
    h.coarse_step()
    with pytest.raises(ValueError):
        h.shadow_end()                                # one level-0 step is not enough
    h.coarse_step()
    h.shadow_end()
    Ms = _step_matrix(_omega2(k, 2 * dx0), 2 * dt0)
    M0 = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0), dt0), 2)
    P = np.prod(np.cos(k * dx0 / 2))                  # the shadow starts from the 2^3 means
    coef = P * max(abs(Ms[0, 0] - M0[0, 0]), abs(Ms[1, 0] - M0[1, 0]))
    ref = coef * np.abs(_centred_cos(n0 // 2, L, k, 1.0)) * amp
    got = h.levels[0].tee[::2, ::2, ::2]
    assert coef > 1e-6
    assert np.max(np.abs(got - ref)) < 1e-12
    h.coarse_step()
    with pytest.raises(ValueError):
        h.shadow_begin()                              # odd number of level-0 steps


def test_tag_modes_and_regrid_rule():
    n0 = 8
    U = random_state(n0, float(n0), 5)
    h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, beta=0)
    h.set_level0(U)
    old = [(0, 0, 0, 7, 7, 7), (8, 0, 0, 15, 7, 7)]
    h.set_layout(1, old)
    h.set_tee(True, te_crit=1e-4, tag_mode=2)
    h.coarse_step()
    L1 = h.levels[1]
    assert np.all(L1.tee[~L1.valid] == 0) and np.any(L1.tee[L1.valid] > 0)
    plaq = tag_cells(L1.U[0], L1.U[1]).astype(bool) & L1.valid
    tee = (L1.tee > 1e-4) & L1.valid
    for mode, want in ((1, plaq), (2, tee), (3, plaq | tee)):
        h.tag_mode = mode
        assert np.array_equal(h.tags(1).astype(bool), want)
    # regrid: kept cells keep their estimate, new cells start at 0
    before = L1.tee.copy()
    new = [(4, 0, 0, 11, 7, 7)]
    h.set_layout(1, new)
    nv = boxes_mask(new, 16)
    kept = nv & boxes_mask(old, 16)
    assert np.array_equal(h.levels[1].tee[kept], before[kept])
    assert np.all(h.levels[1].tee[nv & ~kept] == 0)


# ---- per-field estimates and the modifier of section IV.C ------------------------------

def _plane_wave_two_levels(amp=0.7, kk=(2.0, 1.0, 1.0)):
    n0, L = 16, 16.0
    k = 2 * np.pi / L * np.array(kk)
    zero = np.zeros((n0,) * 3)
    h = Hierarchy(n0, L, 0.25, 0.1, 1, alpha=0.0, lam=0.0, beta=0)
    h.set_level0(np.stack([_centred_cos(n0, L, k, amp), zero, zero, zero]))
    h.set_layout(1, _full_cover_boxes(2 * n0))
    h.levels[1].U[:] = 0.0
    h.levels[1].U[0] = _centred_cos(2 * n0, L, k, amp)
    return h, k, n0, L


def test_per_field_plane_wave_estimates_and_maxima_closed_form():
    amp = 0.7
    h, k, n0, L = _plane_wave_two_levels(amp)
    dx0, dt0 = L / n0, 0.25
    h.set_tee_fields(True, te_crit=[1.0] * 4)
    h.coarse_step()
    Mc = _step_matrix(_omega2(k, dx0), dt0)
    Mf = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0 / 2), dt0 / 2), 2)
    P = np.prod(np.cos(k * dx0 / 4))
    cosc = np.abs(_centred_cos(n0, L, k, 1.0))
    tee = h.levels[1].tee
    assert tee.shape == (4, 2 * n0, 2 * n0, 2 * n0)
    # psi1 and Pi1 carry the standing wave; psi2 and Pi2 stay 0
    for c, row in ((0, 0), (2, 1)):
        ref = abs(Mc[row, 0] - P * Mf[row, 0]) * amp * cosc
        got = average_down_arrays(tee[c])
        assert np.max(ref) > 1e-6
        assert np.max(np.abs(got - ref)) < 1e-12
    assert not tee[1].any() and not tee[3].any()
    # the max-over-components estimate of the same run is their pointwise maximum
    assert np.array_equal(np.maximum(tee[0], tee[2]), np.max(tee, axis=0))
    # maxima over both levels: the fine level holds the wave after two fine steps, level 0
    # its 2^3 means
    fine_cos = np.max(np.abs(_centred_cos(2 * n0, L, k, 1.0)))
    want = [max(abs(Mf[r, 0]) * fine_cos, abs(P * Mf[r, 0]) * np.max(cosc)) * amp for r in (0, 1)]
    m = h.field_absmax()
    assert abs(m[0] - want[0]) < 1e-12 and abs(m[2] - want[1]) < 1e-12
    assert m[1] == 0.0 and m[3] == 0.0
    s = normalising_scales(m)
    assert s[1] == 1.0 and s[3] == 1.0 and abs(s[0] * want[0] - 1.0) < 1e-12


def _nudge(vals, frac):
    """A threshold near frac * max(vals) that no value lies within 1e-9 (relative) of."""
    top = float(np.max(vals))
    eps = frac * top
    while np.min(np.abs(vals - eps)) < 1e-9 * top:
        eps *= 1.0 + 1e-6
    return eps


@pytest.mark.parametrize("which", [0, 2])
def test_per_field_thresholds_tag_each_component_on_its_own(which):
    amp = 0.7
    h, k, n0, L = _plane_wave_two_levels(amp)
    dx0, dt0 = L / n0, 0.25
    h.set_tee_fields(True, te_crit=[1e30] * 4)
    h.coarse_step()
    s = normalising_scales(h.field_absmax())
    h.set_tee_scale(s)
    Mc = _step_matrix(_omega2(k, dx0), dt0)
    Mf = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0 / 2), dt0 / 2), 2)
    P = np.prod(np.cos(k * dx0 / 4))
    row = 0 if which == 0 else 1
    ref = refine_values(abs(Mc[row, 0] - P * Mf[row, 0]) * amp * np.abs(_centred_cos(n0, L, k, 1.0)))
    f = s[which] * ref                                  # f_c(Delta_c) from the closed form
    crit = [1e30] * 4
    crit[which] = _nudge(f, 0.6)
    h.te_crit_c = np.array(crit)
    want = f > crit[which]
    assert 0 < want.sum() < want.size
    assert np.array_equal(h.tags(1).astype(bool), want)
    # modifier scales matter: unscaled, the same threshold tags a different set
    h.set_tee_scale(np.ones(4))
    assert not np.array_equal(h.tags(1).astype(bool), want)


def test_per_field_with_one_threshold_and_unit_scales_equals_the_max_estimate():
    n0 = 8
    U = random_state(n0, float(n0), 6)
    runs = []
    for fields in (False, True):
        h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, beta=0)
        h.set_level0(U)
        h.set_layout(1, [(0, 0, 0, 7, 7, 7), (8, 0, 0, 15, 7, 7), (0, 8, 8, 7, 15, 15)])
        if fields:
            h.set_tee_fields(True, te_crit=[2e-5] * 4, tag_mode=2)
        else:
            h.set_tee(True, te_crit=2e-5, tag_mode=2)
        h.coarse_step()
        runs.append(h)
    a, b = runs
    assert np.array_equal(np.max(b.levels[1].tee, axis=0), a.levels[1].tee)
    crit = _nudge(a.levels[1].tee[a.levels[1].valid], 0.5)
    a.te_crit = crit
    b.te_crit_c = np.full(4, crit)
    ta, tb = a.tags(1), b.tags(1)
    assert 0 < ta.sum() < a.levels[1].valid.sum()
    assert np.array_equal(ta, tb)


def test_per_field_regrid_keeps_every_component_of_kept_cells():
    n0 = 8
    h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, beta=0)
    h.set_level0(random_state(n0, float(n0), 7))
    old = [(0, 0, 0, 7, 7, 7), (8, 0, 0, 15, 7, 7)]
    h.set_layout(1, old)
    h.set_tee_fields(True, te_crit=[1e-4] * 4)
    h.coarse_step()
    before = h.levels[1].tee.copy()
    assert before.shape[0] == 4 and np.all(before[:, ~h.levels[1].valid] == 0)
    new = [(4, 0, 0, 11, 7, 7)]
    h.set_layout(1, new)
    nv = boxes_mask(new, 16)
    kept = nv & boxes_mask(old, 16)
    assert np.array_equal(h.levels[1].tee[:, kept], before[:, kept])
    assert np.all(h.levels[1].tee[:, nv & ~kept] == 0)


def test_per_field_shadow_level_closed_form():
    n0, L, amp = 16, 16.0, 0.4
    k = 2 * np.pi / L * np.array([1.0, 2.0, 0.0])
    dx0, dt0 = L / n0, 0.25
    zero = np.zeros((n0,) * 3)
    h = Hierarchy(n0, L, 0.25, 0.1, 0, alpha=0.0, lam=0.0, beta=0)
    h.set_level0(np.stack([zero, _centred_cos(n0, L, k, amp), zero, zero]))
    h.set_tee_fields(True, te_crit=[1.0] * 4)
    h.shadow_begin()
    h.shadow_advance()
    h.coarse_step()
    h.coarse_step()
    h.shadow_end()
    Ms = _step_matrix(_omega2(k, 2 * dx0), 2 * dt0)
    M0 = np.linalg.matrix_power(_step_matrix(_omega2(k, dx0), dt0), 2)
    P = np.prod(np.cos(k * dx0 / 2))
    tee = h.levels[0].tee
    for c, row in ((1, 0), (3, 1)):
        ref = P * abs(Ms[row, 0] - M0[row, 0]) * np.abs(_centred_cos(n0 // 2, L, k, 1.0)) * amp
        assert np.max(np.abs(tee[c][::2, ::2, ::2] - ref)) < 1e-12
    assert not tee[0].any() and not tee[2].any()


def test_field_maxima_take_every_level_and_propagate_nan():
    n0 = 8
    U = random_state(n0, float(n0), 9)
    h = Hierarchy(n0, float(n0), 0.25, 0.1, 1, beta=0)
    h.set_level0(U)
    h.set_layout(1, [(4, 4, 4, 11, 11, 11)])
    h.levels[1].U[2][5, 6, 7] = 40.0                    # a fine value larger than any on level 0
    m = h.field_absmax()
    assert m[2] == 40.0
    assert m[0] == max(np.max(np.abs(U[0])), np.max(np.abs(h.levels[1].U[0][h.levels[1].valid])))
    h.levels[0].U[1][1, 2, 3] = np.nan
    m = h.field_absmax()
    assert np.isnan(m[1]) and not np.isnan(m[0]) and not np.isnan(m[3])

