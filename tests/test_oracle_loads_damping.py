"""Pins of the oracle parts that the GPU tests of damping, start-up and load shapes rest on.

* the damped central-difference update (eq. DnMdiag with C = alpha M, eq. C) against the
  discrete energy balance that follows from it;
* the start-up point of eq. D0 (initial velocity) against the closed-form discrete motion of
  a free rigid translation, undamped and damped;
* the triangular pulse (eq. Triangle) against its amplitude spectrum (eq. Triangle_A);
* the Hann-windowed sine burst (eq. Lamb) against its closed-form spectrum, its centre
  frequency f_m = n / t1 and the 85 % critical frequency the paper quotes (Sec. 5).

Each check is a function of the oracle routine it pins, and every test also runs it on a
copy of that routine with a plausible mistake planted (a flipped damping sign, a flipped
velocity term, a wrong pulse width, a window without its square, a wrong cycle count) and
requires the check to fail there.
"""

import copy

import numpy as np
import pytest

from meshgen import configs
from oracle import loads
from oracle.solver import Oracle


# --------------------------------------------------------------------------------------------
# damped update: H_{n+1/2} - H_{n-1/2} + alpha/(4 dt) |u_{n+1} - u_{n-1}|_M^2 = 1/2 (u_{n+1} - u_{n-1})^T f_ext,n
#
# Multiply eq. DnMdiag, written as M (u_{n+1} - 2u_n + u_{n-1})/dt^2 + alpha M (u_{n+1} - u_{n-1})/(2 dt)
# + K u_n = f_ext,n, by (u_{n+1} - u_{n-1})^T and use the symmetry of M and K, with
# H_{n+1/2} = 1/2 [ |u_{n+1} - u_n|_M^2 / dt^2 + u_{n+1}^T K u_n ].


def _damped_balance(o, step, dt, alpha, n_steps):
    """max_n |cumulative balance defect| / max_n |H_{n+1/2}| along a run of `step`."""
    M = o.mdiag
    u, um1 = o.initial_state(dt)
    d = u - um1
    H0 = 0.5 * (d @ (M * d)) / dt ** 2 + 0.5 * (u @ o.internal_force(um1))
    Hs, acc, worst = [H0], 0.0, 0.0
    H_prev = H0
    for n in range(n_steps):
        unew, f = step(o, u, um1, n, dt, alpha)
        d = unew - u
        H = 0.5 * (d @ (M * d)) / dt ** 2 + 0.5 * (unew @ f)
        w = unew - um1
        acc += (H - H_prev) + alpha / (4 * dt) * (w @ (M * w)) - 0.5 * (w @ (o.load_at(n * dt) * o.b))
        worst = max(worst, abs(acc))
        Hs.append(H)
        H_prev = H
        um1, u = u, unew
    return worst / np.abs(Hs).max(), np.abs(Hs).max()


def _oracle_step(o, u, um1, n, dt, alpha):
    return o.step(u, um1, n, dt, alpha)


def _step_flipped_damping(o, u, um1, n, dt, alpha):
    """Planted mistake: c = -alpha dt / 2."""
    f = o.internal_force(u)
    r = o.load_at(n * dt) * o.b - f
    c = -0.5 * alpha * dt
    return (dt * dt * o.minv * r + 2.0 * u - (1.0 - c) * um1) / (1.0 + c), f


def _step_undamped_denominator(o, u, um1, n, dt, alpha):
    """Planted mistake: the division by 1 + alpha dt / 2 left out."""
    f = o.internal_force(u)
    r = o.load_at(n * dt) * o.b - f
    c = 0.5 * alpha * dt
    return dt * dt * o.minv * r + 2.0 * u - (1.0 - c) * um1, f


@pytest.fixture(scope="module")
def damped_cube():
    m = configs.cfg1()
    m.load = dict(m.load, alpha=1.5)
    o = Oracle(m)
    return o, 0.5 * o.critical_dt()


def test_damped_energy_balance(damped_cube):
    o, dt = damped_cube
    alpha = 1.5
    defect, hmax = _damped_balance(o, _oracle_step, dt, alpha, 400)
    assert hmax > 0
    assert defect < 1e-12, defect
    # the damping removes energy: without it the same run keeps more
    for wrong in (_step_flipped_damping, _step_undamped_denominator):
        bad, _ = _damped_balance(o, wrong, dt, alpha, 400)
        assert bad > 1e-4, (wrong.__name__, bad)


def test_damped_run_matches_step_loop(damped_cube):
    """Oracle.run takes alpha from the load parameters and applies eq. DnMdiag with it."""
    o, dt = damped_cube
    r = o.run(n_steps=60, dt=dt, snap_every=0, energy=False)
    u, um1 = o.initial_state(dt)
    for n in range(60):
        unew, _ = o.step(u, um1, n, dt, 1.5)
        um1, u = u, unew
    assert np.array_equal(r["u"], u)


# --------------------------------------------------------------------------------------------
# start-up with an initial velocity (eq. D0): a free body in rigid translation, no load.
# K annihilates translations, so eq. DnMdiag reduces to u_{n+1} = (2 u_n - (1 - c) u_{n-1})/(1 + c)
# with c = alpha dt / 2; the acceleration at rest of eq. D0 is -alpha v0.  With u_0 = 0 the
# recurrence has roots 1 and r = (1 - c)/(1 + c), and u_{-1} = -dt v0 (1 + c) gives
#   u_n = dt v0 (1 - c^2)/(2c) (1 - r^n)   (-> n dt v0 as alpha -> 0).


def _free_cube(alpha):
    m = configs.cfg1()
    m = copy.copy(m)
    m.fixed = np.zeros_like(m.fixed)
    m.load_dof = np.zeros(0, np.int64)
    m.load_val = np.zeros(0)
    m.load = dict(m.load, alpha=alpha)
    return m


def _translation_error(o, dt, alpha, v, n_steps, init):
    v0 = np.tile(v, o.n_dof // 3)
    u, um1 = init(o, dt, v0)
    c = 0.5 * alpha * dt
    worst = 0.0
    for n in range(n_steps):
        u_new, _ = o.step(u, um1, n, dt, alpha)
        um1, u = u, u_new
        k = n + 1
        if c == 0.0:
            want = k * dt * v0
        else:
            r = (1.0 - c) / (1.0 + c)
            want = dt * v0 * (1.0 - c * c) / (2.0 * c) * (1.0 - r ** k)
        worst = max(worst, float(np.abs(u - want).max()))
    return worst / (n_steps * dt * np.abs(v).max())


def _oracle_init(o, dt, v0):
    return o.initial_state(dt, v0=v0)


def _init_flipped_velocity(o, dt, v0):
    """Planted mistake: u_{-1} = u_0 + dt v0 + ..."""
    u0, um1 = o.initial_state(dt, v0=v0)
    return u0, um1 + 2 * dt * v0


def _init_no_damping_accel(o, dt, v0):
    """Planted mistake: the start-up acceleration -alpha v0 left out."""
    return np.zeros(o.n_dof), -dt * v0


@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_rigid_translation_from_initial_velocity(alpha):
    m = _free_cube(alpha)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    v = np.array([0.3, -1.1, 0.7])
    err = _translation_error(o, dt, alpha, v, 200, _oracle_init)
    assert err < 1e-11, err  # K u of a translation is zero up to rounding, which the recursion carries
    wrongs = [_init_flipped_velocity] + ([_init_no_damping_accel] if alpha > 0 else [])
    for wrong in wrongs:
        assert _translation_error(o, dt, alpha, v, 200, wrong) > 1e-6, wrong.__name__


def test_rigid_translation_with_initial_displacement():
    """A rigid initial displacement is carried along unchanged (K u_0 = 0 in eq. D0)."""
    m = _free_cube(0.0)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    a = np.tile([1e-3, 2e-3, -5e-4], o.n_dof // 3)
    v0 = np.tile([0.2, 0.0, -0.4], o.n_dof // 3)
    u, um1 = o.initial_state(dt, u0=a, v0=v0)
    for n in range(100):
        u_new, _ = o.step(u, um1, n, dt)
        um1, u = u, u_new
    assert np.abs(u - (a + 100 * dt * v0)).max() < 1e-11 * (100 * dt * 0.4)


# --------------------------------------------------------------------------------------------
# load-time functions against their spectra (Sec. 5)


def _amplitude(fn, t1, span=200.0, per=4000):
    dt = t1 / per
    t = np.arange(0.0, span * t1, dt)
    A = np.abs(np.fft.rfft(fn(t))) * dt
    return np.fft.rfftfreq(len(t), dt), A


def _triangle_spectrum_defect(fn, t1):
    """max |A(f) - t1 sinc^2(f t1)| / t1 over the computed band (eq. Triangle_A times t1, the
    pulse's area)."""
    f, A = _amplitude(fn, t1)
    return float(np.abs(A - t1 * np.sinc(f * t1) ** 2).max() / t1)


@pytest.mark.parametrize("t1", [1.0, 0.37])
def test_triangle_pulse_spectrum(t1):
    assert loads.triangle(t1, t1) == 1.0 and loads.triangle(0.0, t1) == 0.0 and loads.triangle(2 * t1, t1) == 0.0
    assert _triangle_spectrum_defect(lambda t: loads.triangle(t, t1), t1) < 1e-6
    # planted mistakes: half the pulse width, a peak at t1 / 2
    half = lambda t: np.where((t >= 0) & (t <= t1), 1.0 - np.abs(2 * t / t1 - 1.0), 0.0)
    early = lambda t: np.where((t >= 0) & (t <= 2 * t1), np.clip(1.0 - np.abs(t / t1 - 0.5), 0, None), 0.0)
    for wrong in (half, early):
        assert _triangle_spectrum_defect(wrong, t1) > 1e-2


def _burst_closed_form(f, t1, n):
    """|F[P](f)| of eq. Lamb (P0 = 1): sin(2 pi n t/t1) sin^2(pi t/t1) is
    1/2 sin(2 pi n t/t1) - 1/4 sin(2 pi (n+1) t/t1) - 1/4 sin(2 pi (n-1) t/t1) on [0, t1], and
    a whole number k of cycles of sin(a t), a = 2 pi k / t1, transforms to a (1 - e^{-i w t1})/(a^2 - w^2)."""
    w = 2 * np.pi * f
    s = np.zeros_like(f)
    for k, c in ((n, 0.5), (n + 1, -0.25), (n - 1, -0.25)):
        a = 2 * np.pi * k / t1
        s = s + c * a / (a * a - w * w)
    return np.abs(2 * np.sin(np.pi * f * t1)) * np.abs(s)


def _burst_spectrum_defect(fn, t1, n):
    f, A = _amplitude(fn, t1)
    keep = np.ones_like(f, dtype=bool)
    for k in (n - 1, n, n + 1):  # removable singularities of the closed form
        keep &= np.abs(f * t1 - k) > 1e-3
    want = _burst_closed_form(f[keep], t1, n)
    return float(np.abs(A[keep] - want).max() / want.max())


@pytest.mark.parametrize("n", [5, 3])
def test_sine_burst_spectrum(n):
    t1 = 1.0
    assert _burst_spectrum_defect(lambda t: loads.sine_burst(t, t1, n), t1, n) < 1e-5
    no_square = lambda t: np.where((t >= 0) & (t <= t1), np.sin(2 * np.pi * n * t / t1) * np.sin(np.pi * t / t1), 0.0)
    wrong_n = lambda t: loads.sine_burst(t, t1, n + 1)
    for wrong in (no_square, wrong_n):
        assert _burst_spectrum_defect(wrong, t1, n) > 1e-2


def test_sine_burst_centre_and_critical_frequency():
    """Sec. 5: f_m = n / t1 and, for n = 5, 85 % of the spectral area lies below f1 = 5.8 / t1."""
    for n in (3, 5, 8):
        f, A = _amplitude(lambda t: loads.sine_burst(t, 0.5, n), 0.5)
        assert abs(f[np.argmax(A)] - n / 0.5) <= f[1]
    t1 = 0.8
    f, A = _amplitude(lambda t: loads.sine_burst(t, t1, 5), t1)
    cum = np.cumsum(A)
    f1 = f[np.searchsorted(cum, 0.85 * cum[-1])]
    assert abs(f1 * t1 - 5.8) < 0.06, f1 * t1
    assert loads.sine_burst(np.array([-0.1, 0.0, t1, 1.1 * t1]), t1, 5).tolist() == [0.0, 0.0, pytest.approx(0.0, abs=1e-15), 0.0]
