"""Probe time histories of the oracle (displacement at a point, Sec. 5.2; acceleration
history, Sec. 5.3), pinned by the balance of momentum of a free body.

For a body with no fixed dof, summing the equation of motion M a + alpha M v + K u = P(t) b
(eq. DnMdiag with the lumped mass) over all dofs of one axis removes the internal force, since
K annihilates rigid translations and is symmetric: 1_x^T K u = (K 1_x)^T u = 0.  With the
central differences a_n = (u_{n+1} - 2 u_n + u_{n-1}) / dt^2 and v_n = (u_{n+1} - u_{n-1}) / (2 dt)
of the recorded histories,

    sum_i m_i (a_n,i + alpha v_n,i) = P(t_n) sum_i b_i      (i over the dofs of one axis)

holds at every step up to rounding.  An acceleration taken at t_{n+1}, a one-sided difference,
a flipped sign or a missing dt would break it.
"""

import copy

import numpy as np
import pytest

from meshgen import configs
from oracle.solver import Oracle


def _free(m, alpha):
    m = copy.copy(m)
    m.fixed = np.zeros_like(m.fixed)
    m.load = dict(m.load, alpha=alpha)
    return m


def _momentum_residual(o, run, probes, alpha, dt):
    """max over steps and axes of |sum m (a + alpha v) - P(t_n) sum b|, relative."""
    pu, pa = run["probe_u"], run["probe_a"]
    n_steps = pu.shape[0]
    # central velocity at step n from u_{n+1} (row n of probe_u) and u_{n-1}
    before = np.vstack([run["um1_start"][None, probes], run["u_start"][None, probes], pu[:-2]])
    v = (pu - before) / (2.0 * dt)
    m = o.mdiag[probes]
    worst = 0.0
    for axis in range(3):
        sel = probes % 3 == axis
        lhs = (m[sel] * (pa[:, sel] + alpha * v[:, sel])).sum(axis=1)
        rhs = np.array([o.load_at(n * dt) for n in range(n_steps)]) * o.b[probes[sel]].sum()
        scale = max(np.abs(o.b).sum() * np.abs([o.load_at(n * dt) for n in range(n_steps)]).max(), 1e-300)
        worst = max(worst, float(np.abs(lhs - rhs).max() / scale))
    return worst


def _run(mesh, alpha, n_steps, probes):
    o = Oracle(mesh)
    dt = 0.5 * o.critical_dt()
    u0, um1 = o.initial_state(dt)
    run = o.run(n_steps=n_steps, dt=dt, snap_every=1, energy=False, probes=probes)
    run["u_start"], run["um1_start"] = u0, um1
    return o, run, dt


@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_probe_momentum_balance_free_body(alpha):
    m = _free(configs.cfg1(), alpha)
    probes = np.arange(m.n_dof)
    o, run, dt = _run(m, alpha, 120, probes)
    assert run["probe_u"].shape == (120, m.n_dof)
    res = _momentum_residual(o, run, probes, alpha, dt)
    assert res < 1e-9, res
    # planted mistakes in the recorded history, each caught by the balance
    wrong = dict(run)
    wrong["probe_a"] = np.vstack([run["probe_a"][1:], run["probe_a"][-1:]])  # a at t_{n+1}
    assert _momentum_residual(o, wrong, probes, alpha, dt) > 1e-4
    wrong = dict(run)
    wrong["probe_a"] = -run["probe_a"]
    assert _momentum_residual(o, wrong, probes, alpha, dt) > 1e-4


def test_probe_momentum_balance_with_hanging_nodes():
    """The same balance on a mesh with hanging nodes (the small refined-zoo mesh)."""
    m = _free(configs.small_zoo(), 0.0)
    probes = np.arange(m.n_dof)
    o, run, dt = _run(m, 0.0, 40, probes)
    assert _momentum_residual(o, run, probes, 0.0, dt) < 1e-9


def test_probe_rows_are_the_snapshots():
    """Row k of probe_u is u_{k+1} at the probe dofs, in the caller's order (repeats allowed)."""
    m = configs.cfg1()
    rng = np.random.default_rng(3)
    probes = rng.integers(0, m.n_dof, 17)
    probes[5] = probes[2]
    o, run, dt = _run(m, 0.0, 30, probes)
    for k in range(30):
        assert np.array_equal(run["probe_u"][k], run["snapshots"][k + 1][probes])
    # u_1 - 2 u_0 + u_{-1} at step 0
    a0 = (run["snapshots"][1] - 2 * run["u_start"] + run["um1_start"])[probes] / dt ** 2
    assert np.array_equal(run["probe_a"][0], a0)
