"""Load given per step (P(t_n) from a table, R_ext at t_n = n dt in Alg. 1): the oracle's table
kind is pinned by reduction to the Ricker wavelet (its samples as a table reproduce the Ricker
run exactly) and by the discrete work of a table shorter than the run (no external work once
the table has ended; the energy identity of eq. DnMdiag still holds)."""

import copy

import numpy as np

from meshgen import configs
from oracle import loads
from oracle.solver import Oracle, energy_drift


def _cfg1(n_steps):
    m = configs.cfg1(n_steps=n_steps)
    o = Oracle(m)
    dt = m.load["dt_factor"] * o.critical_dt()
    return m, o, dt


def test_table_of_ricker_samples_reproduces_ricker_run():
    m, o, dt = _cfg1(200)
    ref = o.run(n_steps=200, dt=dt, snap_every=50, energy=False)
    P = loads.ricker(np.arange(200) * dt, m.load["t1"], m.load.get("P0", 1.0))
    mt = copy.copy(m)
    mt.load = dict(kind="table", P=P, dt=dt, dt_factor=m.load["dt_factor"], n_steps=200)
    got = Oracle(mt).run(n_steps=200, dt=dt, snap_every=50, energy=False)
    for k in ref["snapshots"]:
        assert np.array_equal(got["snapshots"][k], ref["snapshots"][k])


def test_short_table_does_no_work_after_its_end():
    m, o, dt = _cfg1(300)
    rng = np.random.default_rng(17)
    P = rng.normal(size=120)
    mt = copy.copy(m)
    mt.load = dict(kind="table", P=P, dt=dt, dt_factor=m.load["dt_factor"], n_steps=300)
    run = Oracle(mt).run(n_steps=300, dt=dt, snap_every=0, energy=True)
    W = run["W"]
    # W[n + 1] - W[n] is the work of step n, with P(t_n): zero from step 120 on, not before
    assert np.abs(np.diff(W)[120:]).max() == 0.0
    assert np.abs(np.diff(W)[:120]).max() > 0.0
    assert energy_drift(run["H"], W) < 1e-12


def test_table_index_rounds_to_the_step():
    P = np.arange(1.0, 11.0)
    dt = 0.37
    n = np.arange(-2, 13)
    for eps in (0.0, 1e-12, -1e-12):
        t = n * dt * (1 + eps)
        want = np.where((n >= 0) & (n < 10), P[np.clip(n, 0, 9)], 0.0)
        assert np.array_equal(loads.table(t, P, dt), want)
