"""Degenerate calls through the C ABI: zero steps, empty and partly empty batches, and the
argument errors each entry point documents (no kernel is launched with bad input)."""

import sys

import numpy as np
import pytest

from meshgen import configs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2103_09100_amd import solver
    return solver


def test_zero_steps_change_nothing(sim_mod):
    m = configs.small_zoo()
    s = sim_mod.Simulation(m, prod="fp32", assembly="tiled")
    s.step(7)
    u0, n0 = s.gpu.read(0)
    um0, _ = s.gpu.read(1)
    s.step(0)
    u1, n1 = s.gpu.read(0)
    um1, _ = s.gpu.read(1)
    assert n1 == n0 == 7
    assert np.array_equal(u0, u1) and np.array_equal(um0, um1)


def test_batches_with_empty_entries(sim_mod):
    from paper_2103_09100_amd import binding
    binding.step_batch([], [])  # nothing to do
    ms = [configs.cfg1(), configs.small_zoo()]
    a = [sim_mod.Simulation(m, prod="fp64", assembly="tiled") for m in ms]
    b = [sim_mod.Simulation(m, prod="fp64", assembly="tiled") for m in ms]
    binding.step_batch([x.gpu for x in a], [0, 9])
    b[1].step(9)
    assert a[0].gpu.read(0)[1] == 0 and not np.any(a[0].u())
    ua, na = a[1].gpu.read(0)
    ub, nb = b[1].gpu.read(0)
    assert na == nb == 9
    assert np.abs(ua - ub).max() <= 1e-12 * np.abs(ub).max()
    binding.step_batch([x.gpu for x in a], [0, 0])
    assert a[1].gpu.read(0)[1] == 9


def test_argument_errors(sim_mod):
    from paper_2103_09100_amd import binding
    m = configs.cfg1()
    s = sim_mod.Simulation(m, assembly="tiled")
    t = sim_mod.Simulation(m, assembly="tiled")
    with pytest.raises(binding.SbfemError) as ei:
        s.step(-1)
    assert ei.value.status == binding.EINVAL
    with pytest.raises(binding.SbfemError) as ei:
        binding.step_batch([s.gpu, s.gpu], [1, 1])
    assert ei.value.status == binding.EINVAL
    with pytest.raises(binding.SbfemError) as ei:
        binding.step_batch([s.gpu, t.gpu], [1, -2])
    assert ei.value.status == binding.EINVAL
    with pytest.raises(binding.SbfemError) as ei:
        s.gpu.read(4)
    assert ei.value.status == binding.EINVAL
    with pytest.raises(binding.SbfemError) as ei:
        s.gpu.write(np.zeros(s.n_dof), np.zeros(s.n_dof), -1)
    assert ei.value.status == binding.EINVAL
    # the rejected calls left both meshes usable and untouched
    s.step(3)
    t.step(3)
    assert s.gpu.read(0)[1] == t.gpu.read(0)[1] == 3
    us, ut = s.u(), t.u()
    err = np.abs(us - ut).max() / max(np.abs(ut).max(), 1e-300)
    _say(f"[edge] after the rejected calls: {err:.2e}")
    assert err <= 1e-12
