"""sbfem_step_batch_noalloc (the batched step with its work lists in the library's static
device buffer) against sbfem_step_batch on the same meshes: two calls in a row, the second
with fewer meshes and steps; then the mesh counters and a third ordinary call."""

import sys

import numpy as np
import pytest

from meshgen import configs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(sim_mod, meshes, prod):
    a = [sim_mod.Simulation(m, prod=prod, assembly="tiled") for m in meshes]
    b = [sim_mod.Simulation(m, prod=prod, assembly="tiled") for m in meshes]
    return a, b


@pytest.mark.parametrize("prod,tol", [("fp64", 1e-12), ("fp32", 1e-12)])
def test_noalloc_batch_matches_batch(prod, tol):
    from paper_2103_09100_amd import binding, solver
    meshes = [configs.cfg1(), configs.small_zoo(), configs.request_mesh(7, 8e4, 100),
              configs.cfg2(lcoarse=2, lfine=5, delta=0.1)]
    a, b = _pair(solver, meshes, prod)
    calls = [[40, 25, 33, 18], [9, 0, 4]]  # the second call: fewer meshes and steps
    for k, steps in enumerate(calls):
        sub_a = [x.gpu for x in a[:len(steps)]]
        sub_b = [x.gpu for x in b[:len(steps)]]
        binding.step_batch(sub_a, steps)
        binding.step_batch_noalloc(sub_b, steps)
        for i, (x, y) in enumerate(zip(a, b)):
            ua, na = x.gpu.read(0)
            ub, nb = y.gpu.read(0)
            assert na == nb
            err = np.abs(ua - ub).max() / max(np.abs(ua).max(), 1e-300)
            _say(f"[noalloc call {k} mesh {i} {meshes[i].n_dof} dofs {prod}] step {nb}: {err:.2e}")
            assert err <= tol
    # the meshes stepped without allocation continue normally
    binding.step_batch([y.gpu for y in b], [5, 5, 5, 5])
    binding.step_batch([x.gpu for x in a], [5, 5, 5, 5])
    for x, y in zip(a, b):
        ua, ub = x.u(), y.u()
        assert np.abs(ua - ub).max() <= tol * max(np.abs(ua).max(), 1e-300)
    for s in a + b:
        s.close()


def test_noalloc_rejects_bad_arguments():
    from paper_2103_09100_amd import binding, solver
    s = solver.Simulation(configs.cfg1(), assembly="tiled")
    binding.step_batch_noalloc([], [])
    with pytest.raises(binding.SbfemError) as ei:
        binding.step_batch_noalloc([s.gpu, s.gpu], [1, 1])
    assert ei.value.status == binding.EINVAL
    with pytest.raises(binding.SbfemError) as ei:
        binding.step_batch_noalloc([s.gpu], [-1])
    assert ei.value.status == binding.EINVAL
    assert s.gpu.read(0)[1] == 0
    s.close()
