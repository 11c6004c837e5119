"""Step loops replayed from HIP graphs against the same steps launched one by one.

A graph of G steps reads the step number from device memory, so one captured graph
serves every chunk of a run.  Each check replays the graph several times, with
direct launches, reads (synchronisations) and a state rewrite between the replays,
and compares every intermediate state with a twin mesh that never uses graphs.
Both run the same kernels in the same order; the owner-tile assembly adds forces
with LDS atomics in an order that varies between runs, so the comparison allows
FP64 rounding (1e-12 relative), not bitwise equality.
"""

import sys

import numpy as np
import pytest

from meshgen import configs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2103_09100_amd import solver
    return solver


@pytest.mark.parametrize("prod", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["cfg1", "zoo"])
def test_single_mesh_graph_replays_equal_direct(sim_mod, which, prod):
    m = configs.cfg1() if which == "cfg1" else configs.small_zoo()
    G = 7  # odd: u and u_prev swap roles between replays
    _say(f"[graph single {which} {prod} G={G}]")
    g = sim_mod.Simulation(m, prod=prod, assembly="tiled", graph_steps=G)
    d = sim_mod.Simulation(m, prod=prod, assembly="tiled")
    for n in (20, 7, 3, 15, 30):  # partial chunks, one exact chunk, fewer steps than a chunk
        g.step(n)
        d.step(n)
        ug, sg = g.gpu.read(0)
        ud, sd = d.gpu.read(0)
        um_g, _ = g.gpu.read(1)
        um_d, _ = d.gpu.read(1)
        assert sg == sd
        e = max(_rel(ug, ud), _rel(um_g, um_d))
        _say(f"  step {sg}: {e:.3e}")
        assert e <= TOL
    # a rewritten state (checkpoint restore) is picked up by the next replay
    u, _ = d.gpu.read(0)
    um, _ = d.gpu.read(1)
    g.write(u, um, 40)
    d.write(u, um, 40)
    g.step(21)
    d.step(21)
    ug, sg = g.gpu.read(0)
    ud, sd = d.gpu.read(0)
    assert sg == sd == 61
    assert _rel(ug, ud) <= TOL
    # a new chunk length captures a new graph
    g.gpu.set_graph_steps(4)
    g.step(9)
    d.step(9)
    assert _rel(g.u(), d.u()) <= TOL


def test_batched_graph_replays_equal_direct(sim_mod):
    from paper_2103_09100_amd import binding
    meshes = [configs.cfg1(), configs.small_zoo(), configs.cfg2(lcoarse=2, lfine=5, delta=0.1)]
    G = 5
    gs = [sim_mod.Simulation(m, prod="fp64", assembly="tiled", graph_steps=G) for m in meshes]
    ds = [sim_mod.Simulation(m, prod="fp64", assembly="tiled") for m in meshes]
    # uneven step counts: the active set shrinks inside a call; the same sets recur in the
    # second call (cached graphs), and a subset forms a new set in the third
    for steps, idx in (([23, 17, 9], [0, 1, 2]), ([23, 17, 9], [0, 1, 2]), ([12, 6], [2, 0])):
        _say(f"[graph batch steps {steps} meshes {idx}]")
        binding.step_batch([gs[i].gpu for i in idx], steps)
        for i, n in zip(idx, steps):
            ds[i].step(n)
        for i in range(len(meshes)):
            ug, sg = gs[i].gpu.read(0)
            ud, sd = ds[i].gpu.read(0)
            assert sg == sd
            e = _rel(ug, ud)
            _say(f"  mesh {i} step {sg}: {e:.3e}")
            assert e <= TOL
    # single-mesh graphs and batch graphs of the same mesh interleave
    gs[1].step(11)
    ds[1].step(11)
    binding.step_batch([gs[1].gpu, gs[0].gpu], [10, 10])
    ds[1].step(10)
    ds[0].step(10)
    for i in (0, 1):
        assert gs[i].gpu.read(0)[1] == ds[i].gpu.read(0)[1]
        assert _rel(gs[i].u(), ds[i].u()) <= TOL


def test_graph_steps_rejected_outside_range(sim_mod):
    from paper_2103_09100_amd import binding
    m = configs.cfg1()
    s = sim_mod.Simulation(m, assembly="tiled")
    with pytest.raises(binding.SbfemError):
        s.gpu.set_graph_steps(-1)
    with pytest.raises(binding.SbfemError):
        s.gpu.set_graph_steps(5000)
    c = sim_mod.Simulation(m, assembly="colour")
    with pytest.raises(binding.SbfemError):
        c.gpu.set_graph_steps(8)


def test_graphs_step_directly_while_profiling_and_take_the_smallest_chunk(sim_mod):
    from paper_2103_09100_amd import binding
    m = configs.small_zoo()
    g = sim_mod.Simulation(m, prod="fp64", assembly="tiled", graph_steps=6)
    d = sim_mod.Simulation(m, prod="fp64", assembly="tiled")
    # profiling records an event pair per launch: the steps are launched one by one
    g.gpu.profile(True)
    g.step(12)
    prof = g.gpu.profile_read()
    g.gpu.profile(False)
    assert prof["element_8node"][1] == 12 and prof["element_larger"][1] == 12
    d.step(12)
    assert _rel(g.u(), d.u()) <= TOL
    # a batch of meshes with different chunk lengths replays chunks of the smallest
    h = sim_mod.Simulation(configs.cfg1(), prod="fp64", assembly="tiled", graph_steps=4)
    e = sim_mod.Simulation(configs.cfg1(), prod="fp64", assembly="tiled")
    binding.step_batch([g.gpu, h.gpu], [10, 10])
    d.step(10)
    e.step(10)
    assert g.gpu.read(0)[1] == 22 and h.gpu.read(0)[1] == 10
    assert _rel(g.u(), d.u()) <= TOL and _rel(h.u(), e.u()) <= TOL
