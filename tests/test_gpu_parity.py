"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (max relative displacement error over the sampled steps, the
oracle's e_max):
  * FP64 products and state: 1e-9 (both sides sum in different orders; the
    two libraries of master cells agree to 1e-14);
  * FP32 products with FP64 state: 1e-5 (the target for the mixed path).
"""

import sys

import numpy as np
import pytest

from meshgen import configs
from oracle.solver import Oracle, relative_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2103_09100_amd import solver
    return solver


@pytest.fixture(scope="module")
def cfg1_ref():
    m = configs.cfg1()
    o = Oracle(m)
    return m, o.run()


@pytest.mark.parametrize("assembly", ["atomic", "colour", "tiled"])
def test_cfg1_fp64(sim_mod, cfg1_ref, assembly):
    m, ref = cfg1_ref
    _say(f"[cfg1 fp64 {assembly}]")
    s = sim_mod.Simulation(m, assembly=assembly)
    assert abs(s.dt - ref["dt"]) <= 1e-14 * ref["dt"]
    snaps = s.run(1000, 50)
    e = relative_error(snaps, ref["snapshots"])
    _say(f"  e_max = {e:.3e}")
    assert e <= FP64_TOL


def test_cfg1_colour_bitwise_reproducible(sim_mod):
    m = configs.cfg1()
    a = sim_mod.Simulation(m, assembly="colour")
    b = sim_mod.Simulation(m, assembly="colour")
    a.step(300)
    b.step(120)
    b.step(180)
    assert np.array_equal(a.u(), b.u())


@pytest.fixture(scope="module")
def zoo_ref():
    m = configs.small_zoo(n_steps=200)
    o = Oracle(m, workers=8)
    return m, o, o.run(n_steps=200)


@pytest.mark.parametrize("prod,assembly,tol", [("fp64", "atomic", FP64_TOL), ("fp64", "colour", FP64_TOL),
                                                ("fp32", "atomic", FP32_TOL), ("fp64", "tiled", FP64_TOL),
                                                ("fp32", "tiled", FP32_TOL)])
def test_all_patterns(sim_mod, zoo_ref, prod, assembly, tol):
    m, o, ref = zoo_ref
    _say(f"[all-pattern mesh {m.n_dof} dofs, {prod} {assembly}]")
    s = sim_mod.Simulation(m, prod=prod, assembly=assembly, orient_seed=3)
    snaps = s.run(200, 50)
    e = relative_error(snaps, ref["snapshots"])
    _say(f"  e_max = {e:.3e}")
    assert e <= tol


@pytest.mark.parametrize("assembly", ["colour", "tiled"])
def test_internal_force_elementwise(sim_mod, zoo_ref, assembly):
    m, o, _ = zoo_ref
    u, um1 = configs.random_state(m.n_dof, seed=1, fixed=m.fixed)
    s = sim_mod.Simulation(m, assembly=assembly, orient_seed=5)
    s.write(u, um1, 0)
    f_gpu = s.internal_force()
    f_ref = o.internal_force(u)
    err = np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max()
    _say(f"[R_int elementwise {assembly}] {err:.3e}")
    assert err <= 1e-12


@pytest.fixture(scope="module")
def cfg2_ref():
    m = configs.cfg2()
    o = Oracle(m, workers=8)
    return m, o


@pytest.mark.parametrize("assembly,prod,tol", [("atomic", "fp64", 1e-12), ("tiled", "fp64", 1e-12),
                                                ("tiled", "fp32", 1e-5)])
def test_cfg2_full_size_one_step_sampled(sim_mod, cfg2_ref, assembly, prod, tol):
    m, o = cfg2_ref
    _say(f"[cfg2 one step, {m.n_dof} dofs, {assembly} {prod}]")
    dt = 0.5 * o.critical_dt()
    u, um1 = configs.random_state(m.n_dof, seed=2, fixed=m.fixed)
    s = sim_mod.Simulation(m, dt=dt, assembly=assembly, prod=prod, orient_seed=1)
    s.write(u, um1, 37)
    s.step(1)
    got = s.u().reshape(-1, 3)
    nodes = np.random.default_rng(3).choice(m.n_nodes, 400, replace=False)
    # include nodes of every kind of cell
    nodes = np.unique(np.concatenate([nodes, m.conn[m.conn_ptr[np.flatnonzero(m.cell_slots)[:200]]]]))
    want = o.sampled_step(u, um1, 37, dt, nodes)
    err = np.abs(got[nodes] - want).max() / np.abs(want).max()
    _say(f"  sampled one-step error {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("assembly", ["colour", "tiled"])
def test_checkpoint_resume(sim_mod, assembly):
    m = configs.cfg1()
    a = sim_mod.Simulation(m, assembly=assembly)
    a.step(200)
    u, um1, n = a.state()
    b = sim_mod.Simulation(m, assembly=assembly)
    b.write(u, um1, n)
    a.step(150)
    b.step(150)
    ua, ub = a.u(), b.u()
    if assembly == "colour":        # fixed summation order: bitwise
        assert np.array_equal(ua, ub)
    else:                           # on-chip atomics: summation order varies between runs
        assert np.abs(ua - ub).max() <= 1e-12 * np.abs(ua).max()


def test_single_cell_and_ragged_tiles(sim_mod):
    # one root cube: a single 8-node cell, base fixed, point load on a top corner
    from meshgen.octree import build_mesh
    m = build_mesh((1, 1, 1), 1.0, 0, 0, lambda l, i: np.zeros(len(i), bool), nu=0.25,
                   fixed=lambda lat, lmax: np.repeat((lat[:, 2] == 0)[:, None], 3, axis=1))
    configs.point_load(m, (1.0, 1.0, 1.0), (0, 0, -1.0))
    configs._run_params(m, fm=2.0, n_steps=100)
    o = Oracle(m)
    ref = o.run(n_steps=100)
    s = sim_mod.Simulation(m)
    e = relative_error(s.run(100, 50), ref["snapshots"])
    _say(f"[single cell] {e:.3e}")
    assert e <= FP64_TOL
    # 257 cells in one pattern -> one full and one ragged tile
    m = build_mesh((257, 1, 1), 1.0, 0, 0, lambda l, i: np.zeros(len(i), bool), nu=0.25,
                   fixed=lambda lat, lmax: np.repeat((lat[:, 0] == 0)[:, None], 3, axis=1))
    configs.patch_load(m, (0, 1), (0.5, 0.5), 1.0, pressure=-1.0)
    configs._run_params(m, fm=0.05, n_steps=100)
    o = Oracle(m)
    ref = o.run(n_steps=100)
    for asm in ("colour", "tiled"):
        s = sim_mod.Simulation(m, assembly=asm)
        e = relative_error(s.run(100, 50), ref["snapshots"])
        _say(f"[257-cell bar {asm}] {e:.3e}")
        assert e <= FP64_TOL


def test_unstable_step_reported(sim_mod):
    from paper_2103_09100_amd import binding
    m = configs.cfg1()
    s = sim_mod.Simulation(m)
    s2 = sim_mod.Simulation(m, dt=3.0 * s.dt_cr)
    with pytest.raises(binding.SbfemError) as ei:
        s2.step(2000)
        s2.u()
    assert ei.value.status == binding.EUNSTABLE


def test_unstable_step_reported_within_the_call(sim_mod):
    """With a check interval, the step_n call that produces the non-finite state reports it,
    stops at the end of that chunk and launches nothing more."""
    from paper_2103_09100_amd import binding
    m = configs.cfg1()
    s = sim_mod.Simulation(m)
    s2 = sim_mod.Simulation(m, dt=3.0 * s.dt_cr)
    s2.gpu.set_check_interval(50)
    with pytest.raises(binding.SbfemError) as ei:
        s2.step(100000)
    assert ei.value.status == binding.EUNSTABLE
    u, step = s2.gpu.read(0)  # the record was reported once; the state is that of the chunk's end
    _say(f"[unstable, check every 50 steps] stopped at step {step}")
    assert 0 < step < 100000 and step % 50 == 0
    assert not np.isfinite(u).all()
    # a stable mesh with the same interval steps exactly like one without
    a = sim_mod.Simulation(m, assembly="colour")
    b = sim_mod.Simulation(m, assembly="colour")
    b.gpu.set_check_interval(7)
    a.step(300)
    b.step(300)
    assert np.array_equal(a.u(), b.u())
    with pytest.raises(binding.SbfemError) as ei:
        b.gpu.set_check_interval(-1)
    assert ei.value.status == binding.EINVAL


def test_invalid_mesh_rejected(sim_mod):
    from paper_2103_09100_amd import binding, library
    m = configs.cfg1()
    pats = sim_mod.device_patterns(m.nu)
    pid, code, conn = library.canonicalise(m)
    bad = conn.copy()
    bad[5] = m.n_nodes
    d, keep = binding.make_desc(m, pid, code, bad, dt=0.01)
    with pytest.raises(binding.SbfemError) as ei:
        binding.Mesh(pats, d, keep)
    assert ei.value.status == binding.EINVAL
    p2 = pid.copy()
    p2[0] = 500
    d, keep = binding.make_desc(m, p2, code, conn, dt=0.01)
    with pytest.raises(binding.SbfemError):
        binding.Mesh(pats, d, keep)


def test_batched_meshes_match_alone_and_oracle(sim_mod):
    """Uneven meshes advanced together (one launch per step) == each alone == the oracle."""
    from paper_2103_09100_amd import binding
    meshes = [configs.cfg1(), configs.small_zoo(), configs.cfg2(lcoarse=2, lfine=5, delta=0.1)]
    steps = [120, 60, 90]
    alone, batch = [], []
    for m, n in zip(meshes, steps):
        a = sim_mod.Simulation(m, prod="fp64", assembly="tiled")
        a.step(n)
        alone.append(a.u())
        batch.append(sim_mod.Simulation(m, prod="fp64", assembly="tiled"))
    binding.step_batch([b.gpu for b in batch], steps)
    for m, n, a, b in zip(meshes, steps, alone, batch):
        ub, nb = b.gpu.read(0)
        assert nb == n
        err = np.abs(ub - a).max() / np.abs(a).max()
        _say(f"[batch vs alone {m.n_dof} dofs] {err:.3e}")
        assert err <= 1e-12
    o = Oracle(meshes[0])
    ref = o.run(n_steps=steps[0], snap_every=0, energy=False)
    err = np.abs(batch[0].u() - ref["u"]).max() / np.abs(ref["u"]).max()
    assert err <= FP64_TOL
    # a second batch call continues where the first stopped
    binding.step_batch([b.gpu for b in batch[:2]], [10, 30])
    assert batch[0].gpu.read(0)[1] == steps[0] + 10 and batch[1].gpu.read(0)[1] == steps[1] + 30


@pytest.mark.parametrize("kind", ["triangle", "sine_burst", "damped"])
def test_load_kinds_and_damping(sim_mod, kind):
    m = configs.cfg1(n_steps=300)
    if kind == "triangle":
        m.load.update(kind="triangle", t1=0.3)
    elif kind == "sine_burst":
        m.load.update(kind="sine_burst", t1=1.0, cycles=5)
    else:
        m.load.update(alpha=0.8)
    o = Oracle(m)
    ref = o.run(n_steps=300)
    for asm in ("tiled", "atomic"):
        s = sim_mod.Simulation(m, assembly=asm)
        e = relative_error(s.run(300, 50), ref["snapshots"])
        _say(f"[{kind} {asm}] {e:.3e}")
        assert e <= FP64_TOL


def test_serving_results_equal_alone(sim_mod):
    """Requests served in a mix (admission under a memory budget, batched steps) give the
    same result as each request run alone."""
    import torch
    from paper_2103_09100_amd.serve import Request, Server, latency_stats
    specs = [(1, 2e4, 80, 0.00), (2, 1.5e5, 140, 0.01), (3, 5e4, 60, 0.02), (4, 3e5, 100, 0.02),
             (5, 1e4, 200, 0.05), (6, 8e4, 120, 0.06)]
    reqs = [Request(rid, configs.request_mesh(rid, size, n), n, t) for rid, size, n, t in specs]
    st, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    fps = []
    for r in reqs:
        s = sim_mod.Simulation(r.mesh, prod="fp64")
        fps.append(s.footprint)
        s.step(r.n_steps)
        r.extra["alone"] = s.u()
        s.close()
    server = Server(budget_bytes=int(sum(fps) * 0.45), quantum=25, prod="fp64",
                    stream=st.cuda_stream, setup_stream=st2.cuda_stream)
    server.run(reqs)
    for r in reqs:
        err = np.abs(r.result - r.extra["alone"]).max() / np.abs(r.extra["alone"]).max()
        _say(f"[serve rid {r.rid} {r.dofs} dofs] admitted {r.admitted:.3f}s finished {r.finished:.3f}s err {err:.2e}")
        assert err <= 1e-12
    stats = latency_stats(reqs)
    _say(f"[serve] {stats}")
    assert stats["n"] == len(reqs)


def test_torch_caching_allocator_supplies_device_memory(sim_mod):
    """sbfem_set_allocator: the same run with device memory from torch's caching allocator."""
    import torch
    from paper_2103_09100_amd.torch_memory import use_hip_allocator, use_torch_allocator
    m = configs.small_zoo()
    a = sim_mod.Simulation(m, prod="fp32")
    a.step(60)
    ref = a.u()
    a.close()
    before = torch.cuda.memory_allocated()
    use_torch_allocator()
    try:
        b = sim_mod.Simulation(m, prod="fp32")
        grown = torch.cuda.memory_allocated() - before
        b.step(60)
        got = b.u()
        b.close()
    finally:
        use_hip_allocator()
    _say(f"[torch allocator] {grown / 1e6:.1f} MB from torch, footprint {b.footprint / 1e6:.1f} MB")
    assert grown >= b.footprint  # every buffer of the mesh came from torch (plus its rounding)
    assert torch.cuda.memory_allocated() == before
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_autotuned_shape_gives_the_same_result(sim_mod):
    from paper_2103_09100_amd.autotune import CANDIDATES, ShapeCache
    m = configs.cfg2(lcoarse=2, lfine=5, delta=0.1)
    cache = ShapeCache(prod="fp64", steps=4)
    best = cache.shape(m)
    _say(f"[autotune {m.n_dof} dofs] chosen {best}, table {cache.tables[cache.bucket(m)]}")
    assert best in CANDIDATES and cache.shape(m) is best
    ref = sim_mod.Simulation(m, prod="fp64")
    ref.step(50)
    tn, bt, btm = best
    s = sim_mod.Simulation(m, prod="fp64", tile_nodes=tn, block_threads=bt, block_threads_mixed=btm)
    s.step(50)
    assert np.abs(s.u() - ref.u()).max() <= 1e-12 * np.abs(ref.u()).max()


@pytest.mark.parametrize("shape", [(1024, 512, 256), (512, 256, 128), (64, 64, 64), (128, 512, 512)])
@pytest.mark.parametrize("prod", ["fp64", "fp32"])
def test_tile_shapes_agree(sim_mod, prod, shape):
    """Owner-tile shapes that take the generic staging (owned nodes beyond one per thread, or
    halo nodes beyond two per thread) or the up-front staging agree with the default shape:
    FP64 to rounding, FP32 products to the mixed-path bound (each tile rounds u relative to
    its own first owned node, so different tiles round differently)."""
    m = configs.small_zoo()
    tn, bt, btm = shape
    _say(f"[tile shape {shape} {prod}]")
    ref = sim_mod.Simulation(m, prod=prod)
    ref.step(60)
    s = sim_mod.Simulation(m, prod=prod, tile_nodes=tn, block_threads=bt, block_threads_mixed=btm)
    s.step(60)
    lay = s.gpu.layout()
    assert lay["tile_nodes"] <= tn
    err = np.abs(s.u() - ref.u()).max() / np.abs(ref.u()).max()
    _say(f"  tile_nodes {lay['tile_nodes']}, max local {lay['max_local_nodes']}: {err:.3e}")
    assert err <= (1e-12 if prod == "fp64" else 1e-5)


@pytest.mark.parametrize("prod,assembly,tol", [("fp64", "tiled", FP64_TOL), ("fp32", "tiled", FP32_TOL),
                                                ("fp64", "atomic", FP64_TOL)])
def test_two_poisson_ratio_libraries(sim_mod, prod, assembly, tol):
    """Inclusions with their own Poisson ratio: two pattern libraries in one mesh (pattern id =
    library * 144 + pattern, Sec. 3.2.3), each with its own regular-cell Walsh table, against the
    oracle, which computes every cell with its material's Poisson ratio."""
    m = configs.inclusion_mesh(seed=4, lcoarse=3, lfine=4, band=0.3, nu_incl=0.4)
    configs._run_params(m, fm=2.0, n_steps=150)
    assert (m.cell_mat == 1).any() and (m.cell_mat == 0).any()
    ref = Oracle(m, workers=8).run(n_steps=150)
    s = sim_mod.Simulation(m, prod=prod, assembly=assembly, orient_seed=7)
    assert s.patterns.library.n_patterns == 288
    assert abs(s.dt - ref["dt"]) <= 1e-14 * ref["dt"]
    e = relative_error(s.run(150, 50), ref["snapshots"])
    s.close()
    _say(f"[two Poisson ratios, {m.n_dof} dofs, {prod} {assembly}] e_max {e:.3e}")
    assert e <= tol


@pytest.mark.parametrize("prod,assembly,tol", [("fp64", "tiled", FP64_TOL), ("fp32", "tiled", FP32_TOL),
                                                ("fp64", "atomic", FP64_TOL)])
def test_table_load(sim_mod, prod, assembly, tol):
    """P(t_n) given per step (load kind TABLE), a seeded table shorter than the run, on the
    all-pattern mesh, against the oracle's table load; the table is part of the footprint."""
    m = configs.small_zoo(n_steps=160)
    o = Oracle(m, workers=8)
    dt = m.load["dt_factor"] * o.critical_dt()
    rng = np.random.default_rng(23)
    t = np.arange(120) * dt
    P = np.sin(2 * np.pi * t / (40 * dt)) * np.exp(-t / (60 * dt)) + 0.1 * rng.normal(size=120)
    m.load = dict(m.load, kind="table", P=P, dt=dt)
    ref = Oracle(m, workers=8).run(n_steps=160, dt=dt, snap_every=40, energy=False)
    s = sim_mod.Simulation(m, prod=prod, assembly=assembly)
    assert abs(s.dt - dt) <= 1e-14 * dt
    assert s.gpu.info()["device_bytes"] == s.footprint
    e = relative_error(s.run(160, 40), ref["snapshots"])
    s.close()
    _say(f"[table load {prod} {assembly}] e_max = {e:.3e}")
    assert e <= tol


def test_degenerate_inputs(sim_mod):
    """An empty mesh, a non-positive time step and an empty load table are refused; zero steps
    change nothing; a mesh whose dofs are all fixed stays at rest under load."""
    from paper_2103_09100_amd import binding, library
    m = configs.cfg1()
    pats = sim_mod.device_patterns(m.nu)
    pid, code, conn = library.canonicalise(m)
    d, keep = binding.make_desc(m, pid, code, conn, dt=0.01, assembly="tiled")
    d.n_cells = 0
    with pytest.raises(binding.SbfemError) as ei:
        binding.Mesh(pats, d, keep)
    assert ei.value.status == binding.EINVAL
    for dt in (0.0, -1.0, float("nan")):
        d, keep = binding.make_desc(m, pid, code, conn, dt=dt, assembly="tiled")
        with pytest.raises(binding.SbfemError) as ei:
            binding.Mesh(pats, d, keep)
        assert ei.value.status == binding.EINVAL
    d, keep = binding.make_desc(m, pid, code, conn, dt=0.01, assembly="tiled")
    d.load_kind = 3  # a table without entries
    with pytest.raises(binding.SbfemError) as ei:
        binding.Mesh(pats, d, keep)
    assert ei.value.status == binding.EINVAL
    s = sim_mod.Simulation(m)
    s.step(10)
    u, um1, n = s.state()
    s.step(0)
    u2, um12, n2 = s.state()
    assert n2 == n == 10 and np.array_equal(u, u2) and np.array_equal(um1, um12)
    s.close()
    m.fixed = np.ones_like(m.fixed)
    s = sim_mod.Simulation(m)
    s.step(50)
    assert not s.u().any()
    s.close()
