"""GPU parity at the sizes the workloads name, and the start-up, footprint and serving paths,
against the FP64 oracle (through the C ABI).

* the 2.04e6-dof all-pattern sphere-band mesh over its full 500 steps (FP32 products with FP64
  state, and the plain FP64 path) against a full oracle run;
* one step of the 3.0e8-dof inclusion mesh, in the launch configuration the benchmark times,
  against the oracle at sampled nodes (the oracle visits only the cells around them);
* a non-zero initial displacement and velocity (eq. D0) against the oracle's start-up;
* a request served in a mix against the oracle;
* the footprint that admission uses against the bytes a mesh allocates.

Tolerances are those of the other parity tests: FP64 1e-9, FP32 products 1e-5 (max relative
displacement error over the sampled steps).
"""

import sys

import numpy as np
import pytest

from meshgen import configs
from oracle.solver import Oracle, relative_error, sampled_step_local

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
def cfg2_run():
    m = configs.cfg2()
    o = Oracle(m, workers=16)
    ref = o.run(n_steps=500, snap_every=50, energy=False)
    return m, ref


@pytest.mark.parametrize("prod,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_cfg2_full_run_against_oracle(sim_mod, cfg2_run, prod, tol):
    m, ref = cfg2_run
    _say(f"[cfg2 {m.n_dof} dofs, 500 steps, {prod} products, FP64 state]")
    s = sim_mod.Simulation(m, prod=prod, assembly="tiled", orient_seed=11)
    assert abs(s.dt - ref["dt"]) <= 1e-14 * ref["dt"]
    e = relative_error(s.run(500, 50), ref["snapshots"])
    s.close()
    _say(f"  e_max = {e:.3e}")
    assert e <= tol


@pytest.fixture(scope="module")
def cfg3_state():
    m = configs.cfg3(keep_node_lat=False)
    u, um1 = configs.random_state(m.n_dof, seed=9, fixed=m.fixed)
    rng = np.random.default_rng(10)
    hang_cells = np.flatnonzero(m.cell_slots)
    nodes = np.concatenate([rng.choice(m.n_nodes, 200, replace=False),
                            m.conn[m.conn_ptr[rng.choice(hang_cells, 60, replace=False)] + 3],
                            m.conn[m.conn_ptr[np.flatnonzero(m.cell_mat == 1)[::2000000]]],
                            m.load_dof[::7] // 3])
    return m, u, um1, np.unique(nodes), {}


@pytest.mark.parametrize("prod,tol", [("fp32", FP32_TOL), ("fp64", 1e-12)])
def test_cfg3_one_step_sampled(sim_mod, cfg3_state, prod, tol):
    """One step of the 3.0e8-dof mesh from a seeded random state (owner tiles, the benchmark's
    launch configuration) against the oracle at sampled nodes: random nodes, nodes of
    hanging-node cells, nodes in the inclusions and loaded nodes."""
    m, u, um1, nodes, cache = cfg3_state
    _say(f"[cfg3 {m.n_dof} dofs one step, {prod} products, {len(nodes)} sampled nodes]")
    s = sim_mod.Simulation(m, prod=prod, assembly="tiled")
    dt = s.dt
    s.write(u, um1, 5)
    s.step(1)
    got = s.u().reshape(-1, 3)[nodes]
    s.close()
    want = sampled_step_local(m, u, um1, 5, dt, nodes, cache=cache)
    # relative to the state's scale: one step moves u by O(dt^2 |M^-1 K u|) ~ |u|
    err = np.abs(got - want).max() / np.abs(want).max()
    _say(f"  sampled one-step error {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("assembly", ["tiled", "atomic"])
@pytest.mark.parametrize("alpha", [0.0, 0.7])
def test_initial_displacement_and_velocity(sim_mod, assembly, alpha):
    """Start-up from u0 != 0 and v0 != 0 (eq. D0 with K u0 and the damping term) on the
    all-pattern mesh, FP64, against the oracle."""
    m = configs.small_zoo(n_steps=150)
    m.load["alpha"] = alpha
    rng = np.random.default_rng([8, int(alpha * 10)])
    xyz = m.node_xyz()
    # smooth fields (a random random-phase mode), zero on the fixed base
    k = rng.uniform(1.0, 3.0, size=3)
    shape = np.sin(np.pi * xyz[:, 2] / 2) * np.cos(k[0] * xyz[:, 0] + k[1] * xyz[:, 1])
    u0 = (1e-3 * shape[:, None] * rng.normal(size=3)[None, :]).ravel()
    v0 = (2e-3 * shape[:, None] * rng.normal(size=3)[None, :]).ravel()
    u0[m.fixed.astype(bool)] = 0.0
    v0[m.fixed.astype(bool)] = 0.0
    o = Oracle(m, workers=8)
    ref = o.run(n_steps=150, snap_every=50, u0=u0, v0=v0, energy=False)
    s = sim_mod.Simulation(m, assembly=assembly, u0=u0, v0=v0, orient_seed=6)
    u_start, um1_start, n0 = s.state()
    ou0, oum1 = o.initial_state(s.dt, u0=u0, v0=v0)
    e0 = max(np.abs(u_start - ou0).max(), np.abs(um1_start - oum1).max()) / np.abs(ou0).max()
    e = relative_error(s.run(150, 50), ref["snapshots"])
    s.close()
    _say(f"[u0/v0 {assembly} alpha={alpha}] start-up {e0:.3e}, e_max {e:.3e}")
    assert n0 == 0 and e0 <= 1e-13
    assert e <= FP64_TOL


def test_footprint_equals_device_bytes(sim_mod):
    """The admission footprint is the bytes the mesh allocates, for every assembly and
    precision form, with and without an initial displacement."""
    meshes = [configs.cfg1(), configs.small_zoo(), configs.request_mesh(3, 5e4, 60)]
    cases = [("fp64", "fp64", "tiled"), ("fp32", "fp64", "tiled"), ("fp32", "fp32", "tiled"),
             ("fp16", "kahan32", "tiled"), ("fp64", "fp64", "atomic"), ("fp32", "fp64", "colour")]
    for m in meshes:
        for prod, state, asm in cases:
            s = sim_mod.Simulation(m, prod=prod, state=state, assembly=asm)
            got = s.gpu.info()["device_bytes"]
            s.close()
            assert got == s.footprint, (m.n_dof, prod, state, asm, got, s.footprint)
        u0 = np.zeros(m.n_dof)
        s = sim_mod.Simulation(m, prod="fp32", assembly="tiled", u0=u0)
        assert s.gpu.info()["device_bytes"] == s.footprint
        s.close()
    _say(f"[footprint] {len(meshes) * (len(cases) + 1)} meshes: footprint == device bytes")


def test_planned_create_matches_direct(sim_mod):
    """sbfem_plan_mesh + sbfem_create_mesh_planned: the plan's footprint is the footprint and
    the device bytes, and the mesh steps exactly like one created directly (colour assembly:
    bitwise; owner tiles: to the LDS summation order)."""
    from paper_2103_09100_amd import binding
    from paper_2103_09100_amd.library import canonicalise
    m = configs.small_zoo()
    for prod, asm, tol in (("fp64", "colour", 0.0), ("fp32", "tiled", 1e-12)):
        direct = sim_mod.Simulation(m, prod=prod, assembly=asm)
        pid, code, conn = canonicalise(m)
        desc, keep = binding.make_desc(m, pid, code, conn, dt=direct.dt, prod=prod, assembly=asm)
        plan = binding.Plan(direct.patterns, desc, keep)
        assert plan.footprint == binding.footprint(direct.patterns, desc) == direct.gpu.info()["device_bytes"]
        planned = binding.Mesh(direct.patterns, desc, keep, plan=plan)
        assert plan.handle is None  # consumed and freed
        assert planned.info()["device_bytes"] == plan.footprint
        direct.step(150)
        planned.step(150)
        a, b = direct.u(), planned.read(0)[0]
        err = float(np.abs(a - b).max() / np.abs(a).max())
        _say(f"[planned create {prod} {asm}] max rel diff {err:.2e}")
        assert err <= tol
        planned.close()
        direct.close()
    # a plan serves one create; a null plan is rejected
    import ctypes
    s = sim_mod.Simulation(m, prod="fp32", assembly="tiled")
    desc, keep = binding.make_desc(m, *canonicalise(m), dt=s.dt, prod="fp32", assembly="tiled")
    lib = binding._lib
    plan, nbytes = ctypes.c_void_p(), ctypes.c_int64()
    assert lib.sbfem_plan_mesh(ctypes.byref(plan), s.patterns.handle, ctypes.byref(desc), ctypes.byref(nbytes)) == 0
    first, second = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.sbfem_create_mesh_planned(ctypes.byref(first), plan, None) == 0
    assert lib.sbfem_create_mesh_planned(ctypes.byref(second), plan, None) == binding.EINVAL
    assert not second.value
    assert lib.sbfem_create_mesh_planned(ctypes.byref(second), None, None) == binding.EINVAL
    lib.sbfem_destroy_plan(plan)
    lib.sbfem_destroy_mesh(first)
    s.close()


@pytest.mark.parametrize("prod,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_served_requests_against_oracle(sim_mod, prod, tol):
    """Requests served in a mix (admitted under a memory budget, stepped in batched launches
    with others) against the FP64 oracle run of the same request."""
    import torch
    from paper_2103_09100_amd.serve import Request, Server
    specs = [(21, 1.2e4, 90, 0.00), (22, 6e4, 70, 0.005), (23, 2e4, 120, 0.01), (24, 1e5, 50, 0.01)]
    reqs = [Request(rid, configs.request_mesh(rid, size, n), n, t) for rid, size, n, t in specs]
    fp = [sim_mod.Simulation(r.mesh, prod=prod).footprint for r in reqs]
    st, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    server = Server(budget_bytes=int(sum(fp) * 0.6), quantum=20, prod=prod, stream=st.cuda_stream,
                    setup_stream=st2.cuda_stream)
    server.run(reqs)
    for r in reqs[:3]:
        ref = Oracle(r.mesh).run(n_steps=r.n_steps, snap_every=0, energy=False)
        err = np.abs(r.result - ref["u"]).max() / np.abs(ref["u"]).max()
        _say(f"[served rid {r.rid}, {r.mesh.n_dof} dofs, {r.n_steps} steps, {prod}] vs oracle {err:.3e}")
        assert err <= tol
