"""The 2e7-dof sphere-band octree (levels 4/8, 2000 steps) through the C ABI against the FP64
oracle's stored snapshots (tests/golden/cfg4_oracle_snapshots.txt, written by the committed
script beside it, which calls only the oracle and the seeded mesh generator).

Per snapshot (every 100th step) the file holds |u|_inf over all dofs, the node where it is
reached and the displacements of 512 seeded sample nodes.  The error measure is the oracle's
e_max restricted to those nodes: max over snapshots of the largest displacement difference at
the sample nodes and the max node, over the largest stored |u|_inf.  The full field enters
through |u|_inf, since | |a|_inf - |b|_inf | <= |a - b|_inf.

Bounds: FP64 products and state 1e-9 (summation order only); the mixed forms (FP32 products
with FP64, compensated or FP32 state) 1e-5, the accuracy target over 2000 steps.
"""

import os
import sys

import numpy as np
import pytest

from meshgen import configs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "cfg4_oracle_snapshots.txt")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stored():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_oracle_snapshots import read
    ref = read(GOLDEN)
    mesh = configs.cfg4(n_steps=ref["steps"])
    assert mesh.fingerprint() == ref["mesh_fingerprint"], "mesh generator changed: regenerate the snapshots"
    assert mesh.n_dof == ref["n_dof"]
    return mesh, ref


@pytest.mark.parametrize("prod,state,tol", [("fp64", "fp64", 1e-9), ("fp32", "fp64", 1e-5),
                                            ("fp32", "kahan32", 1e-5), ("fp32", "fp32", 1e-5)])
def test_cfg4_2000_steps_against_stored_oracle(stored, prod, state, tol):
    from paper_2103_09100_amd import solver
    mesh, ref = stored
    _say(f"[cfg4 {mesh.n_dof} dofs, {prod} products, {state} state, {ref['steps']} steps]")
    s = solver.Simulation(mesh, prod=prod, state=state, assembly="tiled")
    assert abs(s.dt - ref["dt"]) <= 1e-14 * ref["dt"]
    sample = ref["sample_nodes"]
    den = max(r["norm"] for r in ref["snaps"])
    num = norm_gap = 0.0
    done = 0
    for r in ref["snaps"]:
        s.step(r["step"] - done)
        done = r["step"]
        u = s.u().reshape(-1, 3)
        num = max(num, float(np.abs(u[sample] - r["u"]).max()), float(np.abs(u[r["imax"]] - r["umax"]).max()))
        norm_gap = max(norm_gap, abs(float(np.abs(u).max()) - r["norm"]))
    s.close()
    e, g = num / den, norm_gap / den
    _say(f"  sampled e_max {e:.3e}, |u|_inf gap {g:.3e}")
    assert e <= tol and g <= tol
