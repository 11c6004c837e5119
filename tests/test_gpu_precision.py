"""GPU precision forms: element products in FP64 / FP32 / FP16 / BF16 (FP32 accumulation for
the reduced ones) crossed with the displacement history stored in FP64, FP32 or as a
compensated FP32 pair, against the FP64 oracle.

Each case reports the oracle's e_max (max relative displacement error over the sampled
steps) and the discrete energy drift of the GPU trajectory, evaluated on the host in FP64
with the oracle's operator (the undamped central-difference scheme conserves
H_{n+1/2} - W_n exactly).  Bounds:
  * FP64 products with FP64 or compensated state: 1e-9 (summation order only);
  * FP32 products with FP64 or compensated state: 1e-5 (the mixed-precision target);
  * FP32 state: each stored value is rounded to 24 bits every step; the central-difference
    recursion carries that rounding as a random walk (measured 7.5e-7 with FP64 products,
    1.8e-6 with FP32 products over 1000 steps of the cube), held to the mixed target 1e-5;
  * FP16 / BF16 operands (unit roundoff 2^-11 / 2^-8): the stiffness seen by the scheme is
    perturbed by about that much, so the phase error grows like omega t u; bounded by
    5e-2 (FP16) and 4e-1 (BF16) over the 1000-step cube run.
"""

import sys

import numpy as np
import pytest

from meshgen import configs
from oracle.solver import Oracle, relative_error

pytestmark = pytest.mark.gpu

PRODS = ("fp64", "fp32", "fp16", "bf16")
STATES = ("fp64", "kahan32", "fp32")
BOUND = {
    ("fp64", "fp64"): 1e-9, ("fp64", "kahan32"): 1e-9, ("fp32", "fp64"): 1e-5, ("fp32", "kahan32"): 1e-5,
    ("fp64", "fp32"): 1e-5, ("fp32", "fp32"): 1e-5,
    ("fp16", "fp64"): 5e-2, ("fp16", "kahan32"): 5e-2, ("fp16", "fp32"): 5e-2,
    ("bf16", "fp64"): 4e-1, ("bf16", "kahan32"): 4e-1, ("bf16", "fp32"): 4e-1,
}


# Energy drift of the GPU trajectory over 300 steps (max |H_{n+1/2} - H_{-1/2} - W_n| / max |H|,
# H and W evaluated in FP64 with the oracle's operator).  The undamped scheme conserves it
# exactly in exact arithmetic; what remains is rounding of the operator (products) and of the
# stored state.  FP64 products with FP64 or compensated state: rounding only.  FP32 products:
# the stiffness the scheme applies differs from K by about 2^-24 relative, so each step's
# identity is off by that much of the energy exchanged.  FP32 state: the stored u_{n+1} is
# rounded to 24 bits.  16-bit operands: unit roundoff 2^-11 (FP16) and 2^-8 (BF16) in the
# products.
# Bounds about ten times the measured drifts (FP64 1.7e-15, compensated 3.9e-15; FP32 products
# 2.0e-8 / 6.2e-8; FP32 state 8.1e-8 / 9.9e-8; FP16 1.5e-4 .. 2.2e-4; BF16 1.0e-3 .. 1.1e-3).
DRIFT = {
    ("fp64", "fp64"): 1e-13, ("fp64", "kahan32"): 1e-13, ("fp32", "fp64"): 1e-6, ("fp32", "kahan32"): 1e-6,
    ("fp64", "fp32"): 1e-6, ("fp32", "fp32"): 1e-6,
    ("fp16", "fp64"): 2e-3, ("fp16", "kahan32"): 2e-3, ("fp16", "fp32"): 2e-3,
    ("bf16", "fp64"): 1e-2, ("bf16", "kahan32"): 1e-2, ("bf16", "fp32"): 1e-2,
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2103_09100_amd import solver
    return solver


@pytest.fixture(scope="module")
def cube():
    m = configs.cfg1()
    o = Oracle(m)
    return m, o, o.run()


def gpu_energy_drift(sim, o, n_steps):
    """Energy drift of the GPU trajectory over n_steps (host FP64, oracle operator)."""
    dt = sim.dt
    u, um1, _ = sim.state()
    d = u - um1
    H = [0.5 * (d @ (o.mdiag * d)) / dt ** 2 + 0.5 * (u @ o.internal_force(um1))]
    W = [0.0]
    for n in range(n_steps):
        sim.step(1)
        unew = sim.u()
        d = unew - u
        H.append(0.5 * (d @ (o.mdiag * d)) / dt ** 2 + 0.5 * (unew @ o.internal_force(u)))
        W.append(W[-1] + 0.5 * ((unew - um1) @ (o.load_at(n * dt) * o.b)))
        um1, u = u, unew
    H, W = np.array(H), np.array(W)
    return float(np.abs(H - H[0] - W).max() / np.abs(H).max())


@pytest.mark.parametrize("prod", PRODS)
@pytest.mark.parametrize("state", STATES)
def test_precision_matrix_cube(sim_mod, cube, prod, state):
    m, o, ref = cube
    s = sim_mod.Simulation(m, prod=prod, state=state, orient_seed=2)
    e = relative_error(s.run(1000, 50), ref["snapshots"])
    s.close()
    s = sim_mod.Simulation(m, prod=prod, state=state, orient_seed=2)
    drift = gpu_energy_drift(s, o, 300)
    s.close()
    _say(f"[precision cube {prod} products, {state} state] e_max {e:.3e}, energy drift (300 steps) {drift:.3e}")
    assert np.isfinite(e) and e <= BOUND[(prod, state)]
    assert np.isfinite(drift) and drift <= DRIFT[(prod, state)]


@pytest.fixture(scope="module")
def zoo():
    m = configs.small_zoo(n_steps=200)
    o = Oracle(m, workers=8)
    return m, o.run(n_steps=200)


@pytest.mark.parametrize("prod,state", [("fp32", "kahan32"), ("fp32", "fp32"), ("fp16", "fp64"), ("bf16", "fp64"),
                                        ("fp64", "kahan32")])
def test_precision_all_patterns(sim_mod, zoo, prod, state):
    """Every hanging-node pattern, random orientations: the dense 16-bit path and the state forms."""
    m, ref = zoo
    s = sim_mod.Simulation(m, prod=prod, state=state, orient_seed=4)
    e = relative_error(s.run(200, 50), ref["snapshots"])
    s.close()
    _say(f"[precision all patterns {m.n_dof} dofs, {prod} products, {state} state] e_max {e:.3e}")
    assert np.isfinite(e) and e <= BOUND[(prod, state)]


def test_lumped_mass_readback(sim_mod, cube):
    """read_state(3): the library's lumped mass equals the oracle's (summation order differs)."""
    m, o, _ = cube
    s = sim_mod.Simulation(m)
    M = s.gpu.read(3)[0]
    s.close()
    assert np.abs(M - o.mdiag).max() <= 1e-14 * np.abs(o.mdiag).max()


def test_reduced_forms_need_tiled_assembly(sim_mod):
    from paper_2103_09100_amd import binding
    m = configs.cfg1()
    for prod, state in (("fp16", "fp64"), ("fp32", "fp32")):
        with pytest.raises(binding.SbfemError):
            sim_mod.Simulation(m, prod=prod, state=state, assembly="atomic")
