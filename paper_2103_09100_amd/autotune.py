"""Owner-tile shape autotuner.

A shape is (tile_nodes, block_threads, block_threads_mixed): nodes owned per block, threads per
block of the 8-node-tile kernel and of the hanging-node-tile kernel.  `tune` builds the mesh once
per candidate, times a few steps with the library's per-launch events (kernel time per step) and
keeps the fastest.  `ShapeCache` tunes once per mesh-size bucket (a factor of 4 in dofs) and
answers later meshes of that bucket from the cache, which is how the server picks shapes.
"""

import math

from .solver import Simulation

CANDIDATES = ((512, 512, 256), (256, 512, 256), (128, 512, 256), (1024, 512, 256), (256, 256, 256))
# one thread shape, so that meshes of every size still advance in the same batched launches
SERVING_CANDIDATES = ((512, 512, 256), (256, 512, 256), (128, 512, 256), (1024, 512, 256))


def time_shape(mesh, shape, prod="fp32", state="fp64", steps=10, warmup=3, stream=None):
    """Mean kernel time per step (ms) of the mesh with this owner-tile shape."""
    tn, bt, btm = shape
    sim = Simulation(mesh, prod=prod, state=state, assembly="tiled", tile_nodes=tn, block_threads=bt,
                     block_threads_mixed=btm, stream=stream)
    try:
        sim.step(warmup)
        sim.gpu.profile(True)
        sim.step(steps)
        prof = sim.gpu.profile_read()
        sim.gpu.profile(False)
    finally:
        sim.close()
    return sum(ms for ms, _ in prof.values()) / steps


def tune(mesh, prod="fp32", state="fp64", candidates=CANDIDATES, steps=10, stream=None):
    """(best shape, [(shape, ms per step), ...]) over the candidates."""
    table = [(tuple(c), time_shape(mesh, c, prod, state, steps, stream=stream)) for c in candidates]
    return min(table, key=lambda r: r[1])[0], table


class ShapeCache:
    """Tuned shapes per (product, state, size bucket); a bucket spans a factor of 4 in dofs."""

    def __init__(self, prod="fp32", state="fp64", candidates=CANDIDATES, steps=10, stream=None):
        self.prod, self.state, self.candidates, self.steps, self.stream = prod, state, candidates, steps, stream
        self.shapes = {}
        self.tables = {}

    def bucket(self, mesh):
        return int(math.log(max(mesh.n_dof, 1), 4))

    def shape(self, mesh):
        b = self.bucket(mesh)
        if b not in self.shapes:
            self.shapes[b], self.tables[b] = tune(mesh, self.prod, self.state, self.candidates, self.steps,
                                                  self.stream)
        return self.shapes[b]
