"""High-level driver: from a natural-order octree mesh to a resident GPU simulation.

``Simulation(mesh)`` builds (or reuses) the pattern library for the mesh's
Poisson ratio, links every cell to its master, takes the time step as
``dt_factor`` times the element stability limit (eqs. tcr, tcr_scale) unless
given, and creates the device-resident state through the C ABI.
"""

import numpy as np

from . import binding
from .library import build_library, canonicalise, combine, material_libraries

_PATTERN_CACHE = {}


def device_patterns(nu, stream=None, workers=0):
    """Device library for one Poisson ratio, or for several (a sequence: one library each,
    pattern id = library index * 144 + pattern)."""
    nus = tuple(float(v) for v in nu) if np.ndim(nu) else (float(nu),)
    if nus not in _PATTERN_CACHE:
        libs = [build_library(v, workers=workers) for v in nus]
        _PATTERN_CACHE[nus] = binding.Patterns(libs[0] if len(libs) == 1 else combine(libs), stream)
    return _PATTERN_CACHE[nus]


class Simulation:
    def __init__(self, mesh, dt=None, prod="fp64", state="fp64", assembly="tiled", orient_seed=None,
                 u0=None, v0=None, stream=None, workers=0, tile_nodes=0, block_threads=0,
                 block_threads_mixed=0, graph_steps=0):
        self.mesh = mesh
        nus, _ = material_libraries(mesh)
        self.patterns = device_patterns(nus[0] if len(nus) == 1 else nus, stream, workers)
        pid, code, conn = canonicalise(mesh, seed=orient_seed)
        desc, keep = binding.make_desc(mesh, pid, code, conn, dt=1.0, prod=prod, state=state,
                                       assembly=assembly, u0=u0, v0=v0, tile_nodes=tile_nodes,
                                       block_threads=block_threads,
                                       block_threads_mixed=block_threads_mixed)
        self.dt_cr = binding.critical_dt(self.patterns, desc)
        if dt is None:
            dt = mesh.load.get("dt_factor", 0.5) * self.dt_cr
        desc.dt = float(dt)
        self.dt = float(dt)
        self._desc, self._keep, self._footprint = desc, keep, None
        self.gpu = binding.Mesh(self.patterns, desc, keep, stream)
        if graph_steps:
            self.gpu.set_graph_steps(graph_steps)
        self.stream = stream
        self.n_dof = mesh.n_dof

    @property
    def footprint(self):
        """Device bytes of this mesh by the library's admission estimate (runs its host set-up)."""
        if self._footprint is None:
            self._footprint = binding.footprint(self.patterns, self._desc)
        return self._footprint

    def step(self, n):
        self.gpu.step(n, self.stream)

    def u(self):
        return self.gpu.read(0, self.stream)[0]

    def state(self):
        u, n = self.gpu.read(0, self.stream)
        um1, _ = self.gpu.read(1, self.stream)
        return u, um1, n

    def internal_force(self):
        return self.gpu.read(2, self.stream)[0]

    def write(self, u, um1, step):
        self.gpu.write(u, um1, step, self.stream)

    def set_probes(self, dofs, capacity):
        """Record u_{n+1} and the central-difference acceleration at these dofs from now on."""
        self.gpu.set_probes(dofs, capacity, self.stream)

    def read_probes(self):
        """(u, a, first step) of the recorded probe rows."""
        return self.gpu.read_probes(self.stream)

    def run(self, n_steps, snap_every=50):
        """Step to n_steps, reading u at every snap_every-th step and the last."""
        snaps = {}
        done = 0
        while done < n_steps:
            k = min(snap_every, n_steps - done) if snap_every else n_steps - done
            self.step(k)
            done += k
            if (snap_every and done % snap_every == 0) or done == n_steps:
                snaps[done] = self.u()
        return snaps

    def close(self):
        self.gpu.close()


def relative_error(test, ref):
    keys = sorted(ref)
    num = max(float(np.abs(test[k] - ref[k]).max()) for k in keys)
    den = max(float(np.abs(ref[k]).max()) for k in keys)
    return num / den
