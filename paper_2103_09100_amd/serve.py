"""Continuous-batching serving loop over the C-ABI library.

Requests (a mesh, a number of steps, an arrival time) are admitted in arrival
order as soon as their device footprint fits the memory budget; every admitted
simulation stays resident.  Active simulations advance together: each round
calls ``sbfem_step_batch`` with up to ``quantum`` steps per simulation, so one
launch per step covers the tiles of every active mesh.  A simulation that has
taken all its steps is read back and released, which frees budget for the
queue.  Latency of a request = result on the host minus arrival.
"""

import time
from dataclasses import dataclass, field

import numpy as np

from . import binding
from .library import canonicalise, material_libraries
from .solver import device_patterns


@dataclass
class Request:
    rid: int
    mesh: object
    n_steps: int
    arrival: float
    result: np.ndarray = None
    admitted: float = None
    finished: float = None
    dofs: int = 0
    canon: tuple = None       # (pattern, orientation, connectivity) from canonicalise(), if done ahead
    extra: dict = field(default_factory=dict)

    def reset(self):
        """Forget the outcome of a previous serving run."""
        self.result, self.admitted, self.finished, self.dofs = None, None, None, 0
        for key in ("prep", "gpu", "left", "fp"):
            self.extra.pop(key, None)


def link_cells(req):
    """Link every cell of the request's mesh to its master pattern (part of building
    the request, like the mesh itself)."""
    req.canon = canonicalise(req.mesh)
    return req


class Server:
    """Admission in arrival order under a device-memory budget; host-side set-up (linking
    cells, building tiles: one host plan per request, which also gives its footprint) and
    the uploads of admitted requests run on two worker threads, the uploads on their own
    stream, so they overlap the stepping of the admitted simulations."""

    def __init__(self, budget_bytes=4 << 30, quantum=50, prod="fp32", stream=None, setup_stream=None,
                 clock=time.perf_counter, shapes=None, graph_steps=0):
        self.budget = int(budget_bytes)
        self.graph_steps = int(graph_steps)  # > 0: batched steps replayed from cached HIP graphs
        self.quantum = int(quantum)
        self.prod = prod
        self.shapes = shapes      # owner-tile shape per mesh: an object with .shape(mesh) (autotune.ShapeCache)
        self.stream = stream
        self.setup_stream = setup_stream
        self.clock = clock

    def _prepare(self, req):
        nus, _ = material_libraries(req.mesh)
        pats = device_patterns(nus[0] if len(nus) == 1 else nus, self.setup_stream)
        pid, code, conn = req.canon if req.canon is not None else canonicalise(req.mesh)
        tn, bt, btm = self.shapes.shape(req.mesh) if self.shapes is not None else (0, 0, 0)
        desc, keep = binding.make_desc(req.mesh, pid, code, conn, dt=1.0, prod=self.prod, assembly="tiled",
                                       tile_nodes=tn, block_threads=bt, block_threads_mixed=btm)
        dt_cr = binding.critical_dt(pats, desc)
        desc.dt = req.mesh.load.get("dt_factor", 0.5) * dt_cr
        plan = binding.Plan(pats, desc, keep)  # host set-up once: footprint now, upload on admission
        return pats, desc, keep, plan

    def run(self, requests, realtime=True):
        """Serve the requests; fills result, admitted and finished (seconds after start)."""
        import queue as q
        import threading

        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        arrived = q.Queue()       # main -> worker: requests to prepare, in arrival order
        prepared = []             # worker -> main: (request, footprint) ready for admission
        to_create = q.Queue()     # main -> worker: admitted (budget reserved), create on device
        created = []              # worker -> main: simulations resident on the device
        lock = threading.Lock()
        errors = []

        def prep_worker():   # host set-up in arrival order
            while True:
                r = arrived.get()
                if r is None:
                    return
                try:
                    r.extra["prep"] = self._prepare(r)
                    with lock:
                        prepared.append(r)
                except Exception as exc:   # surfaced by the main loop
                    with lock:
                        errors.append(exc)

        def create_worker():  # uploads of admitted requests on the set-up stream
            while True:
                r = to_create.get()
                if r is None:
                    return
                try:
                    pats, desc, keep, plan = r.extra.pop("prep")
                    r.extra["gpu"] = binding.Mesh(pats, desc, keep, self.setup_stream, plan=plan)
                    if self.graph_steps:
                        r.extra["gpu"].set_graph_steps(self.graph_steps)
                    with lock:
                        created.append(r)
                except Exception as exc:
                    with lock:
                        errors.append(exc)

        threads = [threading.Thread(target=prep_worker, daemon=True),
                   threading.Thread(target=create_worker, daemon=True)]
        for th in threads:
            th.start()
        active, used, i, n_done = [], 0, 0, 0
        try:
            while n_done < len(pending):
                with lock:
                    if errors:
                        raise errors[0]
                now = self.clock() - t0
                while i < len(pending) and (pending[i].arrival <= now or not realtime):
                    arrived.put(pending[i])
                    i += 1
                with lock:
                    # reserve budget in arrival order
                    while prepared:
                        r = prepared[0]
                        fp = r.extra["prep"][3].footprint
                        if fp > self.budget:
                            raise binding.SbfemError(binding.ENOMEM,
                                                     f"request {r.rid} needs {fp} bytes, budget {self.budget}")
                        if used + fp > self.budget:
                            break
                        prepared.pop(0)
                        used += fp
                        r.extra["fp"] = fp
                        to_create.put(r)
                    for r in created:
                        r.extra["left"] = r.n_steps
                        r.dofs = r.mesh.n_dof
                        r.admitted = self.clock() - t0
                        active.append(r)
                    created.clear()
                if not active:
                    time.sleep(0.001)
                    continue
                steps = [min(self.quantum, r.extra["left"]) for r in active]
                binding.step_batch([r.extra["gpu"] for r in active], steps, self.stream)
                still = []
                for r, k in zip(active, steps):
                    r.extra["left"] -= k
                    if r.extra["left"] == 0:
                        r.result, _ = r.extra["gpu"].read(0, self.stream)
                        r.finished = self.clock() - t0
                        r.extra.pop("gpu").close()
                        used -= r.extra["fp"]
                        n_done += 1
                    else:
                        still.append(r)
                active = still
        finally:
            to_create.put(None)
            arrived.put(None)
            for th in threads:
                th.join(timeout=60)
        return requests


def latency_stats(requests):
    lat = np.array([r.finished - r.arrival for r in requests])
    dof_steps = sum(r.dofs * r.n_steps for r in requests)
    span = max(r.finished for r in requests) - min(r.arrival for r in requests)
    return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()), n=len(requests),
                dof_steps=float(dof_steps), span_s=float(span), dof_steps_per_s=float(dof_steps / span))
