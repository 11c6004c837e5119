"""Balanced octree meshes on dense per-level grids.

The octree is stored as one boolean grid per level marking *refined* cells.
Refinement is decided top-down by a caller-supplied predicate; the 2:1 rule
(adjacent leaves differ by at most one level, Sec. 3.2.1) is then enforced
over face, edge and corner neighbours in one fine-to-coarse sweep: if a cell
at level l+1 is refined, every level-l cell that touches it must be refined.

Nodes are deduplicated on the integer lattice of spacing ``h0 * 2**-lmax``.
Cells are ordered along the Morton curve and nodes are numbered in the order
the cells first touch them (the heavy part runs in ``native/octree_gen.cpp``).
Face-centre nodes follow the face discretisation reading used throughout
this project: a face gets a centre node unless it has no mid-edge node or
exactly two on opposite edges (the two cases that tile by rectangles alone).
"""

import threading
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

from .slots import EDGES, FACES

# edges bounding each face (indices into EDGES), and which pairs are parallel
FACE_EDGES = []
for _f in FACES:
    _a = int(np.nonzero(_f)[0][0])
    FACE_EDGES.append([e for e in range(12) if EDGES[e][_a] == _f[_a]])
FACE_EDGES = np.array(FACE_EDGES, dtype=np.int64)


def face_centre_bits(edge_mask):
    """6-bit face-centre mask implied by a 12-bit edge mask (vectorised)."""
    edge_mask = np.asarray(edge_mask, dtype=np.uint32)
    out = np.zeros(edge_mask.shape, dtype=np.uint32)
    for f in range(6):
        es = FACE_EDGES[f]
        bits = [(edge_mask >> np.uint32(e)) & np.uint32(1) for e in es]
        nh = bits[0] + bits[1] + bits[2] + bits[3]
        # parallel edges of a face: same axis of zero coordinate
        axis = [int(np.nonzero(EDGES[e] == 0)[0][0]) for e in es]
        opposite = np.zeros(edge_mask.shape, dtype=bool)
        for i in range(4):
            for j in range(i + 1, 4):
                if axis[i] == axis[j]:
                    opposite |= (bits[i] == 1) & (bits[j] == 1) & (nh == 2)
        has = (nh >= 1) & ~opposite
        out |= has.astype(np.uint32) << np.uint32(f)
    return out


@dataclass
class Mesh:
    """A balanced octree mesh in natural numbering (see package docstring)."""
    roots: tuple
    h0: float
    lmax: int
    n_nodes: int
    cell_level: np.ndarray          # uint8 [C]
    cell_lat: np.ndarray            # int32 [C,3] min corner, lattice units
    cell_slots: np.ndarray          # uint32 [C]
    conn_ptr: np.ndarray            # int64 [C+1]
    conn: np.ndarray                # int32 [sum]
    node_lat: np.ndarray            # int32 [N,3]
    cell_mat: np.ndarray            # uint8 [C]
    mat_E: np.ndarray               # float64 [n_mat]
    mat_rho: np.ndarray             # float64 [n_mat]
    nu: float
    fixed: np.ndarray               # uint8 [3N]
    load_dof: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    load_val: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float64))
    load: dict = field(default_factory=dict)   # time function parameters
    meta: dict = field(default_factory=dict)
    mat_nu: np.ndarray = None       # float64 [n_mat] Poisson ratio per material (None: nu for all)

    def material_nu(self):
        """Poisson ratio of every material (the mesh-wide nu unless given per material)."""
        if self.mat_nu is None:
            return np.full(len(self.mat_E), self.nu)
        return np.asarray(self.mat_nu, dtype=np.float64)

    @property
    def n_cells(self):
        return int(self.cell_level.shape[0])

    @property
    def n_dof(self):
        return 3 * self.n_nodes

    def cell_h(self):
        return self.h0 * np.exp2(-self.cell_level.astype(np.float64))

    def cell_nodes(self, c):
        return self.conn[self.conn_ptr[c]:self.conn_ptr[c + 1]]

    def node_xyz(self):
        return self.node_lat.astype(np.float64) * (self.h0 * 2.0 ** -self.lmax)

    def fingerprint(self):
        """SHA-256 over the arrays that define the discrete problem (cells, connectivity,
        materials, constraints, loads): stored results of a run are valid for a regenerated
        mesh only if this matches."""
        import hashlib
        h = hashlib.sha256()
        for a in (self.cell_level, self.cell_slots, self.conn_ptr, self.conn, self.cell_mat, self.mat_E,
                  self.mat_rho, self.fixed, self.load_dof, self.load_val):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((self.roots, self.h0, self.lmax, self.n_nodes, self.nu)).encode())
        if self.mat_nu is not None:  # per-material ratios (the mesh-wide nu is hashed above)
            h.update(self.material_nu().tobytes())
        return h.hexdigest()


def _upsample(a):
    return a.repeat(2, 0).repeat(2, 1).repeat(2, 2)


def _block_or(a):
    n0, n1, n2 = a.shape
    return a.reshape(n0 // 2, 2, n1 // 2, 2, n2 // 2, 2).any(axis=(1, 3, 5))


def refine_levels(roots, lmin, lmax, refine):
    """Return list I[l] (l < lmax) of refined-cell grids after 2:1 balancing.

    ``refine(level, idx)`` gets integer cell indices (k,3) at ``level`` and
    returns a bool array; it is consulted only for lmin <= level < lmax.
    """
    roots = tuple(int(r) for r in roots)
    refined = []
    exists = np.ones(roots, dtype=bool)
    for lev in range(lmax):
        if lev < lmin:
            ref = exists.copy()
        else:
            ref = np.zeros_like(exists)
            idx = np.argwhere(exists)
            if idx.shape[0]:
                sel = np.asarray(refine(lev, idx), dtype=bool)
                ref[tuple(idx[sel].T)] = True
        refined.append(ref)
        exists = _upsample(ref)
    # 2:1 balance over the 26-neighbourhood, finest to coarsest
    st = np.ones((3, 3, 3), dtype=bool)
    for lev in range(lmax - 1, 0, -1):
        if refined[lev].any():
            dil = ndimage.binary_dilation(refined[lev], structure=st)
            refined[lev - 1] |= _block_or(dil)
    return refined


_NATIVE = None
# the native generator keeps one result between og_build and og_fetch: one caller at a time
_NATIVE_LOCK = threading.Lock()
_LOAD_LOCK = threading.Lock()


def _native():
    """Load (building on first use) the native leaf/node/connectivity routine."""
    global _NATIVE
    with _LOAD_LOCK:
        if _NATIVE is None:
            _NATIVE = _load_native()
    return _NATIVE


def _load_native():
    import ctypes
    import os
    import subprocess
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native")
    src = os.path.join(here, "octree_gen.cpp")
    lib = os.path.join(here, "libog.so")
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        build_native()
    L = ctypes.CDLL(lib)
    P = ctypes.c_void_p
    L.og_build.argtypes = [P, ctypes.c_int, P, P]
    L.og_fetch.argtypes = [P, P, P, P, P, P]
    return L


def build_native():
    import os
    import subprocess
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native")
    src = os.path.join(here, "octree_gen.cpp")
    lib = os.path.join(here, "libog.so")
    tmp = lib + ".tmp"
    subprocess.run(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp], check=True)
    os.replace(tmp, lib)
    return lib


def build_mesh(roots, h0, lmin, lmax, refine, material=None, mat_E=(1.0,), mat_rho=(1.0,),
               nu=0.25, fixed=None, keep_node_lat=True, mat_nu=None):
    """Build a balanced octree mesh.

    material(xyz_centres (k,3)) -> uint8 material id per cell (default all 0).
    fixed(node_lat (k,3) int, lmax) -> bool (k,3) fixed dofs (default: none).
    Cells follow the Morton curve; nodes are numbered in first-touch order
    along it (corners, mid-edge nodes, face centres of each cell in turn).
    """
    import ctypes
    roots = tuple(int(r) for r in roots)
    refined = [np.ascontiguousarray(r, dtype=np.uint8) for r in refine_levels(roots, lmin, lmax, refine)]
    L = _native()
    ptrs = (ctypes.c_void_p * max(1, len(refined)))(*[r.ctypes.data for r in refined])
    rts = np.array(roots, dtype=np.int64)
    counts = np.zeros(3, dtype=np.int64)
    with _NATIVE_LOCK:
        if L.og_build(rts.ctypes.data, int(lmax), ptrs, counts.ctypes.data) != 0:
            raise RuntimeError("octree generation failed")
        del refined
        C, n_nodes, n_conn = (int(v) for v in counts)
        cell_level = np.empty(C, dtype=np.uint8)
        cell_lat = np.empty((C, 3), dtype=np.int32)
        cell_slots = np.empty(C, dtype=np.uint32)
        conn_ptr = np.empty(C + 1, dtype=np.int64)
        conn = np.empty(n_conn, dtype=np.int32)
        node_lat = np.empty((n_nodes, 3), dtype=np.int32)
        L.og_fetch(cell_level.ctypes.data, cell_lat.ctypes.data, cell_slots.ctypes.data,
                   conn_ptr.ctypes.data, conn.ctypes.data, node_lat.ctypes.data)

    full = np.int64(1) << (lmax - cell_level.astype(np.int64))
    if material is None:
        cell_mat = np.zeros(C, dtype=np.uint8)
    else:
        centres = (cell_lat.astype(np.float64) + 0.5 * full[:, None]) * (h0 * 2.0 ** -lmax)
        cell_mat = np.asarray(material(centres), dtype=np.uint8)
        del centres
    fx = np.zeros(3 * n_nodes, dtype=np.uint8)
    if fixed is not None:
        fx = np.asarray(fixed(node_lat, lmax), dtype=np.uint8).reshape(-1)
    m = Mesh(roots=roots, h0=float(h0), lmax=int(lmax), n_nodes=n_nodes,
             cell_level=cell_level, cell_lat=cell_lat, cell_slots=cell_slots,
             conn_ptr=conn_ptr, conn=conn, node_lat=node_lat, cell_mat=cell_mat,
             mat_E=np.asarray(mat_E, dtype=np.float64),
             mat_rho=np.asarray(mat_rho, dtype=np.float64), nu=float(nu), fixed=fx,
             mat_nu=None if mat_nu is None else np.asarray(mat_nu, dtype=np.float64))
    return m


def node_id_lookup(mesh, lat):
    """Node ids at lattice points (k,3); -1 where no node exists."""
    lat = np.asarray(lat, dtype=np.int64).reshape(-1, 3)
    shape = tuple(r * (1 << mesh.lmax) + 1 for r in mesh.roots)
    grid = mesh.meta.get("_id_grid") if isinstance(mesh.meta, dict) else None
    if grid is None:
        grid = np.full(int(np.prod(shape)), -1, dtype=np.int32)
        nl = mesh.node_lat.astype(np.int64)
        grid[(nl[:, 0] * shape[1] + nl[:, 1]) * shape[2] + nl[:, 2]] = np.arange(mesh.n_nodes, dtype=np.int32)
    ok = (lat >= 0).all(1) & (lat[:, 0] < shape[0]) & (lat[:, 1] < shape[1]) & (lat[:, 2] < shape[2])
    out = np.full(len(lat), -1, dtype=np.int64)
    q = (lat[ok, 0] * shape[1] + lat[ok, 1]) * shape[2] + lat[ok, 2]
    out[ok] = grid[q]
    return out
