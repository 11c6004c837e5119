"""Balanced octree meshes on dense per-level grids.

The octree is stored as one boolean grid per level marking *refined* cells.
Refinement is decided top-down by a caller-supplied predicate; the 2:1 rule
(adjacent leaves differ by at most one level, Sec. 3.2.1) is then enforced
over face, edge and corner neighbours in one fine-to-coarse sweep: if a cell
at level l+1 is refined, every level-l cell that touches it must be refined.

Nodes are deduplicated on the integer lattice of spacing ``h0 * 2**-lmax``
and numbered along a Morton curve; cells are ordered along the same curve.
Face-centre nodes follow the face discretisation reading used throughout
this project: a face gets a centre node unless it has no mid-edge node or
exactly two on opposite edges (the two cases that tile by rectangles alone).
"""

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

from .slots import CORNERS, EDGES, FACES, popcount32

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


def _part1by2(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton3(x, y, z):
    return _part1by2(x) | (_part1by2(y) << np.uint64(1)) | (_part1by2(z) << np.uint64(2))


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


def build_mesh(roots, h0, lmin, lmax, refine, material=None, mat_E=(1.0,), mat_rho=(1.0,),
               nu=0.25, fixed=None, keep_node_lat=True):
    """Build a balanced octree mesh.

    material(xyz_centres (k,3)) -> uint8 material id per cell (default all 0).
    fixed(node_lat (k,3) int, lmax) -> bool (k,3) fixed dofs (default: none).
    """
    roots = tuple(int(r) for r in roots)
    refined = refine_levels(roots, lmin, lmax, refine)
    lat_shape = tuple(r * (1 << lmax) + 1 for r in roots)
    node_flag = np.zeros(lat_shape, dtype=bool)

    # leaves per level
    leaves = []
    for lev in range(lmax + 1):
        ex = np.ones(roots, dtype=bool) if lev == 0 else _upsample(refined[lev - 1])
        lf = ex & ~refined[lev] if lev < lmax else ex
        leaves.append(lf)
        if not lf.any():
            continue
        s = 1 << (lmax - lev)
        cg = np.zeros(tuple(n + 1 for n in lf.shape), dtype=bool)
        for di in (0, 1):
            for dj in (0, 1):
                for dk in (0, 1):
                    cg[di:di + lf.shape[0], dj:dj + lf.shape[1], dk:dk + lf.shape[2]] |= lf
        node_flag[::s, ::s, ::s] |= cg

    # per-level leaf coordinates and edge masks (mid-edge present iff a finer corner sits there)
    lat_list, lev_list, slot_list = [], [], []
    for lev in range(lmax + 1):
        lf = leaves[lev]
        if not lf.any():
            continue
        idx = np.argwhere(lf).astype(np.int64)
        s = 1 << (lmax - lev)
        lat = idx * s
        emask = np.zeros(idx.shape[0], dtype=np.uint32)
        if lev < lmax:
            half = s // 2
            for e in range(12):
                off = (EDGES[e] + 1) * half
                p = lat + off
                emask |= node_flag[p[:, 0], p[:, 1], p[:, 2]].astype(np.uint32) << np.uint32(e)
        lat_list.append(lat)
        lev_list.append(np.full(idx.shape[0], lev, dtype=np.uint8))
        slot_list.append(emask)
        del idx

    # face centres (after every edge mask is known), then mark those nodes
    for i, lat in enumerate(lat_list):
        lev = int(lev_list[i][0])
        fbits = face_centre_bits(slot_list[i])
        slot_list[i] = slot_list[i] | (fbits << np.uint32(12))
        if lev < lmax:
            half = (1 << (lmax - lev)) // 2
            for f in range(6):
                sel = ((fbits >> np.uint32(f)) & np.uint32(1)).astype(bool)
                if sel.any():
                    p = lat[sel] + (FACES[f] + 1) * half
                    node_flag[p[:, 0], p[:, 1], p[:, 2]] = True

    cell_lat = np.concatenate(lat_list).astype(np.int32)
    cell_level = np.concatenate(lev_list)
    cell_slots = np.concatenate(slot_list)
    del lat_list, lev_list, slot_list

    # Morton order of cells (by min corner)
    key = morton3(cell_lat[:, 0], cell_lat[:, 1], cell_lat[:, 2])
    order = np.argsort(key, kind="stable")
    del key
    cell_lat = cell_lat[order]
    cell_level = cell_level[order]
    cell_slots = cell_slots[order]
    del order

    # Morton numbering of nodes
    nidx = np.flatnonzero(node_flag)
    del node_flag
    nz = np.unravel_index(nidx, lat_shape)
    nkey = morton3(nz[0], nz[1], nz[2])
    norder = np.argsort(nkey, kind="stable")
    del nkey
    nidx = nidx[norder]
    n_nodes = int(nidx.shape[0])
    id_grid = np.full(int(np.prod(lat_shape)), -1, dtype=np.int32)
    id_grid[nidx] = np.arange(n_nodes, dtype=np.int32)
    node_lat = None
    if keep_node_lat:
        node_lat = np.stack(np.unravel_index(nidx, lat_shape), axis=1).astype(np.int32)
    del nz, norder

    # connectivity in natural slot order
    nper = 8 + popcount32(cell_slots).astype(np.int64)
    conn_ptr = np.zeros(cell_level.shape[0] + 1, dtype=np.int64)
    np.cumsum(nper, out=conn_ptr[1:])
    conn = np.full(int(conn_ptr[-1]), -1, dtype=np.int32)
    half = (np.int64(1) << (lmax - cell_level.astype(np.int64))) // 2  # 0 for lmax cells
    full = np.int64(1) << (lmax - cell_level.astype(np.int64))
    sy, sz = lat_shape[1] * lat_shape[2], lat_shape[2]

    def flat(p):
        return p[:, 0] * sy + p[:, 1] * sz + p[:, 2]

    for c in range(8):
        off = (CORNERS[c] + 1) // 2  # 0 or 1
        p = cell_lat.astype(np.int64) + off[None, :] * full[:, None]
        conn[conn_ptr[:-1] + c] = id_grid[flat(p)]
    for b in range(18):
        sel = np.flatnonzero((cell_slots >> np.uint32(b)) & np.uint32(1))
        if sel.shape[0] == 0:
            continue
        pos = EDGES[b] if b < 12 else FACES[b - 12]
        rank = 8 + popcount32(cell_slots[sel] & np.uint32((1 << b) - 1)).astype(np.int64)
        p = cell_lat[sel].astype(np.int64) + (pos[None, :] + 1) * half[sel, None]
        conn[conn_ptr[sel] + rank] = id_grid[flat(p)]
    del id_grid
    if (conn < 0).any():
        raise RuntimeError("mesh generator produced a dangling slot")

    centres = (cell_lat.astype(np.float64) + 0.5 * full[:, None]) * (h0 * 2.0 ** -lmax)
    if material is None:
        cell_mat = np.zeros(cell_level.shape[0], dtype=np.uint8)
    else:
        cell_mat = np.asarray(material(centres), dtype=np.uint8)
    del centres
    fx = np.zeros(3 * n_nodes, dtype=np.uint8)
    if fixed is not None:
        if node_lat is None:
            raise ValueError("fixed() needs node lattice coordinates")
        fx = np.asarray(fixed(node_lat, lmax), dtype=np.uint8).reshape(-1)
    return Mesh(roots=roots, h0=float(h0), lmax=int(lmax), n_nodes=n_nodes,
                cell_level=cell_level, cell_lat=cell_lat, cell_slots=cell_slots,
                conn_ptr=conn_ptr, conn=conn, node_lat=node_lat, cell_mat=cell_mat,
                mat_E=np.asarray(mat_E, dtype=np.float64),
                mat_rho=np.asarray(mat_rho, dtype=np.float64), nu=float(nu), fixed=fx)


def node_id_lookup(mesh, lat):
    """Node ids at lattice points (k,3); -1 where no node exists."""
    lat = np.asarray(lat, dtype=np.int64).reshape(-1, 3)
    lat_shape = tuple(r * (1 << mesh.lmax) + 1 for r in mesh.roots)
    nl = mesh.node_lat.astype(np.int64)
    keys = (nl[:, 0] * lat_shape[1] + nl[:, 1]) * lat_shape[2] + nl[:, 2]
    q = (lat[:, 0] * lat_shape[1] + lat[:, 1]) * lat_shape[2] + lat[:, 2]
    order = np.argsort(keys)
    pos = np.searchsorted(keys[order], q)
    pos = np.clip(pos, 0, keys.shape[0] - 1)
    hit = keys[order][pos] == q
    return np.where(hit, order[pos], -1)
