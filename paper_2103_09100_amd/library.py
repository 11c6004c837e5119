"""Host set-up: the pattern library and the canonicalised mesh (Alg. 1, set-up).

``build_library(nu)`` computes K_p, lumped m_p and omega_p for the 144
patterns (Table "Data structure": the pre-computed K_e, M_e).
``canonicalise(mesh)`` links every cell to its master: pattern id,
orientation code and the node list rearranged into master order (the
paper's V, "already arranged according to the transformation matrix").
"""

import numpy as np

from . import patterns as pt
from .sbfem_cell import master_cell

_LIB_CACHE = {}


class Library:
    def __init__(self, nu, K, m, omega, ndof, masks):
        self.nu = nu
        self.K = K            # list of (ndof, ndof) FP64
        self.m = m            # list of (ndof,)
        self.omega = np.asarray(omega, dtype=np.float64)
        self.ndof = np.asarray(ndof, dtype=np.int32)
        self.masks = masks

    @property
    def n_patterns(self):
        return len(self.K)

    def flat(self):
        return (np.concatenate([k.ravel() for k in self.K]), np.concatenate(self.m))


def _one(args):
    mask, nu = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return master_cell(mask, nu)


def build_library(nu, workers=0):
    key = float(nu)
    if key in _LIB_CACHE:
        return _LIB_CACHE[key]
    tab = pt.table()
    args = [(int(m), nu) for m in tab.master_mask]
    if workers:
        from concurrent.futures import ProcessPoolExecutor
        import multiprocessing as mp
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            res = list(ex.map(_one, args, chunksize=4))
    else:
        res = [master_cell(*a) for a in args]
    K = [r[0] for r in res]
    m = [r[1] for r in res]
    om = [r[2] for r in res]
    lib = Library(nu, K, m, om, [k.shape[0] for k in K], tab.master_mask.copy())
    _LIB_CACHE[key] = lib
    return lib


def combine(libs):
    """One library of several Poisson ratios: pattern id = library index * 144 + pattern (each
    Poisson ratio needs its own masters, Sec. 3.2.3; E and rho scale, nu does not)."""
    K = [k for lib in libs for k in lib.K]
    m = [v for lib in libs for v in lib.m]
    om = np.concatenate([lib.omega for lib in libs])
    masks = np.concatenate([lib.masks for lib in libs])
    return Library(tuple(lib.nu for lib in libs), K, m, om, [k.shape[0] for k in K], masks)


def material_libraries(mesh):
    """Distinct Poisson ratios of the mesh's materials (sorted) and, per material, the index
    of its library among them."""
    nus = mesh.material_nu()
    uniq = sorted(set(float(v) for v in nus))
    return uniq, np.array([uniq.index(float(v)) for v in nus], dtype=np.int64)


def canonicalise(mesh, seed=None):
    """Per-cell pattern id, orientation code and master-order node list.

    With ``seed`` the orientation of each cell is drawn uniformly among the
    codes that map it onto its master (several exist for symmetric cells);
    otherwise the first valid code is used.
    """
    tab = pt.table()
    slots = np.asarray(mesh.cell_slots, dtype=np.int64)
    edge = slots & 0xFFF
    pid = tab.pattern_of[edge]
    if seed is None:
        code = tab.first_code[edge]
    else:
        rng = np.random.default_rng([11, seed])
        code = np.empty(len(edge), dtype=np.int64)
        for lo in range(0, len(edge), 1 << 22):
            e = edge[lo:lo + (1 << 22)]
            valid = tab.valid[:, e].T                     # (c, 48)
            cnt = valid.sum(1)
            pick = (rng.random(len(e)) * cnt).astype(np.int64)
            code[lo:lo + len(e)] = np.argmax(np.cumsum(valid, axis=1) > pick[:, None], axis=1)
    key = slots * 64 + code
    conn = np.asarray(mesh.conn)
    ptr = np.asarray(mesh.conn_ptr)
    out = conn.copy()
    # distinct (layout, orientation) pairs; those whose node map is the identity need no work
    present_keys = np.flatnonzero(np.bincount(key, minlength=1))
    moving = np.zeros(int(present_keys.max()) + 1, dtype=bool)
    perms = {}
    for k in present_keys:
        sm, c = int(k // 64), int(k % 64)
        p = tab.pattern_of[sm & 0xFFF]
        # the cell's face-centre nodes must land on its master's
        if int(pt.transform_slot_masks([sm], c)[0]) != int(tab.master_mask[p]):
            raise ValueError("cell layout is not a transformed master cell")
        perm = tab.conn_permutation(sm, c)
        if not np.array_equal(perm, np.arange(len(perm))):
            moving[k] = True
            perms[int(k)] = perm
    sel = np.flatnonzero(moving[key])
    if sel.size:
        ks = key[sel]
        order = np.argsort(ks, kind="stable")
        sel, ks = sel[order], ks[order]
        cuts = np.flatnonzero(np.diff(ks)) + 1
        for cells, k in zip(np.split(sel, cuts), ks[np.concatenate([[0], cuts])]):
            perm = perms[int(k)]
            base = ptr[cells][:, None]
            out[base + np.arange(len(perm))[None, :]] = conn[base + perm[None, :]]
    uniq, lib_of_mat = material_libraries(mesh)
    if len(uniq) > 1:  # pattern ids of the combined library
        pid = pid.astype(np.int64) + pt_count() * lib_of_mat[np.asarray(mesh.cell_mat, dtype=np.int64)]
    return pid.astype(np.uint16), code.astype(np.uint8), out


def pt_count():
    """Patterns per library (144)."""
    return len(pt.table().master_mask)
