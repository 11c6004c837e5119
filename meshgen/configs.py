"""Seeded workload recipes.

Each recipe returns a :class:`meshgen.octree.Mesh` whose ``load`` dict holds
the load-time parameters and the run parameters (``dt_factor``, ``n_steps``,
``alpha``); the nodal load vector b is in ``load_dof``/``load_val``.  The
paper's own geometries (STL terrain, CT foam) are not available, so these
synthetic boxes stand in for them with the shapes, level mixes and sizes the
workloads call for.

* ``cfg1``  unit cube, uniform 8x8x8 cells, base fixed, Ricker point load.
* ``cfg2``  level-7 band around a jittered sphere, level 3 elsewhere, plus
  a seeded zone of random refinement marks so that every cell pattern
  occurs; Ricker pressure on a random surface patch.
* ``cfg3``  three random ellipsoidal inclusions (E ratio 5, rho ratio 2),
  level 9 around and inside them, level 8 elsewhere (one GPU's share of a
  paper-scale panel, ~3e8 dofs).
* ``cfg4``  the cfg2 recipe at levels 8/4 (~2e7 dofs).
* ``serving_requests`` the Poisson request stream.
* ``bar``, ``sliding_cube`` small meshes used by the checks.
"""

import math
import os

import numpy as np

from .octree import build_mesh, node_id_lookup
from .slots import EDGES


def ricker_t1(fm):
    """Ricker parameter t1 for centre frequency fm (eq. Ricker_fm: fm = 5/(sqrt2 pi t1))."""
    return 5.0 / (math.sqrt(2.0) * math.pi * fm)


def _base_fixed(node_lat, lmax):
    z0 = node_lat[:, 2] == 0
    return np.repeat(z0[:, None], 3, axis=1)


def _box_dist_range(idx, level, h0, c):
    h = h0 * 2.0 ** -level
    lo = idx * h
    hi = lo + h
    d_near = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    dmin = np.sqrt((np.maximum(d_near, 0.0) ** 2).sum(1))
    far = np.maximum(np.abs(lo - c), np.abs(hi - c))
    dmax = np.sqrt((far ** 2).sum(1))
    return dmin, dmax


def _run_params(mesh, fm=2.0, P0=1.0, dt_factor=0.5, n_steps=1000, alpha=0.0):
    mesh.load = dict(kind="ricker", t1=ricker_t1(fm), P0=float(P0), fm=float(fm),
                     dt_factor=float(dt_factor), n_steps=int(n_steps), alpha=float(alpha))


def _id_grid(mesh):
    shape = tuple(r * (1 << mesh.lmax) + 1 for r in mesh.roots)
    grid = np.full(int(np.prod(shape)), -1, dtype=np.int32)
    nl = mesh.node_lat.astype(np.int64)
    grid[(nl[:, 0] * shape[1] + nl[:, 1]) * shape[2] + nl[:, 2]] = np.arange(mesh.n_nodes, dtype=np.int32)
    return grid


def point_load(mesh, xyz, direction, magnitude=1.0):
    scale = 2.0 ** mesh.lmax / mesh.h0
    lat = np.rint(np.asarray(xyz, dtype=np.float64) * scale).astype(np.int64)
    nid = int(node_id_lookup(mesh, lat[None, :])[0])
    if nid < 0:
        raise ValueError("no node at the requested load point")
    d = np.asarray(direction, dtype=np.float64)
    dofs, vals = [], []
    for a in range(3):
        if d[a] != 0.0:
            dofs.append(3 * nid + a)
            vals.append(magnitude * d[a])
    mesh.load_dof = np.array(dofs, dtype=np.int64)
    mesh.load_val = np.array(vals, dtype=np.float64)


def patch_load(mesh, face, centre, size, pressure=1.0):
    """Nodal forces of a uniform pressure on a square patch of a domain face.

    ``face`` = (axis, side) with side 0 (min) or 1 (max).  Every leaf face on
    that domain face gives each of its four corners a quarter of
    ``pressure * overlap_area``, along the inward normal.
    """
    axis, side = face
    b, c = (axis + 1) % 3, (axis + 2) % 3
    lmax = mesh.lmax
    ext = np.array(mesh.roots, dtype=np.int64) * (1 << lmax)
    full = (np.int64(1) << (lmax - mesh.cell_level.astype(np.int64)))
    lat = mesh.cell_lat.astype(np.int64)
    if side == 0:
        on = lat[:, axis] == 0
    else:
        on = lat[:, axis] + full == ext[axis]
    sel = np.flatnonzero(on)
    unit = mesh.h0 * 2.0 ** -lmax
    lo_b = lat[sel, b] * unit
    lo_c = lat[sel, c] * unit
    h = full[sel] * unit
    pb0, pb1 = centre[0] - size / 2, centre[0] + size / 2
    pc0, pc1 = centre[1] - size / 2, centre[1] + size / 2
    ob = np.clip(np.minimum(lo_b + h, pb1) - np.maximum(lo_b, pb0), 0.0, None)
    oc = np.clip(np.minimum(lo_c + h, pc1) - np.maximum(lo_c, pc0), 0.0, None)
    area = ob * oc
    keep = area > 0
    sel, area = sel[keep], area[keep]
    inward = 1.0 if side == 0 else -1.0
    forces = {}
    mesh.meta["_id_grid"] = _id_grid(mesh)
    for db in (0, 1):
        for dc in (0, 1):
            p = lat[sel].copy()
            if side == 1:
                p[:, axis] += full[sel]
            p[:, b] += db * full[sel]
            p[:, c] += dc * full[sel]
            nid = node_id_lookup(mesh, p)
            for n, a in zip(nid, area):
                forces[int(n)] = forces.get(int(n), 0.0) + 0.25 * pressure * a * inward
    mesh.meta.pop("_id_grid", None)
    nodes = np.array(sorted(forces), dtype=np.int64)
    mesh.load_dof = 3 * nodes + axis
    mesh.load_val = np.array([forces[int(n)] for n in nodes], dtype=np.float64)


def cfg1(n_steps=1000):
    """Unit cube, uniform 8^3 cells, base z=0 fixed, Ricker (fm=2) point load -z at top centre."""
    m = build_mesh((1, 1, 1), 1.0, 3, 3, lambda l, i: np.zeros(len(i), bool),
                   nu=0.25, fixed=_base_fixed)
    point_load(m, (0.5, 0.5, 1.0), (0.0, 0.0, -1.0))
    _run_params(m, fm=2.0, n_steps=n_steps)
    m.meta = dict(name="cfg1 uniform 8x8x8 cube")
    return m


def zoo_masks():
    """The listed edge configurations (one per class of cube cells)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zoo_masks.txt")
    return [int(l) for l in open(path) if l.strip() and not l.startswith("#")]


def zoo_refinement(level, masks):
    """Test blocks realising given edge configurations.

    Each block is 3x3x3 cells at ``level``; its centre cell is the test cell
    and, for every listed edge, the neighbour across that edge is refined
    once, which puts a mid-edge node on exactly that edge of the test cell.
    Blocks fill small cubes in the eight corners of the unit box.  Returns
    per-level boolean grids of cells to refine.
    """
    n = 1 << level
    rb = 1
    while 8 * rb ** 3 < len(masks):
        rb += 1
    span = 3 * rb
    if 2 * span > n:
        raise ValueError("zoo level too coarse for the number of test configurations")
    origins = []
    for x0 in (0, n - span):
        for y0 in (0, n - span):
            for z0 in (0, n - span):
                for bi in range(rb):
                    for bj in range(rb):
                        for bk in range(rb):
                            origins.append((x0 + 3 * bi, y0 + 3 * bj, z0 + 3 * bk))
    zone = np.zeros((n,) * 3, dtype=bool)
    ref = np.zeros((n,) * 3, dtype=bool)
    for (ox, oy, oz), m in zip(origins, masks):
        zone[ox:ox + 3, oy:oy + 3, oz:oz + 3] = True
        t = np.array([ox + 1, oy + 1, oz + 1])
        for e in range(12):
            if (m >> e) & 1:
                d = t + EDGES[e]
                ref[d[0], d[1], d[2]] = True
    grids = {level: ref}
    z = zone
    for lev in range(level - 1, -1, -1):
        z = z.reshape(z.shape[0] // 2, 2, z.shape[1] // 2, 2, z.shape[2] // 2, 2).any(axis=(1, 3, 5))
        grids[lev] = z
    return grids


def sphere_band_mesh(seed=0, lcoarse=3, lfine=7, radius=0.3, delta=0.1, zoo=None, nu=0.25):
    """Sphere-band octree (cfg2/cfg4 recipe): level lfine where a cell meets the
    shell |x - c| in [radius - delta, radius + delta], level lcoarse elsewhere,
    plus the test blocks of every listed cell configuration at level lfine-1."""
    rng = np.random.default_rng([2, seed])
    centre = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    if zoo is None:                   # the test blocks need a 32^3 grid at lfine-1
        zoo = lfine - 1 >= 5
    zgrids = zoo_refinement(lfine - 1, zoo_masks()) if zoo else {}

    def refine(level, idx):
        dmin, dmax = _box_dist_range(idx.astype(np.float64), level, 1.0, centre)
        band = (dmin <= radius + delta) & (dmax >= radius - delta) & (level < lfine)
        if level in zgrids:
            band |= zgrids[level][idx[:, 0], idx[:, 1], idx[:, 2]]
        return band

    m = build_mesh((1, 1, 1), 1.0, lcoarse, lfine, refine, nu=nu, fixed=_base_fixed)
    face_axis = int(rng.integers(0, 5))          # -x,+x,-y,+y,+z (never the fixed base)
    face = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 1)][face_axis]
    pc = rng.uniform(0.1, 0.9, size=2)
    patch_load(m, face, pc, 0.1)
    m.meta = dict(seed=seed, sphere_centre=centre.tolist(), radius=radius, delta=delta,
                  lcoarse=lcoarse, lfine=lfine, patch_face=face, patch_centre=pc.tolist())
    return m


def cfg2(seed=0, n_steps=500, lcoarse=3, lfine=7, delta=0.1, radius=0.3):
    m = sphere_band_mesh(seed=seed, lcoarse=lcoarse, lfine=lfine, delta=delta, radius=radius)
    _run_params(m, fm=2.0, n_steps=n_steps)
    m.meta["name"] = f"cfg2 sphere band L{lcoarse}/{lfine}"
    return m


def small_zoo(seed=0, n_steps=200):
    """Small mesh holding every cell pattern (levels 2..6, zoo at level 5)."""
    m = sphere_band_mesh(seed=seed, lcoarse=2, lfine=6, delta=0.02, radius=0.15)
    _run_params(m, fm=2.0, n_steps=n_steps)
    m.meta["name"] = "all-pattern test mesh L2/6"
    return m


def cfg4(seed=0, n_steps=2000, delta=0.15):
    m = sphere_band_mesh(seed=seed, lcoarse=4, lfine=8, delta=delta)
    _run_params(m, fm=2.0, n_steps=n_steps)
    m.meta["name"] = "cfg4 sphere band L4/8"
    return m


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ellipsoids(seed, n=3):
    rng = np.random.default_rng([3, seed])
    out = []
    for _ in range(n):
        c = rng.uniform(0.25, 0.75, size=3)
        a = rng.uniform(0.15, 0.3, size=3)
        out.append((c, a, _random_rotation(rng)))
    return out


def _ellipsoid_radius(x, ells, chunk=1 << 22):
    """min over ellipsoids of the scaled radius sqrt(sum((R^T(x-c)/a)^2)); <=1 inside.
    Evaluated in chunks; returns float32."""
    out = np.empty(x.shape[0], dtype=np.float32)
    for lo in range(0, x.shape[0], chunk):
        xs = x[lo:lo + chunk]
        r2 = np.full(xs.shape[0], np.inf, dtype=np.float64)
        for c, a, R in ells:
            y = (xs - c) @ (R / a[None, :])
            np.minimum(r2, np.einsum("ij,ij->i", y, y), out=r2)
        out[lo:lo + chunk] = np.sqrt(r2)
    return out


def inclusion_mesh(seed=0, lcoarse=8, lfine=9, band=1.05, keep_node_lat=True, nu=0.25, n_incl=3, nu_incl=None):
    """Ellipsoid-inclusion octree (cfg3 recipe): level lfine where the scaled
    ellipsoid radius is below 1+band, level lcoarse elsewhere; E=5, rho=2 inside, and the
    Poisson ratio nu_incl inside when given (a second pattern library)."""
    ells = ellipsoids(seed, n_incl)

    def refine(level, idx):
        h = 2.0 ** -level
        cc = (idx + 0.5) * h
        return (_ellipsoid_radius(cc, ells) <= 1.0 + band) & (level < lfine)

    def material(xyz):
        return (_ellipsoid_radius(xyz, ells) <= 1.0).astype(np.uint8)

    m = build_mesh((1, 1, 1), 1.0, lcoarse, lfine, refine, material=material,
                   mat_E=(1.0, 5.0), mat_rho=(1.0, 2.0), nu=nu, fixed=_base_fixed,
                   keep_node_lat=True, mat_nu=None if nu_incl is None else (nu, nu_incl))
    rng = np.random.default_rng([33, seed])
    face = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 1)][int(rng.integers(0, 5))]
    pc = rng.uniform(0.1, 0.9, size=2)
    patch_load(m, face, pc, 0.1)
    if not keep_node_lat:
        m.node_lat = None
    m.meta = dict(seed=seed, lcoarse=lcoarse, lfine=lfine, band=band, patch_face=face,
                  patch_centre=pc.tolist())
    return m


def cfg3(seed=0, n_steps=200, keep_node_lat=False):
    m = inclusion_mesh(seed=seed, lcoarse=8, lfine=9, band=1.05, keep_node_lat=keep_node_lat)
    _run_params(m, fm=4.0, n_steps=n_steps)
    m.meta["name"] = "cfg3 ellipsoid inclusions L8/9"
    return m


def bar(nx=16, level=0, nu=0.0, E=1.0, rho=1.0, fm=2.0):
    """nx x 1 x 1 root cubes (edge 1), optionally refined uniformly; x=0 face fixed;
    uniform end pressure on x = nx (nodal forces: quarter of each face area)."""
    def fixed(node_lat, lmax):
        x0 = node_lat[:, 0] == 0
        return np.repeat(x0[:, None], 3, axis=1)
    m = build_mesh((nx, 1, 1), 1.0, level, level, lambda l, i: np.zeros(len(i), bool),
                   mat_E=(E,), mat_rho=(rho,), nu=nu, fixed=fixed)
    patch_load(m, (0, 1), (0.5, 0.5), 1.0, pressure=-1.0)  # pulls in +x
    _run_params(m, fm=fm)
    m.meta = dict(name=f"bar {nx}x1x1 level {level}")
    return m


def sliding_cube(level, L=8.0, E=1000.0, rho=1.0, nu=0.3):
    """Cube of edge L, uniform cells of edge L/8/2^level, normal displacement
    fixed on every face (the eigenfrequency example of Sec. 5.1)."""
    lev = 3 + level
    ext = 1 << lev

    def fixed(node_lat, lmax):
        out = np.zeros(node_lat.shape, dtype=bool)
        for a in range(3):
            out[:, a] = (node_lat[:, a] == 0) | (node_lat[:, a] == ext)
        return out
    m = build_mesh((1, 1, 1), L, lev, lev, lambda l, i: np.zeros(len(i), bool),
                   mat_E=(E,), mat_rho=(rho,), nu=nu, fixed=fixed)
    m.meta = dict(name=f"sliding cube h={L / ext}")
    return m


def random_state(n_dof, seed, fixed=None, amplitude=1e-3):
    """Seeded displacement pair (u_n, u_{n-1}) for single-step checks; zero on fixed dofs."""
    rng = np.random.default_rng([7, seed])
    u = rng.uniform(-amplitude, amplitude, size=n_dof)
    up = u + rng.uniform(-amplitude, amplitude, size=n_dof) * 1e-2
    if fixed is not None:
        f = np.asarray(fixed).astype(bool)
        u[f] = 0.0
        up[f] = 0.0
    return u, up


def serving_requests(seed=5, n=256, rate=20.0, dof_lo=1e4, dof_hi=5e6):
    """Poisson request stream: arrival times, target sizes, steps and per-request seeds."""
    rng = np.random.default_rng([5, seed])
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.exp(rng.uniform(math.log(dof_lo), math.log(dof_hi), size=n))
    steps = rng.integers(200, 3001, size=n)
    seeds = rng.integers(0, 2 ** 31 - 1, size=n)
    return [dict(arrival=float(a), target_dof=float(s), n_steps=int(k), seed=int(sd))
            for a, s, k, sd in zip(arrivals, sizes, steps, seeds)]


def request_mesh(seed, target_dof, n_steps):
    """A serving request: 1-3 seeded inclusions, two octree levels chosen so that the
    mesh has roughly target_dof dofs, Ricker patch load with a seeded centre frequency
    resolved by at least 10 coarse cells per shear wavelength."""
    rng = np.random.default_rng([55, seed])
    n_incl = int(rng.integers(1, 4))
    nodes = target_dof / 3.0
    lev = int(np.clip(np.round(np.log2(np.cbrt(nodes / 3.0))), 2, 8))
    frac = float(np.clip((nodes / (2 ** lev + 1) ** 3 - 1.0) / 7.0, 0.02, 0.98))
    # band giving that refined fraction on the coarse grid
    ells = ellipsoids(seed, n_incl)
    n = 1 << lev
    g = (np.argwhere(np.ones((n, n, n), dtype=bool)) + 0.5) / n
    r = np.sort(_ellipsoid_radius(g, ells))
    band = max(float(r[min(len(r) - 1, int(frac * len(r)))]) - 1.0, 0.0)
    m = inclusion_mesh(seed=seed, lcoarse=lev, lfine=lev + 1, band=band, n_incl=n_incl)
    # Ricker centre frequency with at least 10 coarse cells per shear wavelength
    # (c_s = sqrt(E / (2 (1 + nu) rho)) of the matrix material)
    c_s = math.sqrt(1.0 / (2.0 * (1.0 + m.nu)))
    fm = float(rng.uniform(0.5, 1.0)) * c_s / (10.0 / n)
    _run_params(m, fm=fm, n_steps=n_steps)
    m.meta.update(name=f"request seed {seed}", target_dof=target_dof)
    return m
