"""Alg. 1 (explicit solver in serial), FP64, element by element.

Set-up (Alg. 1, initialisation part):
  * each cell layout (slot mask) gets its own SBFEM matrices from
    :class:`oracle.element.Cell` at unit size, modulus and density, computed
    in the cell's natural node order, for the Poisson ratio of the cell's material
    (E and rho scale the unit matrices, nu does not: Sec. 3.2.3);
  * cell matrices scale as K = E h K_unit and M = rho h^3 M_unit (eq. KM_scale);
  * the global diagonal mass is the sum of the cells' lumped masses;
    Dirichlet dofs are enforced by a zero inverse mass (the dof never moves);
  * dt = dt_factor * min_e 2/omega_max,e (eqs. tcr, tcr_scale);
  * u_0 = 0 and, starting at rest, u_-1 = dt^2/2 M^-1 R_ext(0) (eq. D0).

Time loop (Alg. 1): R_int = sum_e K_e U_e (eq. Rinte), evaluated as one
matrix product per cell layout followed by a fixed-order scatter; R_ext at
t_n = n dt; u_{n+1} from eq. DnMdiag.
"""

import numpy as np

from . import loads
from .element import Cell


def _make_cell(args):
    mask, nu = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return Cell(mask, nu)


class Oracle:
    """Cell matrices are cached per (slot mask, Poisson ratio); ``groups`` lists, per such
    key, the cells and their dofs."""

    def __init__(self, mesh, cell_cache=None, workers=0):
        self.mesh = mesh
        self.cache = {} if cell_cache is None else cell_cache
        mat_nu = mesh.material_nu()
        self.nus = np.unique(mat_nu)
        # layout key of every cell: slot mask and the index of its material's Poisson ratio
        nu_idx = np.searchsorted(self.nus, mat_nu)[np.asarray(mesh.cell_mat, dtype=np.int64)]
        keys = mesh.cell_slots.astype(np.int64) * len(self.nus) + nu_idx
        self._key_nu = lambda k: (int(k) // len(self.nus), float(self.nus[int(k) % len(self.nus)]))
        self._cell_keys = keys
        self._prefill([self._key_nu(k) for k in np.unique(keys)], workers)
        n_dof = mesh.n_dof
        self.n_dof = n_dof
        self.groups = []
        h = mesh.cell_h()
        E = mesh.mat_E[mesh.cell_mat]
        rho = mesh.mat_rho[mesh.cell_mat]
        self.k_scale = E * h
        self.m_scale = rho * h ** 3
        for key in np.unique(keys):
            cells = np.flatnonzero(keys == key)
            ck = self._key_nu(key)
            cell = self.cell(*ck)
            n = cell.n_nodes
            nodes = mesh.conn[mesh.conn_ptr[cells][:, None] + np.arange(n)[None, :]].astype(np.int64)
            dofs = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(len(cells), 3 * n)
            self.groups.append((ck, cells, dofs))
        self._all_dofs = np.concatenate([g[2].ravel() for g in self.groups])
        # lumped global mass
        mdiag = np.zeros(n_dof)
        for key, cells, dofs in self.groups:
            m = self.cache[key].m
            mdiag += np.bincount(dofs.ravel(), (self.m_scale[cells][:, None] * m[None, :]).ravel(),
                                 minlength=n_dof)
        self.mdiag = mdiag
        fixed = mesh.fixed.astype(bool)
        if (mdiag[~fixed] <= 0).any():
            raise ValueError("non-positive lumped mass on a free dof")
        self.minv = np.where(fixed, 0.0, 1.0 / np.where(mdiag > 0, mdiag, 1.0))
        self.b = np.zeros(n_dof)
        np.add.at(self.b, mesh.load_dof, mesh.load_val)

    def _prefill(self, keys, workers):
        """Compute missing (mask, nu) cell layouts, optionally in a process pool."""
        todo = [k for k in keys if k not in self.cache]
        if workers and len(todo) > 8:
            from concurrent.futures import ProcessPoolExecutor
            import multiprocessing as mp
            with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
                for k, c in zip(todo, ex.map(_make_cell, todo, chunksize=4)):
                    self.cache[k] = c
        for k in todo:
            self.cell(*k)

    def cell(self, mask, nu):
        key = (int(mask), float(nu))
        if key not in self.cache:
            self.cache[key] = Cell(int(mask), float(nu))
        return self.cache[key]

    def cell_of(self, c):
        """The matrices of cell c (its layout and its material's Poisson ratio)."""
        return self.cell(*self._key_nu(self._cell_keys[c]))

    def critical_dt(self):
        """min over cells of 2/omega_max,e with omega_max,e = omega_unit sqrt(E/rho)/h."""
        mesh = self.mesh
        h = mesh.cell_h()
        E = mesh.mat_E[mesh.cell_mat]
        rho = mesh.mat_rho[mesh.cell_mat]
        best = np.inf
        for key, cells, _ in self.groups:
            w = self.cache[key].omega_max * np.sqrt(E[cells] / rho[cells]) / h[cells]
            best = min(best, float((2.0 / w).min()))
        return best

    def internal_force(self, u):
        """R_int = sum_e (E h)_e K_unit U_e: one product per layout, then one
        scatter of every element force in a fixed order (layouts ascending)."""
        parts = []
        for key, cells, dofs in self.groups:
            K = self.cache[key].K
            U = u[dofs]
            parts.append(((U @ K.T) * self.k_scale[cells][:, None]).ravel())
        return np.bincount(self._all_dofs, np.concatenate(parts), minlength=self.n_dof)

    def stiffness_sparse(self):
        """Assembled global K (scipy CSR) for checks."""
        from scipy import sparse
        rows, cols, vals = [], [], []
        for key, cells, dofs in self.groups:
            K = self.cache[key].K
            n = K.shape[0]
            rows.append(np.repeat(dofs, n, axis=1).ravel())
            cols.append(np.tile(dofs, (1, n)).ravel())
            vals.append((self.k_scale[cells][:, None, None] * K[None, :, :]).reshape(len(cells), -1).ravel())
        return sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(self.n_dof, self.n_dof))

    def load_at(self, t):
        return float(loads.evaluate(self.mesh.load, t))

    def initial_state(self, dt, u0=None, v0=None):
        """u_0 and the start-up point u_-1 (eq. D0) with U''_0 from the equation of motion."""
        alpha = self.mesh.load.get("alpha", 0.0)
        u0 = np.zeros(self.n_dof) if u0 is None else np.array(u0, dtype=np.float64)
        v0 = np.zeros(self.n_dof) if v0 is None else np.array(v0, dtype=np.float64)
        a0 = self.minv * (self.load_at(0.0) * self.b - self.internal_force(u0)) - alpha * v0 * (self.minv > 0)
        um1 = u0 - dt * v0 + 0.5 * dt * dt * a0
        return u0, um1

    def step(self, u, um1, n, dt, alpha=0.0, f=None):
        """One step of eq. DnMdiag; returns (u_{n+1}, f_n)."""
        if f is None:
            f = self.internal_force(u)
        r = self.load_at(n * dt) * self.b - f
        c = 0.5 * alpha * dt
        unew = (dt * dt * self.minv * r + 2.0 * u - (1.0 - c) * um1) / (1.0 + c)
        return unew, f

    def run(self, n_steps=None, dt=None, snap_every=50, energy=True, u0=None, v0=None, state=None, probes=None):
        """Run Alg. 1; returns dict with dt, snapshots {n: u_n}, energy terms, final state.

        probes: dofs whose time histories are kept (displacement at a point, Sec. 5.2;
        acceleration, Sec. 5.3): row k of probe_u holds u_{n+1} of step n = n0 + k, row k of
        probe_a the central-difference acceleration (u_{n+1} - 2 u_n + u_{n-1}) / dt^2 at t_n.
        """
        load = self.mesh.load
        if n_steps is None:
            n_steps = load["n_steps"]
        if dt is None:
            dt = load.get("dt_factor", 0.5) * self.critical_dt()
        alpha = load.get("alpha", 0.0)
        if state is not None:
            u, um1, n0 = state
            u, um1 = u.copy(), um1.copy()
        else:
            u, um1 = self.initial_state(dt, u0, v0)
            n0 = 0
        snaps = {}
        H, W = [], []
        probes = None if probes is None else np.asarray(probes, dtype=np.int64)
        pu, pa = [], []
        if energy:
            d = u - um1
            H.append(0.5 * (d @ (self.mdiag * d)) / dt ** 2 + 0.5 * (u @ self.internal_force(um1)))
            W.append(0.0)
        for k in range(n_steps):
            n = n0 + k
            unew, f = self.step(u, um1, n, dt, alpha)
            if energy:
                d = unew - u
                H.append(0.5 * (d @ (self.mdiag * d)) / dt ** 2 + 0.5 * (unew @ f))
                W.append(W[-1] + 0.5 * ((unew - um1) @ (self.load_at(n * dt) * self.b)))
            if probes is not None:
                pu.append(unew[probes])
                pa.append((unew[probes] - 2.0 * u[probes] + um1[probes]) / (dt * dt))
            um1, u = u, unew
            m = n + 1
            if (snap_every and m % snap_every == 0) or k == n_steps - 1:
                snaps[m] = u.copy()
        out = dict(dt=dt, snapshots=snaps, H=np.array(H), W=np.array(W), u=u, um1=um1, step=n0 + n_steps)
        if probes is not None:
            out["probe_u"] = np.array(pu).reshape(n_steps, len(probes))
            out["probe_a"] = np.array(pa).reshape(n_steps, len(probes))
        return out

    def sampled_step(self, u, um1, n, dt, nodes, alpha=0.0):
        """u_{n+1} at the given nodes only: each incident cell's force at that node."""
        mesh = self.mesh
        nodes = np.asarray(nodes, dtype=np.int64)
        pos = np.flatnonzero(np.isin(mesh.conn, nodes))
        cells = np.searchsorted(mesh.conn_ptr, pos, side="right") - 1
        f = {int(v): np.zeros(3) for v in nodes}
        for p, c in zip(pos, cells):
            nd = int(mesh.conn[p])
            lo, hi = mesh.conn_ptr[c], mesh.conn_ptr[c + 1]
            cn = mesh.conn[lo:hi].astype(np.int64)
            K = self.cell_of(c).K
            i = int(p - lo)
            ue = u[(3 * cn[:, None] + np.arange(3)).ravel()]
            f[nd] += self.k_scale[c] * (K[3 * i:3 * i + 3] @ ue)
        out = np.zeros((len(nodes), 3))
        P = self.load_at(n * dt)
        c = 0.5 * alpha * dt
        for j, v in enumerate(nodes):
            d = 3 * int(v) + np.arange(3)
            r = P * self.b[d] - f[int(v)]
            out[j] = (dt * dt * self.minv[d] * r + 2.0 * u[d] - (1.0 - c) * um1[d]) / (1.0 + c)
        return out


def sampled_step_local(mesh, u, um1, n, dt, nodes, alpha=0.0, cache=None):
    """u_{n+1} at the given nodes from one step of eq. DnMdiag, for meshes too large for
    :class:`Oracle`: only the cells incident to the nodes are visited.  Each node's force is
    the sum over its cells of s_e K_e u_e (rows of the node, eq. Rinte) and its lumped mass
    the sum of rho_e h_e^3 m_e (its entries, Sec. 3.3); fixed dofs keep a zero inverse mass;
    the load is P(t_n) b at the node.  Same arithmetic as :meth:`Oracle.sampled_step`."""
    cache = {} if cache is None else cache
    nodes = np.asarray(nodes, dtype=np.int64)
    sel = np.zeros(mesh.n_nodes, dtype=bool)
    sel[nodes] = True
    pos = np.flatnonzero(sel[mesh.conn])
    cells = np.searchsorted(mesh.conn_ptr, pos, side="right") - 1
    h = mesh.h0 * np.exp2(-mesh.cell_level[cells].astype(np.float64))
    E = mesh.mat_E[mesh.cell_mat[cells]]
    rho = mesh.mat_rho[mesh.cell_mat[cells]]
    f = {int(v): np.zeros(3) for v in nodes}
    mass = {int(v): np.zeros(3) for v in nodes}
    mat_nu = mesh.material_nu()
    for p, c, hc, Ec, rc in zip(pos, cells, h, E, rho):
        key = (int(mesh.cell_slots[c]), float(mat_nu[mesh.cell_mat[c]]))
        if key not in cache:
            cache[key] = Cell(*key)
        cell = cache[key]
        lo, hi = mesh.conn_ptr[c], mesh.conn_ptr[c + 1]
        cn = mesh.conn[lo:hi].astype(np.int64)
        i = int(p - lo)
        nd = int(mesh.conn[p])
        ue = u[(3 * cn[:, None] + np.arange(3)).ravel()]
        f[nd] += Ec * hc * (cell.K[3 * i:3 * i + 3] @ ue)
        mass[nd] += rc * hc ** 3 * cell.m[3 * i:3 * i + 3]
    b = {}
    for dof, val in zip(np.asarray(mesh.load_dof).tolist(), np.asarray(mesh.load_val).tolist()):
        b[dof] = b.get(dof, 0.0) + val
    P = float(loads.evaluate(mesh.load, n * dt))
    c = 0.5 * alpha * dt
    fixed = np.asarray(mesh.fixed).astype(bool)
    out = np.zeros((len(nodes), 3))
    for j, v in enumerate(nodes):
        d = 3 * int(v) + np.arange(3)
        minv = np.where(fixed[d], 0.0, 1.0 / mass[int(v)])
        bv = np.array([b.get(int(x), 0.0) for x in d])
        r = P * bv - f[int(v)]
        out[j] = (dt * dt * minv * r + 2.0 * u[d] - (1.0 - c) * um1[d]) / (1.0 + c)
    return out


def relative_error(test_snaps, ref_snaps):
    """max over sampled steps of |u_test - u_ref|_inf / max over the same steps of |u_ref|_inf."""
    keys = sorted(ref_snaps)
    num = max(float(np.abs(test_snaps[k] - ref_snaps[k]).max()) for k in keys)
    den = max(float(np.abs(ref_snaps[k]).max()) for k in keys)
    return num / den


def energy_drift(H, W):
    """max_n |H_{n+1/2} - H_{-1/2} - W_n| / max_n |H_{n+1/2}|."""
    H = np.asarray(H)
    W = np.asarray(W)
    return float(np.abs(H - H[0] - W).max() / np.abs(H).max())
