"""Pins of the oracle's Alg. 1 loop against closed forms, invariants and brute force."""

import copy
import os

import numpy as np
import pytest

from meshgen import configs
from oracle import loads
from oracle.solver import Oracle, energy_drift, relative_error

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ricker_beam.txt")


@pytest.fixture(scope="module")
def cfg1_run():
    m = configs.cfg1()
    o = Oracle(m)
    return m, o, o.run()


def test_energy_identity_cfg1(cfg1_run):
    """Undamped CDM conserves H_{n+1/2} up to the external work (derived from eq. DnMdiag)."""
    _, _, r = cfg1_run
    assert energy_drift(r["H"], r["W"]) < 1e-12
    assert np.abs(r["H"]).max() > 0


def test_cfg1_dt_and_mass(cfg1_run):
    m, o, r = cfg1_run
    assert np.isclose(o.mdiag.sum() / 3, 1.0, rtol=1e-13)          # total mass rho V
    # 8-node cell: 2/omega_max = h sqrt(rho/E)/sqrt(2) for nu = 0.25, h = 1/8
    assert np.isclose(r["dt"], 0.5 * (1 / 8) / np.sqrt(2), rtol=1e-12)


def test_cfg1_mirror_symmetry(cfg1_run):
    """D4 symmetry of cfg1 about the vertical axis through the load."""
    m, _, r = cfg1_run
    lat = m.node_lat.astype(np.int64)
    key = {tuple(p): i for i, p in enumerate(lat.tolist())}
    mx = np.array([key[(8 - x, y, z)] for x, y, z in lat.tolist()])
    sw = np.array([key[(y, x, z)] for x, y, z in lat.tolist()])
    for n in (100, 500, 1000):
        u = r["snapshots"][n].reshape(-1, 3)
        s = np.abs(u).max()
        um = u[mx]
        assert np.abs(um[:, 0] + u[:, 0]).max() < 1e-10 * s
        assert np.abs(um[:, 1:] - u[:, 1:]).max() < 1e-10 * s
        us = u[sw]
        assert np.abs(us[:, 0] - u[:, 1]).max() < 1e-10 * s
        assert np.abs(us[:, 2] - u[:, 2]).max() < 1e-10 * s


def test_ebe_force_equals_assembled_and_bruteforce():
    m = configs.cfg2(lcoarse=2, lfine=4, delta=0.1)
    o = Oracle(m)
    rng = np.random.default_rng(0)
    u = rng.normal(size=m.n_dof)
    f = o.internal_force(u)
    K = o.stiffness_sparse()
    assert np.abs(f - K @ u).max() < 1e-12 * np.abs(f).max()
    g = np.zeros(m.n_dof)
    for c in range(m.n_cells):
        nodes = m.cell_nodes(c).astype(np.int64)
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        g[dofs] += o.k_scale[c] * (o.cell_of(c).K @ u[dofs])
    assert np.abs(f - g).max() < 1e-12 * np.abs(f).max()
    # assembled K symmetric, rigid modes removed only by the fixed base
    assert abs(K - K.T).max() < 1e-12 * abs(K).max()


def _chain(n_el, dt, n_steps, P):
    """Textbook 1D lumped linear-element chain (E=A=rho=h=1), fixed at node 0, force P(t) at the end."""
    k = np.zeros((n_el + 1, n_el + 1))
    for e in range(n_el):
        k[e:e + 2, e:e + 2] += np.array([[1, -1], [-1, 1.0]])
    mass = np.ones(n_el + 1)
    mass[-1] = 0.5
    minv = 1 / mass
    minv[0] = 0.0
    b = np.zeros(n_el + 1)
    b[-1] = 1.0
    u = np.zeros(n_el + 1)
    um1 = 0.5 * dt * dt * minv * P(0.0) * b
    hist = []
    for n in range(n_steps):
        unew = dt * dt * minv * (P(n * dt) * b - k @ u) + 2 * u - um1
        um1, u = u, unew
        hist.append(u.copy())
    return np.array(hist)


def test_bar_reduces_to_1d_chain_and_travels_at_wave_speed():
    """nu = 0 bar: 3D lumped SBFEM == 1D lumped chain (exact) and matches d'Alembert."""
    nx = 48
    m = configs.bar(nx=nx)
    t1 = 40.0
    m.load = dict(kind="ricker", t1=t1, P0=1.0, dt_factor=0.5, n_steps=0, alpha=0.0)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    assert np.isclose(o.critical_dt(), 1.0, rtol=1e-12)           # 2/omega = h/c for nu = 0
    n_steps = int((t1 * 2 + 0.5 * nx) / dt)
    snaps = o.run(n_steps=n_steps, dt=dt, snap_every=1, energy=False)["snapshots"]
    chain = _chain(nx, dt, n_steps, lambda t: loads.ricker(t, t1))
    lat = m.node_lat.astype(np.int64)
    sec = lat[:, 0]
    scale = np.abs(chain).max()
    for n in range(1, n_steps + 1, 7):
        u = snaps[n].reshape(-1, 3)
        assert np.abs(u[:, 1:]).max() < 1e-12 * scale
        assert np.abs(u[:, 0] - chain[n - 1][sec]).max() < 1e-11 * scale
    # d'Alembert before the reflection from the fixed end returns:
    # u(x,t) = (c/EA) int_0^{t-(L-x)/c} P
    x = nx // 2
    tt = np.arange(1, n_steps + 1) * dt
    fine = np.linspace(0, tt.max(), 200001)
    cum = np.concatenate([[0], np.cumsum(0.5 * (loads.ricker(fine[1:], t1) + loads.ricker(fine[:-1], t1))
                                         * np.diff(fine))])
    exact = np.interp(tt - (nx - x), fine, cum, left=0.0)
    window = tt < nx + x - 1.0
    num = chain[:, x][window]
    assert np.abs(num - exact[window]).max() < 0.03 * np.abs(exact[window]).max()


def test_stability_threshold_cfg1():
    """Element-wise limit bounds the global one; CDM diverges just above 2/omega_global (eq. tcr)."""
    m = configs.cfg1()
    o = Oracle(m)
    K = o.stiffness_sparse().toarray()
    free = np.flatnonzero(~m.fixed.astype(bool))
    s = 1 / np.sqrt(o.mdiag[free])
    A = K[np.ix_(free, free)] * s[:, None] * s[None, :]
    w_glob = np.sqrt(np.linalg.eigvalsh(A).max())
    assert 2 / w_glob >= o.critical_dt() * (1 - 1e-12)
    m0 = copy.copy(m)
    m0.load_dof = np.zeros(0, np.int64)
    m0.load_val = np.zeros(0)
    o0 = Oracle(m0)
    rng = np.random.default_rng(1)
    u0 = rng.normal(size=m.n_dof) * (~m.fixed.astype(bool))
    grow = {}
    for fac in (0.98, 1.02):
        r = o0.run(n_steps=400, dt=fac * 2 / w_glob, snap_every=0, energy=False, state=(u0, u0, 0))
        grow[fac] = np.abs(r["u"]).max() / np.abs(u0).max()
    assert grow[0.98] < 10
    assert grow[1.02] > 1e6


def _cube_reference(L, E, nu, rho, count):
    vp = np.sqrt(E * (1 - nu) / (rho * (1 + nu) * (1 - 2 * nu)))
    vs = np.sqrt(E / (2 * rho * (1 + nu)))
    out = []
    for l in range(12):
        for mm in range(12):
            for n in range(12):
                if l == mm == n == 0:
                    continue
                k = np.pi * np.sqrt(l * l + mm * mm + n * n) / L
                zeros = (l == 0) + (mm == 0) + (n == 0)
                out.append(vp * k)
                out += [vs * k] * {2: 0, 1: 1, 0: 2}[zeros]
    return np.sort(out)[:count]


@pytest.mark.slow
def test_cube_eigenfrequencies_converge():
    """Sec. 5.1: lumped-mass eigenfrequencies approach the analytic 3D values with rate ~2/3 in N_dof."""
    from scipy.sparse.linalg import eigsh
    L, E, nu, rho = 8.0, 1000.0, 0.3, 1.0
    ref = _cube_reference(L, E, nu, rho, 100)
    errs, ndofs = [], []
    for level in (0, 1):
        m = configs.sliding_cube(level, L=L, E=E, rho=rho, nu=nu)
        o = Oracle(m)
        K = o.stiffness_sparse()
        free = np.flatnonzero(~m.fixed.astype(bool))
        s = 1 / np.sqrt(o.mdiag[free])
        from scipy import sparse
        S = sparse.diags(s)
        A = (S @ K[free][:, free] @ S).tocsc()
        w2 = eigsh(A, k=100, sigma=0, which="LM", return_eigenvectors=False)
        w = np.sqrt(np.sort(w2))
        errs.append(np.sqrt(((w - ref) ** 2).sum() / (ref ** 2).sum()))
        ndofs.append(m.n_dof)
    rate = np.log(errs[1] / errs[0]) / np.log(ndofs[1] / ndofs[0])
    assert errs[0] < 0.15 and errs[1] < 0.04
    assert -0.8 < rate < -0.55, (errs, rate)


def test_ricker_wavelet():
    gold = {l.split()[0]: float(l.split()[1]) for l in open(GOLD) if l.strip() and not l.startswith("#")}
    t1 = gold["t1"]
    assert np.isclose(loads.ricker(t1, t1), 1.0)
    assert abs(loads.ricker(t1 * 1.2, t1)) < 1e-15 and abs(loads.ricker(t1 * 0.8, t1)) < 1e-15
    # amplitude spectrum by FFT: peak at fm (eq. Ricker_fm), 95 % of the area below f1 ~ 2.2/t1
    dt = t1 / 2000
    t = np.arange(0, 40 * t1, dt)
    A = np.abs(np.fft.rfft(loads.ricker(t, t1))) * dt
    f = np.fft.rfftfreq(len(t), dt)
    assert abs(f[np.argmax(A)] - loads.ricker_fm(t1)) <= f[1]
    cum = np.cumsum(A)
    f1 = f[np.searchsorted(cum, 0.95 * cum[-1])]
    assert abs(f1 * t1 - gold["f1_t1"]) < 0.05
    assert abs(f1 - gold["f1"]) / gold["f1"] < 0.02
    vp = np.sqrt(gold["E"] * (1 - gold["nu"]) / (gold["rho"] * (1 + gold["nu"]) * (1 - 2 * gold["nu"])))
    assert np.isclose(vp, gold["vP"])


def test_sampled_step_matches_full_step():
    m = configs.cfg2(lcoarse=2, lfine=4, delta=0.1)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    u, um1 = configs.random_state(m.n_dof, seed=3, fixed=m.fixed)
    full, _ = o.step(u, um1, 17, dt)
    nodes = np.random.default_rng(2).choice(m.n_nodes, 25, replace=False)
    part = o.sampled_step(u, um1, 17, dt, nodes)
    assert np.abs(part - full.reshape(-1, 3)[nodes]).max() <= 1e-14 * np.abs(full).max()


def test_relative_error_metric():
    a = {1: np.array([1.0, -2.0]), 2: np.array([0.5, 4.0])}
    b = {1: np.array([1.0, -2.0 + 1e-3]), 2: np.array([0.5, 4.0])}
    assert np.isclose(relative_error(b, a), 1e-3 / 4.0)


def test_local_sampled_step_matches_full_step():
    """The cell-local one-step form (no global arrays) equals a full step at the sampled nodes,
    including nodes of hanging-node cells, load nodes and fixed nodes."""
    from oracle.solver import sampled_step_local
    m = configs.cfg2(lcoarse=2, lfine=4, delta=0.1)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    u, um1 = configs.random_state(m.n_dof, seed=4, fixed=m.fixed)
    full, _ = o.step(u, um1, 23, dt, alpha=0.3)
    rng = np.random.default_rng(5)
    hang = m.conn[m.conn_ptr[np.flatnonzero(m.cell_slots)[:10]]]
    fixed_nodes = np.flatnonzero(m.fixed.reshape(-1, 3).all(1))[:5]
    nodes = np.unique(np.concatenate([rng.choice(m.n_nodes, 30, replace=False), hang,
                                      m.load_dof[:5] // 3, fixed_nodes]))
    part = sampled_step_local(m, u, um1, 23, dt, nodes, alpha=0.3, cache=o.cache)
    assert np.abs(part - full.reshape(-1, 3)[nodes]).max() <= 1e-14 * np.abs(full).max()
    assert np.abs(part[np.isin(nodes, fixed_nodes)]).max() == 0.0


def _chain_k(ks, dt, n_steps, P):
    """1D lumped linear-element chain (A = rho = h = 1), element stiffnesses ks, fixed at node 0,
    force P(t) at the free end."""
    n_el = len(ks)
    k = np.zeros((n_el + 1, n_el + 1))
    for e, ke in enumerate(ks):
        k[e:e + 2, e:e + 2] += ke * np.array([[1, -1], [-1, 1.0]])
    mass = np.ones(n_el + 1)
    mass[-1] = 0.5
    minv = 1 / mass
    minv[0] = 0.0
    b = np.zeros(n_el + 1)
    b[-1] = 1.0
    u = np.zeros(n_el + 1)
    um1 = 0.5 * dt * dt * minv * P(0.0) * b
    hist = []
    for n in range(n_steps):
        unew = dt * dt * minv * (P(n * dt) * b - k @ u) + 2 * u - um1
        um1, u = u, unew
        hist.append(u.copy())
    return np.array(hist)


def _two_nu_bar(nx, nus):
    """nx x 1 x 1 unit cells, fixed at x = 0, every lateral dof held (uniaxial strain), material 1
    (Poisson ratio nus[1]) in x > nx/2, uniform end pressure; E = rho = 1."""
    from meshgen.octree import build_mesh

    def fixed(lat, lmax):
        out = np.ones(lat.shape, dtype=bool)
        out[:, 0] = lat[:, 0] == 0
        return out
    m = build_mesh((nx, 1, 1), 1.0, 0, 0, lambda l, i: np.zeros(len(i), bool),
                   material=lambda xyz: (xyz[:, 0] > nx / 2).astype(np.uint8), mat_E=(1.0, 1.0),
                   mat_rho=(1.0, 1.0), nu=nus[0], fixed=fixed, mat_nu=nus)
    configs.patch_load(m, (0, 1), (0.5, 0.5), 1.0, pressure=-1.0)
    return m


def test_two_poisson_ratios_reduce_to_chain():
    """Each material uses its own Poisson ratio (its own pattern library, Sec. 3.2.3): with every
    lateral dof held, the bar is exactly the 1D lumped chain whose element stiffness is the
    constrained modulus E (1 - nu) / ((1 + nu)(1 - 2 nu)) of the element's material."""
    nx, nus, t1 = 24, (0.2, 0.35), 12.0
    m = _two_nu_bar(nx, nus)
    m.load = dict(kind="ricker", t1=t1, P0=1.0, dt_factor=0.5, n_steps=0, alpha=0.0)
    o = Oracle(m)
    dt = 0.5 * o.critical_dt()
    n_steps = 300
    snaps = o.run(n_steps=n_steps, dt=dt, snap_every=1, energy=False)["snapshots"]
    mc = lambda nu: (1 - nu) / ((1 + nu) * (1 - 2 * nu))
    ks = [mc(nus[1] if e + 0.5 > nx / 2 else nus[0]) for e in range(nx)]
    chain = _chain_k(ks, dt, n_steps, lambda t: loads.ricker(t, t1))
    sec = m.node_lat[:, 0].astype(np.int64)
    scale = np.abs(chain).max()
    for n in range(1, n_steps + 1, 9):
        u = snaps[n].reshape(-1, 3)
        assert np.abs(u[:, 0] - chain[n - 1][sec]).max() < 1e-11 * scale
    # the same bar read with one Poisson ratio for both halves is a different chain
    one = _chain_k([mc(nus[0])] * nx, dt, n_steps, lambda t: loads.ricker(t, t1))
    assert np.abs(one - chain).max() > 1e-3 * scale
